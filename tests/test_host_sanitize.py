"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU code.

* The oracle (oracle/bdref.c) with every function called on small inputs
  and edge cases (tests/sanitize_oracle.c), gcc -fsanitize=address,undefined.
* The library's host-side argument validation (tests/sanitize_abi.c): every
  source under csrc/ compiled by hipcc with the sanitizers on the host pass
  only (-Xarch_host; the gfx950 code is built as usual), linked into a
  driver that calls every entry point with malformed arguments.

Both drivers exit 0 only when no sanitizer reported anything and (for the
ABI) every return code is the documented one."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
          "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
          "-o", exe, os.path.join(HERE, "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "bdref.c"), "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=120)
    assert "no reports" in r.stdout


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_validation_under_asan_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops"]
    sources = sorted(glob.glob(os.path.join(ROOT, "paper_2108_08380_amd", "csrc", "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *flags, *san, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(sources))) as ex:
        objs = list(ex.map(compile_one, sources))
    drv = str(tmp_path / "sanitize_abi.o")
    _run([HIPCC, "-x", "c", "-O1", "-g", *san, "-c", os.path.join(HERE, "sanitize_abi.c"), "-o", drv])
    exe = str(tmp_path / "sanitize_abi")
    _run([HIPCC, "--offload-arch=gfx950", *san, drv, *objs, "-o", exe])
    r = _run([exe], env=dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0"), timeout=120)
    assert "every code as documented" in r.stdout
