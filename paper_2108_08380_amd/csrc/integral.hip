// Integral image of a u8 image (Sec. III-A: box averages in constant time).
//
// Reduce-then-scan over 16-row x 256-column tiles, one wavefront per tile
// (each lane owns four adjacent columns):
//   1. tile_sums   per tile: row totals (one per row), column totals (one per
//                  column) and the tile total, appended to the column table;
//   2. carry_scan  exclusive scans: column totals down the strips (also the
//                  tile totals, which gives the corner term) and row totals
//                  across the slabs;
//   3. tile_write  re-reads the u8 tile, forms the in-tile 2-D prefix with
//                  an in-lane prefix plus a wavefront scan per row and adds
//                  the three carries.
// Single images of up to kMaxRawGroups groups of four strips (2048 rows)
// skip pass 2: pass 1 (group_sums) also writes the totals of each group of
// strips, and the write pass sums its carries from the unscanned tables
// (at most groups + 3 column-table rows, the row totals of the slabs to the
// left), one dependent launch fewer.  The batch keeps the three passes.
// For output entry (y+1, x+1) with (y, x) in tile (s, c) at origin (y0, x0):
//   ii = sum_{x'<x0, y'<y0} I           (corner: 2-D prefix of tile totals)
//      + sum_{x0<=x'<=x} colcarry[x']    (pixels above the strip)
//      + sum_{y0<=y'<=y} rowcarry[y']    (pixels left of the slab)
//      + sum_{y0<=y'<=y, x0<=x'<=x} I    (in-tile prefix)
// All sums are u32 and wrap modulo 2^32 consistently.  HBM traffic is about
// 2 bytes read and 4 written per pixel plus 0.5 byte of carries.
#include "order_body.hpp"

namespace bd {
namespace {

constexpr int kTileRows = 16;
constexpr int kTileCols = 256;  // 64 lanes x 4 columns
constexpr int kWavesPerBlock = 4;

// Four pixels of row `y` starting at column x, packed little-endian into one
// u32 (a byte per pixel); columns >= W read as zero.  Only for tiles that
// cross the right image edge (per-lane bounds checks).
__device__ __forceinline__ uint32_t load_quad(const uint8_t* __restrict__ img, int64_t pitch, int32_t y,
                                              int32_t x, int32_t W, bool aligned)
{
    const uint8_t* row = img + (int64_t)y * pitch;
    if (aligned && x + 3 < W) return *reinterpret_cast<const uint32_t*>(row + x);
    uint32_t w = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (x + k < W) w |= (uint32_t)row[x + k] << (8 * k);
    return w;
}

// The 16 row quads of a tile at rows y0.. and column x of this lane.  A
// tile wholly inside the image (a wave-uniform test) issues all 16 loads
// back to back, with no branch between them; edge tiles check rows and
// columns.  Unaligned rows: the aligned dwords holding the first and the
// last of the four bytes (the same dword when the row happens to be
// aligned) shifted into place with v_alignbyte; each holds a byte of the
// row, so neither reaches memory the image does not own.
__device__ __forceinline__ void load_tile(const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t y0,
                                          int32_t rows, int32_t x0, int32_t x, bool aligned, uint32_t (&q)[16])
{
    if (rows == 16 && x0 + 256 <= W) {
        const uint8_t* p = img + (int64_t)y0 * pitch + x;
        if (aligned) {
#pragma unroll
            for (int r = 0; r < 16; ++r) q[r] = *reinterpret_cast<const uint32_t*>(p + r * pitch);
        } else {
            uint32_t lo[16], hi[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uintptr_t a = reinterpret_cast<uintptr_t>(p + r * pitch);
                lo[r] = *reinterpret_cast<const uint32_t*>(a & ~(uintptr_t)3);
                hi[r] = *reinterpret_cast<const uint32_t*>((a + 3) & ~(uintptr_t)3);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                q[r] = __builtin_amdgcn_alignbyte(hi[r], lo[r], (uint32_t)(reinterpret_cast<uintptr_t>(p + r * pitch) & 3u));
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) q[r] = r < rows ? load_quad(img, pitch, y0 + r, x, W, aligned) : 0u;
    }
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xffu; }

__device__ __forceinline__ uint32_t quad_sum(uint32_t w)
{
    return byte_of(w, 0) + byte_of(w, 1) + byte_of(w, 2) + byte_of(w, 3);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive prefix sum over the 64 lanes: inclusive scans inside each row of
// 16 lanes with DPP row shifts, then the totals of the earlier rows (read
// from lanes 15, 31, 47) are added.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, int lane)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane(x, 15);
    const uint32_t r1 = r0 + (uint32_t)__builtin_amdgcn_readlane(x, 31);
    const uint32_t r2 = r1 + (uint32_t)__builtin_amdgcn_readlane(x, 47);
    const int row = lane >> 4;
    const uint32_t before = row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r1 : r2;
    return (uint32_t)x + before - v;
}

// Sums of rs[r] over the 64 lanes for r = 0..15 with a halving butterfly
// (17 shuffles); lane l ends with the total of row l >> 2.
__device__ __forceinline__ uint32_t wave_sum16(const uint32_t (&rs)[16], int lane)
{
    uint32_t a[8];
    {
        const bool hi = lane & 32;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t keep = hi ? rs[8 + r] : rs[r];
            const uint32_t send = hi ? rs[r] : rs[8 + r];
            a[r] = keep + __shfl_xor(send, 32, kWave);
        }
    }
    uint32_t b[4];
    {
        const bool hi = lane & 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t keep = hi ? a[4 + r] : a[r];
            const uint32_t send = hi ? a[r] : a[4 + r];
            b[r] = keep + __shfl_xor(send, 16, kWave);
        }
    }
    uint32_t c[2];
    {
        const bool hi = lane & 8;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t keep = hi ? b[2 + r] : b[r];
            const uint32_t send = hi ? b[r] : b[2 + r];
            c[r] = keep + __shfl_xor(send, 8, kWave);
        }
    }
    const bool hi = lane & 4;
    uint32_t d = (hi ? c[1] : c[0]) + __shfl_xor(hi ? c[0] : c[1], 4, kWave);
    d += __shfl_xor(d, 2, kWave);
    d += __shfl_xor(d, 1, kWave);
    return d;
}

// ---- bodies shared by the single-image and the batched kernels

// One wavefront: the sums of tile `tile` (its column totals and tile total
// are also left in col / tile_total).
__device__ __forceinline__ void tile_sums_body(const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t H,
                                               int32_t slabs, int64_t col_pitch, bool aligned,
                                               uint32_t* __restrict__ colsum, uint32_t* __restrict__ rowsum,
                                               int tile, int lane, uint32_t (&col)[4], uint32_t& tile_total)
{
    const int s = tile / slabs, c = tile % slabs;
    const int y0 = s * kTileRows, x = c * kTileCols + 4 * lane;
    const int rows = min(kTileRows, H - y0);
    uint32_t q[kTileRows];
    load_tile(img, pitch, W, y0, rows, c * kTileCols, x, aligned, q);
    col[0] = col[1] = col[2] = col[3] = 0u;
    uint32_t rs[kTileRows];
#pragma unroll
    for (int r = 0; r < kTileRows; ++r) {
#pragma unroll
        for (int k = 0; k < 4; ++k) col[k] += byte_of(q[r], k);
        rs[r] = quad_sum(q[r]);
    }
    const uint32_t row_total = wave_sum16(rs, lane);  // row lane >> 2 of the tile
    tile_total = wave_sum((lane & 3) == 0 ? row_total : 0u);
    if ((lane & 3) == 0 && (lane >> 2) < rows) rowsum[(int64_t)(y0 + (lane >> 2)) * slabs + c] = row_total;
    uint32_t* dst = colsum + (int64_t)s * col_pitch + x;
    *reinterpret_cast<uint4*>(dst) = make_uint4(col[0], col[1], col[2], col[3]);
    if (lane == 0) colsum[(int64_t)s * col_pitch + (int64_t)slabs * kTileCols + c] = tile_total;
}

__device__ __forceinline__ void tile_sums_body(const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t H,
                                               int32_t slabs, int64_t col_pitch, bool aligned,
                                               uint32_t* __restrict__ colsum, uint32_t* __restrict__ rowsum,
                                               int tile, int lane)
{
    uint32_t col[4], total;
    tile_sums_body(img, pitch, W, H, slabs, col_pitch, aligned, colsum, rowsum, tile, lane, col, total);
}

// One thread: exclusive scan down the strips of column x of the column table.
// The scan is a chain of load round trips, so 32 strips are loaded per
// round, unconditionally for whole rounds.
__device__ __forceinline__ void carry_col_body(uint32_t* __restrict__ colsum, int32_t strips, int64_t col_pitch,
                                               int64_t x)
{
    constexpr int kBatch = 32;
    uint32_t acc = 0u;
    uint32_t* col = colsum + x;
    int s0 = 0;
    for (; s0 + kBatch <= strips; s0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = col[(int64_t)(s0 + k) * col_pitch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            col[(int64_t)(s0 + k) * col_pitch] = acc;
            acc += v[k];
        }
    }
    if (s0 < strips) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = s0 + k < strips ? col[(int64_t)(s0 + k) * col_pitch] : 0u;
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (s0 + k < strips) col[(int64_t)(s0 + k) * col_pitch] = acc;
            acc += v[k];
        }
    }
}

// One thread: exclusive scan across the slabs of image row y.
__device__ __forceinline__ void carry_row_body(uint32_t* __restrict__ rowsum, int32_t slabs, int64_t y)
{
    constexpr int kBatch = 8;
    uint32_t acc = 0u;
    for (int c0 = 0; c0 < slabs; c0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = c0 + k < slabs ? rowsum[y * slabs + c0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (c0 + k < slabs) rowsum[y * slabs + c0 + k] = acc;
            acc += v[k];
        }
    }
}

// Carries of a tile from the exclusive scans of the carry pass: the row
// totals of the slabs to the left, the column totals of the strips above
// and, summed over the slabs to the left, the tile totals above.
struct ScannedCarries {
    const uint32_t* __restrict__ colcarry;
    const uint32_t* __restrict__ rowcarry;

    __device__ __forceinline__ void load(int s, int c, int slabs, int64_t col_pitch, int y0, int rows, int x,
                                         int lane, uint32_t (&rc)[kTileRows], uint4& cv,
                                         uint32_t& corner_part) const
    {
        if (rows == kTileRows) {
#pragma unroll
            for (int r = 0; r < kTileRows; ++r) rc[r] = rowcarry[(int64_t)(y0 + r) * slabs + c];
        } else {
#pragma unroll
            for (int r = 0; r < kTileRows; ++r) rc[r] = r < rows ? rowcarry[(int64_t)(y0 + r) * slabs + c] : 0u;
        }
        const uint32_t* strip_row = colcarry + (int64_t)s * col_pitch;
        cv = *reinterpret_cast<const uint4*>(strip_row + x);
        corner_part = 0u;
        for (int cc = lane; cc < c; cc += kWave) corner_part += strip_row[(int64_t)slabs * kTileCols + cc];
    }
};

// Carries of a tile summed directly from the unscanned tables: the column
// totals of each strip (colsum), of each group of kGroupStrips strips
// (group) and the row totals of each slab (rowsum).  The strips above a tile
// are the whole groups above its own plus the strips of its group above it.
constexpr int kGroupStrips = 4;

struct RawCarries {
    const uint32_t* __restrict__ colsum;
    const uint32_t* __restrict__ rowsum;
    const uint32_t* __restrict__ group;

    __device__ __forceinline__ void load(int s, int c, int slabs, int64_t col_pitch, int y0, int rows, int x,
                                         int lane, uint32_t (&rc)[kTileRows], uint4& cv,
                                         uint32_t& corner_part) const
    {
        const int kg = s / kGroupStrips, s_first = kg * kGroupStrips;
        const int n_col = kg + (s - s_first);  // column-total rows to add
        // pixels above the strip in this lane's four columns, 16 rows of a table in flight at a time
        uint32_t a0 = 0u, a1 = 0u, a2 = 0u, a3 = 0u;
        for (int k0 = 0; k0 < n_col; k0 += 16) {
            uint4 v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int k = k0 + j;
                const uint32_t* row = k < kg ? group + (int64_t)k * col_pitch
                                             : colsum + (int64_t)(s_first + (k - kg)) * col_pitch;
                v[j] = k < n_col ? *reinterpret_cast<const uint4*>(row + x) : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                a0 += v[j].x;
                a1 += v[j].y;
                a2 += v[j].z;
                a3 += v[j].w;
            }
        }
        cv = make_uint4(a0, a1, a2, a3);
        // tiles above-left: entry (k, cc), k < n_col, cc < c, of the tile-total columns
        corner_part = 0u;
        for (int e = lane; e < n_col * c; e += kWave) {
            const int k = e / c, cc = e - k * c;
            const uint32_t* row = k < kg ? group + (int64_t)k * col_pitch
                                         : colsum + (int64_t)(s_first + (k - kg)) * col_pitch;
            corner_part += row[(int64_t)slabs * kTileCols + cc];
        }
        // row r of the tile: lanes r, r + 16, r + 32, r + 48 add the slabs to the left
        const int r = lane & 15;
        uint32_t part = 0u;
        if (r < rows)
            for (int cc = lane >> 4; cc < c; cc += 4) part += rowsum[(int64_t)(y0 + r) * slabs + cc];
        part += (uint32_t)__shfl_xor((int)part, 16, kWave);
        part += (uint32_t)__shfl_xor((int)part, 32, kWave);
#pragma unroll
        for (int rr = 0; rr < kTileRows; ++rr) rc[rr] = (uint32_t)__builtin_amdgcn_readlane((int)part, rr);
    }
};

// One wavefront: the integral-image entries of tile `tile`, with the
// carries of `cr` (ScannedCarries or RawCarries).
template <class Carries>
__device__ __forceinline__ void tile_write_body(const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t H,
                                                int32_t slabs, int64_t col_pitch, bool aligned, const Carries& cr,
                                                uint32_t* __restrict__ ii, int64_t ii_pitch, int tile, int lane)
{
    const int s = tile / slabs, c = tile % slabs;
    const int y0 = s * kTileRows, x0 = c * kTileCols, x = x0 + 4 * lane;
    const int rows = min(kTileRows, H - y0);

    // every load of the tile is issued before any arithmetic
    uint32_t q[kTileRows], rc[kTileRows];
    load_tile(img, pitch, W, y0, rows, x0, x, aligned, q);
    uint4 cv;
    uint32_t corner_part;
    cr.load(s, c, slabs, col_pitch, y0, rows, x, lane, rc, cv, corner_part);

    // corner (tiles above-left) plus the pixels above the strip, summed along the slab
    const uint32_t corner = wave_sum(corner_part);
    uint32_t above[4];
    above[0] = cv.x;
    above[1] = above[0] + cv.y;
    above[2] = above[1] + cv.z;
    above[3] = above[2] + cv.w;
    const uint32_t above_off = corner + wave_exclusive_scan(above[3], lane);
#pragma unroll
    for (int k = 0; k < 4; ++k) above[k] += above_off;

    // Stores.  With 16-byte aligned output rows, a tile wholly inside the
    // image writes output columns x0 .. x0 + 255 as one aligned 16-byte
    // store per lane: lane l takes the last value of lane l - 1 (a DPP
    // wavefront shift), lane 0 the boundary column x0 = corner + left, and
    // the rightmost tile also writes column W.  Otherwise each lane writes
    // its columns x + 1 .. x + 4 one by one; next to an aligned tile it also
    // writes the boundary column x0 the tile on its left leaves out.
    const bool rows_aligned = ((reinterpret_cast<uintptr_t>(ii) | (uintptr_t)ii_pitch * 4u) & 15u) == 0;
    const bool wide = rows_aligned && x0 + kTileCols <= W;
    const bool last_col = x0 + kTileCols == W && lane == kWave - 1;
    const bool boundary = rows_aligned && !wide && c > 0 && lane == 0;

    if (s == 0) {  // zero first row of the integral image
        if (wide) {
            *reinterpret_cast<uint4*>(ii + x0 + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
            if (last_col) ii[W] = 0u;
        } else {
            for (int k = 0; k < 4; ++k)
                if (x + k < W) ii[x + k + 1] = 0u;
            if (c == 0 && lane == 0) ii[0] = 0u;
            if (boundary) ii[x0] = 0u;
        }
    }

    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    uint32_t left = 0u;
#pragma unroll
    for (int r = 0; r < kTileRows; ++r) {
        if (r >= rows) break;
        left += rc[r];
        uint32_t p[4];
        p[0] = byte_of(q[r], 0);
        p[1] = p[0] + byte_of(q[r], 1);
        p[2] = p[1] + byte_of(q[r], 2);
        p[3] = p[2] + byte_of(q[r], 3);
        const uint32_t off = wave_exclusive_scan(p[3], lane);
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[k] += p[k] + off;
            v[k] = above[k] + left + acc[k];
        }
        uint32_t* out = ii + (int64_t)(y0 + r + 1) * ii_pitch;
        if (wide) {
            // wave_shr:1; lane 0 keeps `old`, the boundary column
            const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp((int)(corner + left), (int)v[3], 0x138, 0xf,
                                                                        0xf, false);
            *reinterpret_cast<uint4*>(out + x0 + 4 * lane) = make_uint4(prev, v[0], v[1], v[2]);
            if (last_col) out[W] = v[3];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (x + k < W) out[x + k + 1] = v[k];
            if (c == 0 && lane == 0) out[0] = 0u;
            if (boundary) out[x0] = corner + left;
        }
    }
}

// ---- single-image kernels

__global__ __launch_bounds__(256) void integral_tile_sums(const uint8_t* __restrict__ img, int64_t pitch,
                                                          int32_t W, int32_t H, int32_t strips,
                                                          int32_t slabs, int64_t col_pitch, bool aligned,
                                                          uint32_t* __restrict__ colsum,
                                                          uint32_t* __restrict__ rowsum)
{
    const int tile = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= strips * slabs) return;
    tile_sums_body(img, pitch, W, H, slabs, col_pitch, aligned, colsum, rowsum, tile, threadIdx.x % kWave);
}

// Blocks [0, col_blocks): column scans; remaining blocks: row scans.
__global__ __launch_bounds__(256) void integral_carry_scan(uint32_t* __restrict__ colsum,
                                                           uint32_t* __restrict__ rowsum, int32_t H,
                                                           int32_t strips, int32_t slabs,
                                                           int64_t col_pitch, int32_t col_blocks)
{
    if ((int)blockIdx.x < col_blocks) {
        const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (x < col_pitch) carry_col_body(colsum, strips, col_pitch, x);
    } else {
        const int64_t y = (int64_t)(blockIdx.x - col_blocks) * blockDim.x + threadIdx.x;
        if (y < H) carry_row_body(rowsum, slabs, y);
    }
}

__global__ __launch_bounds__(256) void integral_tile_write(const uint8_t* __restrict__ img, int64_t pitch,
                                                           int32_t W, int32_t H, int32_t strips,
                                                           int32_t slabs, int64_t col_pitch, bool aligned,
                                                           const uint32_t* __restrict__ colcarry,
                                                           const uint32_t* __restrict__ rowcarry,
                                                           uint32_t* __restrict__ ii, int64_t ii_pitch)
{
    const int tile = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= strips * slabs) return;
    tile_write_body(img, pitch, W, H, slabs, col_pitch, aligned, ScannedCarries{colcarry, rowcarry}, ii, ii_pitch, tile,
                    threadIdx.x % kWave);
}

// ---- single-image kernels without the carry pass (images of up to
// kMaxRawGroups groups of strips): the first pass also writes the column and
// tile totals of each group of kGroupStrips strips, and the write pass sums
// its carries from the unscanned tables.

constexpr int kMaxRawGroups = 32;

// Block g of the group pass takes slab g / groups and group g % groups; its
// wavefront w < kGroupStrips sums strip kGroupStrips * group + w as
// tile_sums_body, and the block adds the column and tile totals of its
// strips into the group table.
__device__ __forceinline__ void group_sums_body(const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t H,
                                                int32_t strips, int32_t slabs, int64_t col_pitch, bool aligned,
                                                uint32_t* __restrict__ colsum, uint32_t* __restrict__ rowsum,
                                                uint32_t* __restrict__ group, int g, uint4 (*part)[kWave],
                                                uint32_t* tot)
{
    const int groups = (strips + kGroupStrips - 1) / kGroupStrips;
    const int c = g / groups, k = g % groups;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (wave < kGroupStrips) {
        const int s = k * kGroupStrips + wave;
        uint32_t col[4] = {0u, 0u, 0u, 0u}, total = 0u;
        if (s < strips)
            tile_sums_body(img, pitch, W, H, slabs, col_pitch, aligned, colsum, rowsum, s * slabs + c, lane, col,
                           total);
        part[wave][lane] = make_uint4(col[0], col[1], col[2], col[3]);
        if (lane == 0) tot[wave] = total;
    }
    __syncthreads();
    if (wave == 0) {
        uint4 a = part[0][lane];
#pragma unroll
        for (int w = 1; w < kGroupStrips; ++w) {
            const uint4 b = part[w][lane];
            a.x += b.x;
            a.y += b.y;
            a.z += b.z;
            a.w += b.w;
        }
        uint32_t* row = group + (int64_t)k * col_pitch;
        *reinterpret_cast<uint4*>(row + c * kTileCols + 4 * lane) = a;
        if (lane == 0) {
            uint32_t t = 0u;
#pragma unroll
            for (int w = 0; w < kGroupStrips; ++w) t += tot[w];
            row[(int64_t)slabs * kTileCols + c] = t;
        }
    }
}

__global__ __launch_bounds__(256) void integral_group_sums(const uint8_t* __restrict__ img, int64_t pitch, int32_t W,
                                                           int32_t H, int32_t strips, int32_t slabs,
                                                           int64_t col_pitch, bool aligned,
                                                           uint32_t* __restrict__ colsum,
                                                           uint32_t* __restrict__ rowsum,
                                                           uint32_t* __restrict__ group)
{
    __shared__ uint4 part[kGroupStrips][kWave];
    __shared__ uint32_t tot[kGroupStrips];
    group_sums_body(img, pitch, W, H, strips, slabs, col_pitch, aligned, colsum, rowsum, group, blockIdx.x, part, tot);
}

// Rows b, b + n_blocks, ... of the row-pair copy of a float image (the
// HashSIFT source of bd_prepare_view): element (y, x) = (I[y][x],
// I[min(y + 1, H - 1)][x]).
__device__ __forceinline__ void pack_rows_body(const float* __restrict__ hs, int64_t hs_pitch, int32_t W, int32_t H,
                                               float2* __restrict__ pairs, int64_t pairs_pitch, int b, int n_blocks)
{
    for (int y = b; y < H; y += n_blocks) {
        const float* r0 = hs + (int64_t)y * hs_pitch;
        const float* r1 = hs + (int64_t)(y + 1 < H ? y + 1 : H - 1) * hs_pitch;
        float2* out = pairs + (int64_t)y * pairs_pitch;
        for (int x = threadIdx.x; x < W; x += blockDim.x) out[x] = make_float2(r0[x], r1[x]);
    }
}

// The group pass with the rest of a view's preparation alongside
// (bd_build_integral_order, bd_prepare_view): block 0 sorts the keypoints,
// blocks 1 .. n_group are the group pass (its first kGroupStrips
// wavefronts), the n_pack blocks after them write the row-pair copy of the
// HashSIFT image (none without one).  The jobs share no data; in one launch
// they run beside each other instead of one after another.
__global__ __launch_bounds__(order_impl::kOrderThreads) void integral_group_sums_order(
    const uint8_t* __restrict__ img, int64_t pitch, int32_t W, int32_t H, int32_t strips, int32_t slabs,
    int64_t col_pitch, bool aligned, uint32_t* __restrict__ colsum, uint32_t* __restrict__ rowsum,
    uint32_t* __restrict__ group, const bd_keypoint* __restrict__ kps, int32_t n_kp, float inv_cell,
    int32_t* __restrict__ order, int32_t n_group, const float* __restrict__ hs, int64_t hs_pitch,
    float2* __restrict__ pairs, int64_t pairs_pitch, int32_t n_pack)
{
    __shared__ uint32_t bins[order_impl::kOrderBins];
    __shared__ uint32_t opart[order_impl::kOrderThreads];
    __shared__ uint4 part[kGroupStrips][kWave];
    __shared__ uint32_t tot[kGroupStrips];
    const int b = (int)blockIdx.x;
    if (b == 0) {
        order_impl::order_body(kps, n_kp, inv_cell, order, bins, opart);
    } else if (b <= n_group) {
        group_sums_body(img, pitch, W, H, strips, slabs, col_pitch, aligned, colsum, rowsum, group, b - 1, part,
                        tot);
    } else {
        pack_rows_body(hs, hs_pitch, W, H, pairs, pairs_pitch, b - 1 - n_group, n_pack);
    }
}

__global__ __launch_bounds__(1024) void pack_rowpairs_kernel(const float* __restrict__ hs, int64_t hs_pitch,
                                                             int32_t W, int32_t H, float2* __restrict__ pairs,
                                                             int64_t pairs_pitch)
{
    pack_rows_body(hs, hs_pitch, W, H, pairs, pairs_pitch, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void integral_tile_write_raw(const uint8_t* __restrict__ img, int64_t pitch,
                                                               int32_t W, int32_t H, int32_t strips, int32_t slabs,
                                                               int64_t col_pitch, bool aligned,
                                                               const uint32_t* __restrict__ colsum,
                                                               const uint32_t* __restrict__ rowsum,
                                                               const uint32_t* __restrict__ group,
                                                               uint32_t* __restrict__ ii, int64_t ii_pitch)
{
    const int tile = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= strips * slabs) return;
    tile_write_body(img, pitch, W, H, slabs, col_pitch, aligned, RawCarries{colsum, rowsum, group}, ii, ii_pitch,
                    tile, threadIdx.x % kWave);
}

// ---- persistent batch kernels: units are blocks of four tiles (tile passes)
// or 256-column / 256-row blocks (carry scans) of every image in turn

__global__ __launch_bounds__(256) void integral_tile_sums_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                                const int32_t* __restrict__ pre)
{
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        const int tile = (u - pre[i]) * kWavesPerBlock + threadIdx.x / kWave;
        if (tile < im.strips * im.slabs)
            tile_sums_body(im.img_u8, im.pitch_u8, im.W, im.H, im.slabs, im.col_pitch, im.aligned != 0, im.colsum,
                           im.rowsum, tile, threadIdx.x % kWave);
    }
}

__global__ __launch_bounds__(256) void integral_carry_scan_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                                 const int32_t* __restrict__ pre)
{
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        const int lb = u - pre[i];
        const int col_blocks = (int)((im.col_pitch + 255) / 256);
        if (lb < col_blocks) {
            const int64_t x = (int64_t)lb * 256 + threadIdx.x;
            if (x < im.col_pitch) carry_col_body(im.colsum, im.strips, im.col_pitch, x);
        } else {
            const int64_t y = (int64_t)(lb - col_blocks) * 256 + threadIdx.x;
            if (y < im.H) carry_row_body(im.rowsum, im.slabs, y);
        }
    }
}

__global__ __launch_bounds__(256) void integral_tile_write_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                                 const int32_t* __restrict__ pre)
{
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        const int tile = (u - pre[i]) * kWavesPerBlock + threadIdx.x / kWave;
        if (tile < im.strips * im.slabs)
            tile_write_body(im.img_u8, im.pitch_u8, im.W, im.H, im.slabs, im.col_pitch, im.aligned != 0,
                            ScannedCarries{im.colsum, im.rowsum}, im.ii, im.ii_pitch, tile, threadIdx.x % kWave);
    }
}

}  // namespace

namespace {

int raw_groups(const IntegralPlan& p) { return (p.strips + kGroupStrips - 1) / kGroupStrips; }

// Elements before the group table in the workspace (16-byte aligned).
size_t group_offset(const IntegralPlan& p)
{
    return ((size_t)p.strips * (size_t)p.col_pitch + (size_t)p.H * (size_t)p.slabs + 3) / 4 * 4;
}

}  // namespace

size_t IntegralPlan::workspace_bytes() const
{
    const size_t groups = (size_t)raw_groups(*this);
    return sizeof(uint32_t) * (group_offset(*this) + (groups <= (size_t)kMaxRawGroups ? groups * (size_t)col_pitch : 0));
}

IntegralPlan plan_integral(int32_t W, int32_t H)
{
    IntegralPlan p;
    p.W = W;
    p.H = H;
    p.strips = (H + kTileRows - 1) / kTileRows;
    p.slabs = (W + kTileCols - 1) / kTileCols;
    // pixel columns (padded to whole slabs), one tile-total column per slab,
    // rounded up to a multiple of 4 so every strip row stays 16-byte aligned
    p.col_pitch = (((int64_t)p.slabs * kTileCols + p.slabs) + 3) / 4 * 4;
    return p;
}


void launch_integral(const IntegralPlan& p, const uint8_t* img, int64_t img_pitch, uint32_t* ii,
                     int64_t ii_pitch, void* workspace, hipStream_t stream)
{
    uint32_t* colsum = static_cast<uint32_t*>(workspace);
    uint32_t* rowsum = colsum + (size_t)p.strips * (size_t)p.col_pitch;
    const bool aligned = (img_pitch % 4 == 0) && (reinterpret_cast<uintptr_t>(img) % 4 == 0);
    const int tiles = p.strips * p.slabs;
    const int tile_blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (raw_groups(p) <= kMaxRawGroups) {
        uint32_t* group = colsum + group_offset(p);
        hipLaunchKernelGGL(integral_group_sums, dim3(p.slabs * raw_groups(p)), dim3(256), 0, stream, img, img_pitch,
                           p.W, p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum, group);
        hipLaunchKernelGGL(integral_tile_write_raw, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W,
                           p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum, group, ii, ii_pitch);
        return;
    }
    hipLaunchKernelGGL(integral_tile_sums, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W,
                       p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum);
    const int col_blocks = (int)((p.col_pitch + 255) / 256);
    const int row_blocks = (p.H + 255) / 256;
    hipLaunchKernelGGL(integral_carry_scan, dim3(col_blocks + row_blocks), dim3(256), 0, stream, colsum,
                       rowsum, p.H, p.strips, p.slabs, p.col_pitch, col_blocks);
    hipLaunchKernelGGL(integral_tile_write, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W,
                       p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum, ii, ii_pitch);
}

void launch_prepare_view(const IntegralPlan& p, const uint8_t* img, int64_t img_pitch, uint32_t* ii,
                         int64_t ii_pitch, void* workspace, const bd_keypoint* kps, int32_t n_kp, int32_t* order,
                         const float* hs, int64_t hs_pitch, float* pairs, int64_t pairs_pitch, hipStream_t stream)
{
    const int n_pack = hs ? (p.H < 256 ? p.H : 256) : 0;  // pitches below are in elements
    if (raw_groups(p) > kMaxRawGroups) {  // tall images: one launch per job, then the three passes
        if (n_kp > 0) launch_keypoint_order(kps, n_kp, p.W, p.H, order, stream);
        if (hs)
            hipLaunchKernelGGL(pack_rowpairs_kernel, dim3(n_pack), dim3(1024), 0, stream, hs, hs_pitch, p.W, p.H,
                               reinterpret_cast<float2*>(pairs), pairs_pitch);
        launch_integral(p, img, img_pitch, ii, ii_pitch, workspace, stream);
        return;
    }
    uint32_t* colsum = static_cast<uint32_t*>(workspace);
    uint32_t* rowsum = colsum + (size_t)p.strips * (size_t)p.col_pitch;
    uint32_t* group = colsum + group_offset(p);
    const bool aligned = (img_pitch % 4 == 0) && (reinterpret_cast<uintptr_t>(img) % 4 == 0);
    const int tile_blocks = (p.strips * p.slabs + kWavesPerBlock - 1) / kWavesPerBlock;
    const int n_group = p.slabs * raw_groups(p);
    hipLaunchKernelGGL(integral_group_sums_order, dim3(1 + n_group + n_pack), dim3(order_impl::kOrderThreads), 0,
                       stream, img, img_pitch, p.W, p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum,
                       group, kps, n_kp, order_inv_cell(p.W, p.H), order, n_group, hs, hs_pitch,
                       reinterpret_cast<float2*>(pairs), pairs_pitch, n_pack);
    hipLaunchKernelGGL(integral_tile_write_raw, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W, p.H,
                       p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum, group, ii, ii_pitch);
}

int integral_tile_blocks(const IntegralPlan& p) { return (p.strips * p.slabs + kWavesPerBlock - 1) / kWavesPerBlock; }
int integral_carry_blocks(const IntegralPlan& p) { return (int)((p.col_pitch + 255) / 256) + (p.H + 255) / 256; }

void launch_integral_batch(const BatchImage* imgs, int32_t n_img, const int32_t* tile_pre, const int32_t* carry_pre,
                           int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(integral_tile_sums_batch, dim3(grid), dim3(256), 0, stream, imgs, n_img, tile_pre);
    hipLaunchKernelGGL(integral_carry_scan_batch, dim3(grid), dim3(256), 0, stream, imgs, n_img, carry_pre);
    hipLaunchKernelGGL(integral_tile_write_batch, dim3(grid), dim3(256), 0, stream, imgs, n_img, tile_pre);
}

}  // namespace bd
