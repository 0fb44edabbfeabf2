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
// For output entry (y+1, x+1) with (y, x) in tile (s, c) at origin (y0, x0):
//   ii = sum_{x'<x0, y'<y0} I           (corner: 2-D prefix of tile totals)
//      + sum_{x0<=x'<=x} colcarry[x']    (pixels above the strip)
//      + sum_{y0<=y'<=y} rowcarry[y']    (pixels left of the slab)
//      + sum_{y0<=y'<=y, x0<=x'<=x} I    (in-tile prefix)
// All sums are u32 and wrap modulo 2^32 consistently.  HBM traffic is about
// 2 bytes read and 4 written per pixel plus 0.5 byte of carries.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kTileRows = 16;
constexpr int kTileCols = 256;  // 64 lanes x 4 columns
constexpr int kWavesPerBlock = 4;

struct Quad {
    uint32_t v[4];
};

// Four pixels starting at column x of row y; columns >= W read as zero.
__device__ __forceinline__ Quad load_quad(const uint8_t* __restrict__ img, int64_t pitch, int32_t y,
                                          int32_t x, int32_t W, bool aligned)
{
    Quad q;
    const uint8_t* row = img + (int64_t)y * pitch;
    if (aligned && x + 3 < W) {
        uint32_t w = *reinterpret_cast<const uint32_t*>(row + x);
        q.v[0] = w & 0xffu;
        q.v[1] = (w >> 8) & 0xffu;
        q.v[2] = (w >> 16) & 0xffu;
        q.v[3] = w >> 24;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) q.v[k] = (x + k < W) ? row[x + k] : 0u;
    }
    return q;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, int lane)
{
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    return incl - v;
}

__global__ __launch_bounds__(256) void integral_tile_sums(const uint8_t* __restrict__ img, int64_t pitch,
                                                          int32_t W, int32_t H, int32_t strips,
                                                          int32_t slabs, int64_t col_pitch, bool aligned,
                                                          uint32_t* __restrict__ colsum,
                                                          uint32_t* __restrict__ rowsum)
{
    const int lane = threadIdx.x % kWave;
    const int tile = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= strips * slabs) return;
    const int s = tile / slabs, c = tile % slabs;
    const int y0 = s * kTileRows, x = c * kTileCols + 4 * lane;
    uint32_t col[4] = {0u, 0u, 0u, 0u};
    uint32_t tile_total = 0u;
    for (int r = 0; r < kTileRows; ++r) {
        const int y = y0 + r;
        if (y >= H) break;
        Quad q = load_quad(img, pitch, y, x, W, aligned);
        uint32_t part = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            col[k] += q.v[k];
            part += q.v[k];
        }
        uint32_t row_total = wave_sum(part);
        tile_total += row_total;
        if (lane == 0) rowsum[(int64_t)y * slabs + c] = row_total;
    }
    uint32_t* dst = colsum + (int64_t)s * col_pitch + x;
    *reinterpret_cast<uint4*>(dst) = make_uint4(col[0], col[1], col[2], col[3]);
    if (lane == 0) colsum[(int64_t)s * col_pitch + (int64_t)slabs * kTileCols + c] = tile_total;
}

// Blocks [0, col_blocks): exclusive scan down the strips for every column of
// the column table (pixel columns and the tile-total columns).  Remaining
// blocks: exclusive scan across the slabs for every image row.
__global__ __launch_bounds__(256) void integral_carry_scan(uint32_t* __restrict__ colsum,
                                                           uint32_t* __restrict__ rowsum, int32_t H,
                                                           int32_t strips, int32_t slabs,
                                                           int64_t col_pitch, int32_t col_blocks)
{
    if ((int)blockIdx.x < col_blocks) {
        const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (x >= col_pitch) return;
        uint32_t acc = 0u;
        for (int s = 0; s < strips; ++s) {
            uint32_t* p = colsum + (int64_t)s * col_pitch + x;
            uint32_t v = *p;
            *p = acc;
            acc += v;
        }
    } else {
        const int64_t y = (int64_t)(blockIdx.x - col_blocks) * blockDim.x + threadIdx.x;
        if (y >= H) return;
        uint32_t acc = 0u;
        for (int c = 0; c < slabs; ++c) {
            uint32_t* p = rowsum + y * slabs + c;
            uint32_t v = *p;
            *p = acc;
            acc += v;
        }
    }
}

__global__ __launch_bounds__(256) void integral_tile_write(const uint8_t* __restrict__ img, int64_t pitch,
                                                           int32_t W, int32_t H, int32_t strips,
                                                           int32_t slabs, int64_t col_pitch, bool aligned,
                                                           const uint32_t* __restrict__ colcarry,
                                                           const uint32_t* __restrict__ rowcarry,
                                                           uint32_t* __restrict__ ii, int64_t ii_pitch)
{
    const int lane = threadIdx.x % kWave;
    const int tile = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= strips * slabs) return;
    const int s = tile / slabs, c = tile % slabs;
    const int y0 = s * kTileRows, x0 = c * kTileCols, x = x0 + 4 * lane;

    // corner = sum over tiles above-left: the scanned tile totals of this strip, slabs < c
    const uint32_t* strip_row = colcarry + (int64_t)s * col_pitch;
    uint32_t corner_part = 0u;
    for (int cc = lane; cc < c; cc += kWave) corner_part += strip_row[(int64_t)slabs * kTileCols + cc];
    const uint32_t corner = wave_sum(corner_part);

    // pixels above the strip, summed over the slab's columns up to each column
    uint4 cv = *reinterpret_cast<const uint4*>(strip_row + x);
    uint32_t above[4];
    above[0] = cv.x;
    above[1] = above[0] + cv.y;
    above[2] = above[1] + cv.z;
    above[3] = above[2] + cv.w;
    const uint32_t above_off = corner + wave_exclusive_scan(above[3], lane);
#pragma unroll
    for (int k = 0; k < 4; ++k) above[k] += above_off;

    if (s == 0) {  // zero first row of the integral image
        for (int k = 0; k < 4; ++k)
            if (x + k < W) ii[x + k + 1] = 0u;
        if (c == 0 && lane == 0) ii[0] = 0u;
    }

    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    uint32_t left = 0u;
    for (int r = 0; r < kTileRows; ++r) {
        const int y = y0 + r;
        if (y >= H) break;
        left += rowcarry[(int64_t)y * slabs + c];
        Quad q = load_quad(img, pitch, y, x, W, aligned);
        uint32_t p[4];
        p[0] = q.v[0];
        p[1] = p[0] + q.v[1];
        p[2] = p[1] + q.v[2];
        p[3] = p[2] + q.v[3];
        const uint32_t off = wave_exclusive_scan(p[3], lane);
        uint32_t* out = ii + (int64_t)(y + 1) * ii_pitch;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[k] += p[k] + off;
            if (x + k < W) out[x + k + 1] = above[k] + left + acc[k];
        }
        if (c == 0 && lane == 0) out[0] = 0u;
    }
}

}  // namespace

size_t IntegralPlan::workspace_bytes() const
{
    return sizeof(uint32_t) * ((size_t)strips * (size_t)col_pitch + (size_t)H * (size_t)slabs);
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
    hipLaunchKernelGGL(integral_tile_sums, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W,
                       p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum);
    const int col_blocks = (int)((p.col_pitch + 255) / 256);
    const int row_blocks = (p.H + 255) / 256;
    hipLaunchKernelGGL(integral_carry_scan, dim3(col_blocks + row_blocks), dim3(256), 0, stream, colsum,
                       rowsum, p.H, p.strips, p.slabs, p.col_pitch, col_blocks);
    hipLaunchKernelGGL(integral_tile_write, dim3(tile_blocks), dim3(256), 0, stream, img, img_pitch, p.W,
                       p.H, p.strips, p.slabs, p.col_pitch, aligned, colsum, rowsum, ii, ii_pitch);
}

}  // namespace bd
