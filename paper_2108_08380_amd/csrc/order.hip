// Spatial processing order of keypoints.
//
// Describing keypoints in a spatially coherent order lets every XCD's L2
// hold the part of the image its workgroups touch: with the XCD-aware block
// mapping of the describe kernels, XCD x processes the x-th eighth of the
// ordered list, i.e. one compact region of the image.  The order is a
// counting sort of keypoints by the Morton index of their cell in a 64 x 64
// grid laid over the image.  It only changes which workgroup describes a
// keypoint, never the code written for it.
#include "order_body.hpp"

namespace bd {
namespace {

using order_impl::kOrderBins;
using order_impl::kOrderThreads;
using order_impl::order_body;

__global__ __launch_bounds__(kOrderThreads) void keypoint_order_kernel(const bd_keypoint* __restrict__ kps,
                                                                      int32_t n, float inv_cell,
                                                                      int32_t* __restrict__ order)
{
    __shared__ uint32_t bins[kOrderBins];
    __shared__ uint32_t part[kOrderThreads];
    order_body(kps, n, inv_cell, order, bins, part);
}

// Batch: one image per unit; order entries are indices local to the image.
__global__ __launch_bounds__(kOrderThreads) void keypoint_order_batch(const BatchImage* __restrict__ imgs,
                                                                     int32_t n_img,
                                                                     const bd_keypoint* __restrict__ kps,
                                                                     int32_t* __restrict__ order)
{
    __shared__ uint32_t bins[kOrderBins];
    __shared__ uint32_t part[kOrderThreads];
    const UnitRange ur = xcd_units(n_img);
    for (int i = ur.first; i < ur.end; i += ur.stride) {
        const BatchImage& im = imgs[i];
        order_body(kps + im.kp_offset, im.n_kp, im.inv_cell, order + im.kp_offset, bins, part);
    }
}

}  // namespace

float order_inv_cell(int32_t W, int32_t H)
{
    const int side = W > H ? W : H;
    return 1.0f / (float)((side + 63) / 64 > 0 ? (side + 63) / 64 : 1);
}

void launch_keypoint_order(const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H, int32_t* order,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(keypoint_order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, kps, n_kp,
                       order_inv_cell(W, H), order);
}

void launch_keypoint_order_batch(const BatchImage* imgs, int32_t n_img, const bd_keypoint* kps, int32_t* order,
                                 int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(keypoint_order_batch, dim3(grid), dim3(kOrderThreads), 0, stream, imgs, n_img, kps, order);
}

}  // namespace bd
