// Batched tangent vmult over 3-D problems of degrees 1 to 3 in one persistent
// launch: a grid of as many workgroups as the GPU holds at once walks the
// list of (problem, cell block, degree) items of every degree, each
// workgroup taking items of an XCD-local range (neighbouring cell blocks of a
// problem share an L2), and runs the block body of the item's degree.  The
// alternative to one launch per degree bin; the footprint (registers, LDS) is
// the largest of the three degrees, which is what the per-bin launches avoid.
#include "cellops.hpp"
#include "fused.hpp"

namespace mfh {

template <typename T>
constexpr int fused_lds() {
  constexpr int a = TangentLdsSize<3, 2, T>::value, b = TangentLdsSize<3, 3, T>::value,
                c = TangentLdsSize<3, 4, T>::value;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <typename T, int POL, bool O32>
__global__ void __launch_bounds__(kBlock) k_tangent_batch_fused(const CellArgs<T>* __restrict__ args,
                                                                const int4* __restrict__ items, int n_items,
                                                                const T* const* __restrict__ xs,
                                                                T* const* __restrict__ ys) {
  __shared__ T lds[fused_lds<T>()];
  using CArgs = const CellArgs<T> __attribute__((address_space(4)));
  using CInt = const int __attribute__((address_space(4)));
  using CPtrX = const T* const __attribute__((address_space(4)));
  using CPtrY = T* const __attribute__((address_space(4)));
  // XCD-local item ranges: workgroup w runs on XCD w % 8 and takes items of
  // that XCD's contiguous eighth of the list, striding by the XCD's workgroups
  const int g = gridDim.x, w = blockIdx.x;
  const int xcd = w & 7, nx = (g - xcd + 7) >> 3, lw = w >> 3;
  const long long lo = (long long)n_items * xcd / 8, hi = (long long)n_items * (xcd + 1) / 8;
  for (long long i = lo + lw; i < hi; i += nx) {
    const CInt* it = (CInt*)(items + i);
    const int p = it[0], blk = it[1], deg = it[2];
    const CellArgs<T>& a = *(const CellArgs<T>*)((CArgs*)args + p);
    const T* x = ((CPtrX*)xs)[p];
    T* y = ((CPtrY*)ys)[p];
    if (deg == 1)
      tangent_block<3, 1, T, POL, O32>(a, x, y, blk, lds);
    else if (deg == 2)
      tangent_block<3, 2, T, POL, O32>(a, x, y, blk, lds);
    else
      tangent_block<3, 3, T, POL, O32>(a, x, y, blk, lds);
    __syncthreads();   // the next item reuses the LDS
  }
}

template <typename T, int POL, bool O32>
void launch_fused(const CellArgs<T>* args, const int4* items, int n_items, const T* const* xs, T* const* ys,
                  hipStream_t s) {
  static int grid = 0;   // workgroups resident at once on the device
  if (grid == 0) {
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tangent_batch_fused<T, POL, O32>, kBlock, 0);
    grid = std::max(8, cus * std::max(1, per));
  }
  const int g = std::min(grid, std::max(8, n_items));
  hipLaunchKernelGGL((k_tangent_batch_fused<T, POL, O32>), dim3(g), dim3(kBlock), 0, s, args, items, n_items, xs,
                     ys);
}

template <typename T>
void tangent_batch_fused(int policy, bool off32, const CellArgs<T>* args, const int4* items, int n_items,
                         const T* const* xs, T* const* ys, hipStream_t s) {
  switch (policy * 2 + (off32 ? 1 : 0)) {
    case 0: launch_fused<T, 0, false>(args, items, n_items, xs, ys, s); break;
    case 1: launch_fused<T, 0, true>(args, items, n_items, xs, ys, s); break;
    case 2: launch_fused<T, 1, false>(args, items, n_items, xs, ys, s); break;
    case 3: launch_fused<T, 1, true>(args, items, n_items, xs, ys, s); break;
    case 4: launch_fused<T, 2, false>(args, items, n_items, xs, ys, s); break;
    case 5: launch_fused<T, 2, true>(args, items, n_items, xs, ys, s); break;
    case 6: launch_fused<T, 3, false>(args, items, n_items, xs, ys, s); break;
    default: launch_fused<T, 3, true>(args, items, n_items, xs, ys, s); break;
  }
}

template void tangent_batch_fused<double>(int, bool, const CellArgs<double>*, const int4*, int,
                                          const double* const*, double* const*, hipStream_t);
template void tangent_batch_fused<float>(int, bool, const CellArgs<float>*, const int4*, int, const float* const*,
                                         float* const*, hipStream_t);

}  // namespace mfh
