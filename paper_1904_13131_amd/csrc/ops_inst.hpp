// Instantiates the cell kernels of one (dim, degree) and its launch table.
// Included once per ops_d<dim>_p<degree>.hip so that the degrees compile in
// parallel.
#pragma once

#include "cellops.hpp"
#include "ops.hpp"

namespace mfh {

template <int DIM, int P>
struct OpInst {
  template <typename T, int POL>
  static void tangent(const CellArgs<T>& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_tangent<DIM, P, T, POL>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  static void residual(const CellArgs<double>& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_residual<DIM, P>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  template <typename T, int POL>
  static void qpdata(const CellArgs<double>& a, T* cache, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_qpdata<DIM, P, T, POL>), dim3(grid), dim3(kBlock), 0, s, a, cache);
  }
  static void diag(const CellArgs<double>& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_diag<DIM, P>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  static void coarse_assemble(const CellArgs<double>& a, const int* fmap, long long nf, double* K,
                              unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_coarse_assemble<DIM, P>), dim3(grid), dim3(kBlock), 0, s, a, fmap, nf, K);
  }
  static const OpFns* table() {
    static const OpFns t = {
        {&tangent<double, POL_R>, &tangent<double, POL_CF>, &tangent<double, POL_C2>},
        {&tangent<float, POL_R>, &tangent<float, POL_CF>, &tangent<float, POL_C2>},
        &residual,
        {&qpdata<double, POL_R>, &qpdata<double, POL_CF>, &qpdata<double, POL_C2>},
        {&qpdata<float, POL_R>, &qpdata<float, POL_CF>, &qpdata<float, POL_C2>},
        &diag,
        &coarse_assemble,
        Geo<DIM, P + 1>::CPB,
        kBlock / (DIM == 3 ? (P + 1) * (P + 1) * (P + 1) : (P + 1) * (P + 1)),
        {CacheWords<DIM, POL_R>::value, CacheWords<DIM, POL_CF>::value, CacheWords<DIM, POL_C2>::value},
    };
    return &t;
  }
};

}  // namespace mfh

#define MFH_DEFINE_OPS(D, P) \
  namespace mfh {            \
  const OpFns* op_fns_##D##_##P() { return OpInst<D, P>::table(); } \
  }
