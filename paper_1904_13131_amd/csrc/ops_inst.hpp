// Instantiates the cell kernels of one (dim, degree) and its launch table.
// Included once per ops_d<dim>_p<degree>.hip so that the degrees compile in
// parallel.
#pragma once

#include "cellops.hpp"
#include "ops.hpp"

namespace mfh {

// Tile shapes (cells per axis) and components per sweep batch of the tile
// kernel, per dimension, degree and precision: two shapes each, the tuned
// table (or the descriptor's tile_shape) picks one per level.  A tile uses
// cells x (pencils per cell) threads, rounded up to whole wavefronts; shape 0
// keeps FP64 tiles within 256 threads (two resident blocks per CU, FP64
// kernels hold about 2x the registers of FP32 ones), shape 1 is the
// alternative: larger tiles (fewer tile faces, hence fewer atomics) where the
// LDS allows, smaller ones where shape 0 is already large.
template <int DIM, int P, typename T, int V>
struct TileCfg;
#define MFH_TILE(D, P, T, V, X, Y, Z, C) \
  template <> struct TileCfg<D, P, T, V> { static constexpr int TX = X, TY = Y, TZ = Z, NC = C; };
MFH_TILE(3, 1, double, 0, 4, 4, 4, 3)
MFH_TILE(3, 1, double, 1, 8, 4, 2, 3)
MFH_TILE(3, 1, float, 0, 4, 4, 4, 3)
MFH_TILE(3, 1, float, 1, 8, 8, 2, 3)
MFH_TILE(3, 2, double, 0, 3, 3, 3, 3)
MFH_TILE(3, 2, double, 1, 4, 4, 2, 3)
MFH_TILE(3, 2, float, 0, 4, 4, 2, 3)
MFH_TILE(3, 2, float, 1, 3, 3, 3, 3)
MFH_TILE(3, 3, double, 0, 2, 2, 4, 1)
MFH_TILE(3, 3, double, 1, 4, 2, 2, 1)
MFH_TILE(3, 3, float, 0, 2, 2, 4, 3)
MFH_TILE(3, 3, float, 1, 2, 2, 2, 3)
MFH_TILE(3, 4, double, 0, 2, 2, 2, 1)
MFH_TILE(3, 4, double, 1, 4, 2, 2, 1)
MFH_TILE(3, 4, float, 0, 2, 2, 2, 1)
MFH_TILE(3, 4, float, 1, 2, 2, 2, 3)
MFH_TILE(2, 1, double, 0, 16, 8, 1, 2)
MFH_TILE(2, 1, double, 1, 16, 16, 1, 2)
MFH_TILE(2, 1, float, 0, 16, 8, 1, 2)
MFH_TILE(2, 1, float, 1, 16, 16, 1, 2)
MFH_TILE(2, 2, double, 0, 16, 5, 1, 2)
MFH_TILE(2, 2, double, 1, 8, 8, 1, 2)
MFH_TILE(2, 2, float, 0, 16, 5, 1, 2)
MFH_TILE(2, 2, float, 1, 8, 8, 1, 2)
MFH_TILE(2, 3, double, 0, 8, 8, 1, 2)
MFH_TILE(2, 3, double, 1, 16, 4, 1, 2)
MFH_TILE(2, 3, float, 0, 8, 8, 1, 2)
MFH_TILE(2, 3, float, 1, 16, 4, 1, 2)
MFH_TILE(2, 4, double, 0, 8, 6, 1, 2)
MFH_TILE(2, 4, double, 1, 8, 4, 1, 2)
MFH_TILE(2, 4, float, 0, 8, 6, 1, 2)
MFH_TILE(2, 4, float, 1, 8, 4, 1, 2)
#undef MFH_TILE

template <int DIM, int P>
struct OpInst {
  template <typename T, int POL, int V>
  static void tangent_tile(const CellArgs<T>& a, unsigned grid, hipStream_t s) {
    using TC = TileCfg<DIM, P, T, V>;
    using TGeo = TileGeo<DIM, P, TC::TX, TC::TY, TC::TZ>;
    hipLaunchKernelGGL((k_tangent_tile<DIM, P, T, POL, TC::TX, TC::TY, TC::TZ, TC::NC>), dim3(grid),
                       dim3(TGeo::BLOCK), 0, s, a);
  }
  template <typename T, int V>
  static long long tiles(int N) {
    using TC = TileCfg<DIM, P, T, V>;
    const long long tx = (N + TC::TX - 1) / TC::TX, ty = (N + TC::TY - 1) / TC::TY;
    const long long tz = DIM == 3 ? (N + TC::TZ - 1) / TC::TZ : 1;
    return tx * ty * tz;
  }
  template <typename T, int V>
  static constexpr TileShape shape() {
    using TC = TileCfg<DIM, P, T, V>;
    return TileShape{TC::TX, TC::TY, DIM == 3 ? TC::TZ : 1};
  }
  // 32-bit lane offsets (see lane_load) when every per-lane offset of a level
  // with `cells` cells fits, including those into arrays of T pairs
  template <typename T>
  static bool off32(long long cells) {
    return (long long)Geo<DIM, P + 1>::NV * cells * 2 * (long long)sizeof(T) < (1LL << 32);
  }
  template <typename T, int POL, int V>
  static void tangent(const CellArgs<T>& a, unsigned grid, hipStream_t s) {
    using CB = CellBlock<DIM, P + 1, V>;
    if (off32<T>(a.ncells))
      hipLaunchKernelGGL((k_tangent<DIM, P, T, POL, true, CB::value>), dim3(grid), dim3(CB::threads), 0, s, a);
    else
      hipLaunchKernelGGL((k_tangent<DIM, P, T, POL, false, CB::value>), dim3(grid), dim3(CB::threads), 0, s, a);
  }
  template <typename T, int POL>
  static void tangent_batch(const CellArgs<T>* args, const int2* items, const T* const* xs, T* const* ys,
                            unsigned n_items, long long max_cells, hipStream_t s) {
    if (off32<T>(max_cells))
      hipLaunchKernelGGL((k_tangent_batch<DIM, P, T, POL, true>), dim3(n_items), dim3(kBlock), 0, s, args, items, xs,
                         ys);
    else
      hipLaunchKernelGGL((k_tangent_batch<DIM, P, T, POL, false>), dim3(n_items), dim3(kBlock), 0, s, args, items,
                         xs, ys);
  }
  template <typename T>
  static void elem_gather_batch(const CellArgs<T>* args, const GatherItem* items, const T* const* xs, T* const* ys,
                                unsigned n_items, hipStream_t s) {
    hipLaunchKernelGGL((k_elem_gather_batch<DIM, P, T>), dim3(n_items), dim3(kBlock), 0, s, args, items, xs, ys);
  }
  template <typename T, int V>
  static void elem_gather(const CellArgs<T>& a, hipStream_t s) {
    const unsigned plane = (unsigned)a.L * (unsigned)a.L;
    const unsigned magic = (unsigned)((((unsigned long long)1 << 32) + (unsigned)a.L - 1) / (unsigned)a.L);
    const dim3 grid((plane + kBlock - 1) / kBlock, DIM == 3 ? a.L : 1, 1);
    hipLaunchKernelGGL((k_elem_gather<DIM, P, T, CellBlock<DIM, P + 1, V>::value>), grid, dim3(kBlock), 0, s, a,
                       magic);
  }
  template <typename T, int V>
  static void elem_gather_cheb(const CellArgs<T>& a, const ChebOut<T>& out, hipStream_t s) {
    const unsigned plane = (unsigned)a.L * (unsigned)a.L;
    const unsigned magic = (unsigned)((((unsigned long long)1 << 32) + (unsigned)a.L - 1) / (unsigned)a.L);
    const dim3 grid((plane + kBlock - 1) / kBlock, DIM == 3 ? a.L : 1, 1);
    hipLaunchKernelGGL((k_elem_gather_cheb<DIM, P, T, CellBlock<DIM, P + 1, V>::value>), grid, dim3(kBlock), 0, s,
                       a, magic, out);
  }
  static void residual(const CellArgs<double>& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_residual<DIM, P>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  template <typename T, int POL>
  static void qpdata(const CellArgs<double>& a, T* cache, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_qpdata<DIM, P, T, POL>), dim3(grid), dim3(kBlock), 0, s, a, cache);
  }
  // the setup kernels take the material law from a.law (0: the closed forms
  // of the Neo-Hookean law, 1: the general route)
  template <int LAW>
  static void diag_law(const CellArgs<double>& a, hipStream_t s) {
    constexpr int cpb = DiagShape<DIM, P, LAW>::CPB;
    const unsigned grid = (unsigned)((a.ncells + cpb - 1) / cpb);
    hipLaunchKernelGGL((k_diag<DIM, P, LAW>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  static void diag(const CellArgs<double>& a, hipStream_t s) {
    if (a.law)
      diag_law<1>(a, s);
    else
      diag_law<0>(a, s);
  }
  template <typename Sink>
  static void cell_matrix(const CellArgs<double>& a, const Sink& sink, unsigned grid, hipStream_t s) {
    if (a.law)
      hipLaunchKernelGGL((k_cell_matrix<DIM, P, Sink, 1>), dim3(grid), dim3(kBlock), 0, s, a, sink);
    else
      hipLaunchKernelGGL((k_cell_matrix<DIM, P, Sink, 0>), dim3(grid), dim3(kBlock), 0, s, a, sink);
  }
  static void coarse_assemble(const CellArgs<double>& a, const int* fmap, long long nf, double* K,
                              unsigned grid, hipStream_t s) {
    cell_matrix(a, DenseSink{fmap, nf, K, {}}, grid, s);
  }
  static void csr_assemble(const CellArgs<double>& a, const long long* row_ptr, double* val, unsigned grid,
                           hipStream_t s) {
    cell_matrix(a, CsrSink{row_ptr, val, P, {}, {}, {}, 0}, grid, s);
  }
  static const OpFns* table() {
    static const OpFns t = {
        {{&tangent<double, POL_R, 0>, &tangent<double, POL_CF, 0>, &tangent<double, POL_C2, 0>,
          &tangent<double, POL_C4, 0>},
         {&tangent<double, POL_R, 1>, &tangent<double, POL_CF, 1>, &tangent<double, POL_C2, 1>,
          &tangent<double, POL_C4, 1>}},
        {{&tangent<float, POL_R, 0>, &tangent<float, POL_CF, 0>, &tangent<float, POL_C2, 0>,
          &tangent<float, POL_C4, 0>},
         {&tangent<float, POL_R, 1>, &tangent<float, POL_CF, 1>, &tangent<float, POL_C2, 1>,
          &tangent<float, POL_C4, 1>}},
        &residual,
        {&qpdata<double, POL_R>, &qpdata<double, POL_CF>, &qpdata<double, POL_C2>, &qpdata<double, POL_C4>},
        {&qpdata<float, POL_R>, &qpdata<float, POL_CF>, &qpdata<float, POL_C2>, &qpdata<float, POL_C4>},
        &diag,
        {{&tangent_tile<double, POL_R, 0>, &tangent_tile<double, POL_CF, 0>, &tangent_tile<double, POL_C2, 0>,
          &tangent_tile<double, POL_C4, 0>},
         {&tangent_tile<double, POL_R, 1>, &tangent_tile<double, POL_CF, 1>, &tangent_tile<double, POL_C2, 1>,
          &tangent_tile<double, POL_C4, 1>}},
        {{&tangent_tile<float, POL_R, 0>, &tangent_tile<float, POL_CF, 0>, &tangent_tile<float, POL_C2, 0>,
          &tangent_tile<float, POL_C4, 0>},
         {&tangent_tile<float, POL_R, 1>, &tangent_tile<float, POL_CF, 1>, &tangent_tile<float, POL_C2, 1>,
          &tangent_tile<float, POL_C4, 1>}},
        {{&tiles<double, 0>, &tiles<double, 1>}, {&tiles<float, 0>, &tiles<float, 1>}},
        {{shape<double, 0>(), shape<double, 1>()}, {shape<float, 0>(), shape<float, 1>()}},
        {&tangent_batch<double, POL_R>, &tangent_batch<double, POL_CF>, &tangent_batch<double, POL_C2>,
         &tangent_batch<double, POL_C4>},
        {&tangent_batch<float, POL_R>, &tangent_batch<float, POL_CF>, &tangent_batch<float, POL_C2>,
         &tangent_batch<float, POL_C4>},
        {&elem_gather<double, 0>, &elem_gather<double, 1>},
        {&elem_gather<float, 0>, &elem_gather<float, 1>},
        &elem_gather_batch<double>,
        &elem_gather_batch<float>,
        {&elem_gather_cheb<double, 0>, &elem_gather_cheb<double, 1>},
        {&elem_gather_cheb<float, 0>, &elem_gather_cheb<float, 1>},
        &coarse_assemble,
        &csr_assemble,
        {CellBlock<DIM, P + 1, 0>::value, CellBlock<DIM, P + 1, 1>::value},
        {CacheWords<DIM, POL_R>::value, CacheWords<DIM, POL_CF>::value, CacheWords<DIM, POL_C2>::value,
         CacheWords<DIM, POL_C4>::value},
    };
    return &t;
  }
};

}  // namespace mfh

#define MFH_DEFINE_OPS(D, P) \
  namespace mfh {            \
  const OpFns* op_fns_##D##_##P() { return OpInst<D, P>::table(); } \
  }
