// Launch table of the cell kernels, one entry per (dim, degree).
#pragma once

#include "common.hpp"

namespace mfh {

struct TileShape {
  int tx, ty, tz;
};

struct OpFns {
  // tangent vmult per cell-block variant and policy (0 R, 1 CF, 2 C2, 3 C4); grid = ceil(cells / cpb[variant])
  void (*tangent_d[2][4])(const CellArgs<double>&, unsigned grid, hipStream_t);
  void (*tangent_f[2][4])(const CellArgs<float>&, unsigned grid, hipStream_t);
  void (*residual)(const CellArgs<double>&, unsigned grid, hipStream_t);
  // quadrature data (min J and the policy cache in double / float)
  void (*qpdata_d[4])(const CellArgs<double>&, double* cache, unsigned grid, hipStream_t);
  void (*qpdata_f[4])(const CellArgs<double>&, float* cache, unsigned grid, hipStream_t);
  void (*diag)(const CellArgs<double>&, hipStream_t);   // adds into a.y
  // tile variant of the tangent vmult per tile shape [shape][policy]; grid = tiles[dtype][shape](N)
  void (*tangent_tile_d[2][4])(const CellArgs<double>&, unsigned grid, hipStream_t);
  void (*tangent_tile_f[2][4])(const CellArgs<float>&, unsigned grid, hipStream_t);
  long long (*tiles[2][2])(int N);   // [0] double, [1] float
  TileShape tile_shape[2][2];        // cells per axis of each shape, [dtype][shape]
  // batched vmult over problems of this (dim, degree): one workgroup per (problem, cell block) item
  // (max_cells: the largest cell count of the bin's problems)
  void (*tangent_batch_d[4])(const CellArgs<double>* args, const int2* items, const double* const* xs,
                             double* const* ys, unsigned n_items, long long max_cells, hipStream_t);
  void (*tangent_batch_f[4])(const CellArgs<float>* args, const int2* items, const float* const* xs,
                             float* const* ys, unsigned n_items, long long max_cells, hipStream_t);
  // second pass of the ELEMENT scatter, per cell-block variant of the cell kernel that wrote the buffer
  void (*elem_gather_d[2])(const CellArgs<double>&, hipStream_t);
  void (*elem_gather_f[2])(const CellArgs<float>&, hipStream_t);
  void (*elem_gather_batch_d)(const CellArgs<double>* args, const GatherItem* items, const double* const* xs,
                              double* const* ys, unsigned n_items, hipStream_t);
  void (*elem_gather_batch_f)(const CellArgs<float>* args, const GatherItem* items, const float* const* xs,
                              float* const* ys, unsigned n_items, hipStream_t);
  // node sums fused with one Chebyshev step (ELEMENT levels of the smoother)
  void (*elem_gather_cheb_d[2])(const CellArgs<double>&, const ChebOut<double>&, hipStream_t);
  void (*elem_gather_cheb_f[2])(const CellArgs<float>&, const ChebOut<float>&, hipStream_t);
  void (*coarse_assemble)(const CellArgs<double>&, const int* fmap, long long nf, double* K,
                          unsigned grid, hipStream_t);
  // element tangents added into the CSR values of K_c (pattern of the lattice)
  void (*csr_assemble)(const CellArgs<double>&, const long long* row_ptr, double* val, unsigned grid,
                       hipStream_t);
  int cpb[2];     // cells per block of the tangent vmult's variants ([0]: the other pencil kernels' length too)
  int cache_words[4];
};

const OpFns* op_fns(int dim, int degree);

#define MFH_DECLARE_OPS(D, P) const OpFns* op_fns_##D##_##P();
MFH_DECLARE_OPS(2, 1)
MFH_DECLARE_OPS(2, 2)
MFH_DECLARE_OPS(2, 3)
MFH_DECLARE_OPS(2, 4)
MFH_DECLARE_OPS(3, 1)
MFH_DECLARE_OPS(3, 2)
MFH_DECLARE_OPS(3, 3)
MFH_DECLARE_OPS(3, 4)
#undef MFH_DECLARE_OPS

}  // namespace mfh
