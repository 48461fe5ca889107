// Launch forms measured by the autotuner: the batched tangent vmult as one
// persistent launch over 3-D problems of degrees 1 to 3 (ops_batch_fused.hip),
// and the contraction stage in VALU and MFMA form (contract.hip).
#pragma once

#include "common.hpp"

namespace mfh {

// items: (problem index into args/xs/ys, cell block, degree, unused) per
// workgroup-sized piece of work; off32: every problem fits 32-bit lane offsets.
template <typename T>
void tangent_batch_fused(int policy, bool off32, const CellArgs<T>* args, const int4* items, int n_items,
                         const T* const* xs, T* const* ys, hipStream_t s);

// The sum factorisation's 1-D contraction stage in VALU (mfma = 0) or MFMA
// form, for the autotuner (contract.hip): blocks x 256 lines of degree + 1
// values, `sweeps` dependent applications of the Gauss-point table pair;
// out: blocks * (degree + 1) * 256 floats.
void contraction_stage(int degree, int mfma, int sweeps, int blocks, float* out, hipStream_t s);

}  // namespace mfh
