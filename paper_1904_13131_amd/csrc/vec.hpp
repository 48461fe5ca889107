// Vector, transfer and coarse-solve kernels (launch wrappers).
#pragma once

#include "common.hpp"

namespace mfh {

constexpr int kRedBlocks = 1024;   // partial sums per reduction

// Device scalar slots used by the CG iterations (double each).
enum Scalar {
  SC_RZ = 0,      // r.z
  SC_RZNEW,       // new r.z
  SC_PAP,         // p.Ap
  SC_ALPHA,       // rz / pAp
  SC_BETA,        // rznew / rz
  SC_RR,          // r.r
  SC_BB,          // b.b
  SC_TMP,
  SC_MINJ,
  SC_COUNT = 16
};

// 1-D banded operator applied along one axis of a lattice vector.
template <typename T>
struct Band {
  int nout, nin, K;
  const int* start;   // [nout], start + K <= nin
  const T* vals;      // [nout][K]
};

template <typename T>
struct SweepArgs {
  Band<T> band;
  int axis;
  int n[3];                    // input lattice extents (x fastest); 2-D: n[2] = 1
  int comps;
  long long in_cs, out_cs;     // component strides of input / output
  int add;                     // 1: out += result
  int mask;                    // 1: zero constrained output entries (final sweep)
  Lattice lt;                  // lattice of the output (when mask)
};

template <typename T> void fill_dirichlet(T* y, const T* x, long long n, const Lattice& lt, hipStream_t s);

// Batched fill: item k covers entries [chunk*c, chunk*(c+1)) of problem k's
// vectors; off[k] is the first chunk of problem k (off[n] = total chunks).
template <typename T>
struct FillItem {
  T* y;
  const T* x;
  Lattice lt;
  long long n;
};
constexpr long long kFillChunk = 4096;
template <typename T> void fill_dirichlet_batch(const FillItem<T>* items, const long long* off, int n, long long chunks,
                                                hipStream_t s);
template <typename T> void zero_constrained(T* v, long long n, const Lattice& lt, hipStream_t s);
template <typename T> void fill(T* v, T val, long long n, hipStream_t s);
template <typename TI, typename TO> void cast(const TI* in, TO* out, long long n, hipStream_t s);
template <typename TA, typename TB> void dot(const TA* a, const TB* b, long long n, double* part, double* out, hipStream_t s);
void min_reduce(const double* part, int np, double* out, hipStream_t s);
void set_scalar(double* p, double v, hipStream_t s);
// scalar ops: dst = num / den; optionally hist[idx] = dst, and rz <- rznew
void scalar_div(double* sc, int dst, int num, int den, int copy_to, int copy_from, double* hist, int hidx, hipStream_t s);

// x += alpha p; r -= alpha Ap; part = partial sums of r.r (alpha = sc[SC_ALPHA])
template <typename T> void cg_update(T* x, T* r, const T* p, const T* Ap, long long n, const double* sc,
                                     double* part, hipStream_t s);
// r -= alpha Ap; z = dinv r; part = partial r.z   (x not needed: eigenvalue estimate)
template <typename T> void lanczos_update(T* r, T* z, const T* Ap, const T* dinv, long long n, const double* sc,
                                          double* part, hipStream_t s);
// p = z + beta p (beta = sc[SC_BETA])
template <typename T> void cg_pupdate(T* p, const T* z, long long n, const double* sc, hipStream_t s);
// y = a * x + b * y
template <typename T> void axpby(T* y, const T* x, T a, T b, long long n, hipStream_t s);
// z = a*x + b*y + c*w (any may be null with coefficient 0)
template <typename T> void lincomb3(T* z, T a, const T* x, T b, const T* y, T c, const T* w, long long n, hipStream_t s);
// Chebyshev step: r = f - t (t == null: r = f); d = cd * d + cr * dinv * r; x += d (xzero: x = d)
template <typename T> void cheb_step(const T* f, const T* t, const T* dinv, T* d, T* x, T cd, T cr, int xzero,
                                     long long n, hipStream_t s);
// v[i] = value on constrained DoFs (others untouched)
template <typename T> void set_constrained(T* v, T val, long long n, const Lattice& lt, hipStream_t s);
// v[i] = 2 * (top 53 bits of SplitMix64 output i) / 2^53 - 1: the i-th output of
// the generator seeded with `seed` is the published SplitMix64 finaliser applied
// to seed + (i + 1) * 0x9E3779B97F4A7C15.
template <typename T> void splitmix_uniform(T* v, long long n, unsigned long long seed, hipStream_t s);
// out = 1 / in
template <typename TO> void reciprocal(const double* in, TO* out, long long n, hipStream_t s);
template <typename T> void sweep(const T* in, T* out, const SweepArgs<T>& a, hipStream_t s);

// Dirichlet values: u[dof] = scale * fv[face*dim + comp] on constrained DoFs (later
// face wins); fv is a host array of 2*dim*dim values passed to the kernel by value.
void set_dirichlet(double* u, const Lattice& lt, const double* fv, double scale, long long n, hipStream_t s);
// dg = constrained ? scale * fv - u : 0
// f = nodal forces of dead face tractions ft[2*axis + side][comp] (host
// array), g = 1-D lattice integrals of the basis functions (device, L values).
void traction_force(double* f, const Lattice& lt, const double* ft, const double* g, long long n, hipStream_t s);
// CSR form of K_c: pattern (columns, identity rows, zero values) and y = A x.
void csr_pattern(const long long* row_ptr, int* col, double* val, const Lattice& lt, int P, long long n,
                 hipStream_t s);
// group: lanes per row, 8 (eight entries per lane in flight) or 16 (four)
void csr_spmv(const long long* row_ptr, const int* col, const double* val, const double* x, double* y, long long n,
              int group, hipStream_t s);
void dirichlet_delta(const double* u, double* dg, const Lattice& lt, const double* fv, double scale,
                     long long n, hipStream_t s);

// Material bits of every cell: bit q of word (e*nwords + q/32) = material id of qp q.
void material_bits(uint32_t* bits, long long ncells, int N, int dim, int n1, const Tables<double>& tb, double h,
                   const double* incl, int nincl, int nwords, hipStream_t s);

// Coarse direct solve (dense FP64 inverse of a symmetric nonsingular matrix).
// Work arrays: Pinv 64 x 64, C and R n x 64, sw 1 + 4 * 64 ints, flag 3 ints
// (zeroed by the caller), scale 1.
struct DenseInvWork {
  double *Pinv, *C, *R, *scale;
  int *sw, *flag;
};
// X <- A^-1 for the symmetric n x n matrix A (row-major).  First block
// Gauss-Jordan in plain diagonal order on a copy in X, kept (decided on the
// device, without a host round trip) when every pivot is positive and above
// tol * max |A_ii|, i.e. A is positive definite; A and perm are then left
// unchanged.  Otherwise (flag[2] = 1) the pivoted pass inverts A in place in a
// permuted basis, A <- (Q A Q^T)^-1 with perm <- Q perm (perm[i] = original
// index of position i; the caller initialises it), and X receives that
// inverse in the original order (natural) or as it is, in the permuted basis
// (!natural, perm then maps its positions).  flag[0] = numerically singular,
// flag[1] = negative eigenvalues (Sylvester: the signs of the pivots).
void dense_inverse(double* A, double* X, long long n, int* perm, const DenseInvWork& w, double tol, bool natural,
                   hipStream_t s);
void iota(int* v, long long n, hipStream_t s);
// Most free coarse DoFs the pivoted inverse handles (LDS bitmap of the pivot choice).
constexpr int kGJMaxFree = 20480;
// Block steps of dense_inverse.  gate: NULL, or a device flag that lets the
// launches run only when it is nonzero.  gj_choose_block chooses a block
// step's pivots (Bunch-Kaufman on the current Schur complement) and exchanges
// them into [k0, k0 + nb); perm (free index -> DoF) follows.  V: 64 n doubles
// of scratch; sw: 1 + 4 * 64 ints (exchange pairs and the pivot list that
// gj_pivot follows).
void gj_choose_block(double* A, long long n, long long k0, int nb, double* V, int* sw, int* perm, const int* gate,
                     hipStream_t s);
void gj_pivot(double* A, long long n, long long k0, int nb, double* Pinv, int* flag, const double* scale, double tol,
              const int* sw, const int* gate, hipStream_t s);
void diag_absmax(const double* A, long long n, double* scale, const int* gate, hipStream_t s);
void gj_panels(const double* A, long long n, long long k0, int nb, const double* Pinv, double* Cb, double* R,
               const int* gate, hipStream_t s);
void gj_update(double* A, long long n, long long k0, int nb, const double* Cb, const double* R, const int* gate,
               hipStream_t s);
void gj_finish(double* A, long long n, long long k0, int nb, const double* Cb, const double* R, const double* Pinv,
               const int* gate, hipStream_t s);
void gj_blocks(double* A, long long n, int* perm, const DenseInvWork& w, double tol, bool pivoted, const int* gate,
               hipStream_t s);
// z[dof_of[f]] = sum_g Kinv[f][g] r[dof_of[g]]  (z pre-zeroed)
template <typename T> void coarse_apply(const double* Kinv, long long nf, const int* dof_of, const T* r, double* rf,
                                        double* zf, T* z, hipStream_t s);

}  // namespace mfh
