// Shared device/host definitions of the mfh library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfh {

constexpr int kMaxDeg = 4;            // polynomial degree 1..4
constexpr int kMaxN1 = kMaxDeg + 1;   // 1-D support / Gauss points
constexpr int kBlock = 256;           // threads per block of the cell kernels

// 1-D tables on the reference interval [0,1]:  S[q][a] = phi_a(xg_q),
// D[q][a] = phi_a'(xg_q) (GLL support points a, Gauss points q), w[q] Gauss
// weights.  Passed by value so that every entry becomes a scalar operand.
template <typename T>
struct Tables {
  T S[kMaxN1][kMaxN1];
  T D[kMaxN1][kMaxN1];
  T w[kMaxN1];
  T xg[kMaxN1];   // Gauss points on [0,1]
  // Even-odd halves of M = S, D, S^T, D^T (index 0..3; n = p + 1, h = n / 2):
  // eo[M][0][r][c] = (M[r][c] + M[r][n-1-c]) / 2, eo[M][1][r][c] =
  // (M[r][c] - M[r][n-1-c]) / 2 for c < h, r <= h; mid[M][r] = M[r][h].
  T eo[4][2][kMaxN1][kMaxN1 / 2];
  T mid[4][kMaxN1];
};

// Everything a cell kernel needs about one level, by value.
template <typename T>
struct CellArgs {
  Tables<T> tb;
  int N;                // cells per direction
  int L;                // lattice nodes per direction
  long long nn;         // nodes per component (L^dim)
  long long ncells;     // cells of the level
  long long nlaunch;    // cells covered by this launch (all, or one colour)
  int color;            // colour of this launch (coloured scatter), else -1
  unsigned fmask[3];    // per component: bit f set if face f = 2*axis+side fixes it
  T invh;               // 1 / h
  T wscale;             // h^(dim-1): quadrature weight * |cell| / h
  T mu[2], lam[2];      // material table
  T mu2[2];             // second-invariant moduli (general law; zero for Neo-Hookean)
  int law;              // 0: Neo-Hookean closed forms, 1: general (Mooney-Rivlin) route
  const uint32_t* matbits;   // per cell, nwords words: bit q = material id of qp q
  int nwords;
  const T* u;           // level displacement (recompute policy / residual / cache build)
  const T* cache;       // policy cache: word w of qp q of cell e at (w*nQ + q)*ncells + e
  const T* x;           // input vector
  T* y;                 // output vector
  double* blockmin;     // per-block min J (cache build)
  T* elem;              // element buffer (ELEMENT scatter): value of node n, component c of
                        // cell e at (c * (p+1)^dim + n) * ncells + e; null: scatter into y
  int mask_in;          // 1: constrained entries of x read as zero (K_c); 0: read as given
};

// The kernel's first argument read in place from the kernarg segment (offset
// 0, constant address space): uniform reads become scalar loads and the
// compiler does not copy the argument block to private memory, which it does
// for large blocks whose fields are used many times (degree >= 3).
template <typename A>
__device__ __forceinline__ const A& kernel_args(const A& byval) {
  (void)byval;
  using CA = const A __attribute__((address_space(4)));
  return *(const A*)(CA*)__builtin_amdgcn_kernarg_segment_ptr();
}

// Work item of the batched node-sum kernel (ELEMENT scatter).
struct GatherItem {
  int p;            // problem index in the bin's argument table
  int k;            // plane k of the lattice (0 in 2-D)
  int blk;          // block of kBlock nodes in the (i, j) plane
  unsigned magic;   // ceil(2^32 / L) of the problem's lattice
};

// Destinations of the node sums: the output vector, or one Chebyshev
// smoothing step applied to the sum t = (K_c x)_i right away,
//   d_i <- cd d_i + cr dinv_i (f_i - t_i),  x_i <- x_i + d_i,
// so that the smoother does not write and re-read the product vector.  The
// update of x_i is safe: x_i is read only by this thread (constrained rows)
// and the cell kernel that read x has completed.
template <typename T>
struct StoreOut {
  T* y;
  __device__ void operator()(long long gi, T v) const { y[gi] = v; }
};
template <typename T>
struct ChebOut {
  const T* f;
  const T* dinv;
  T* d;
  T* x;
  T cd, cr;
  __device__ void operator()(long long gi, T t) const {
    const T r = f[gi] - t;
    const T di = (cd != T(0) ? cd * d[gi] : T(0)) + cr * dinv[gi] * r;
    d[gi] = di;
    x[gi] = x[gi] + di;
  }
};

// Lattice description for the vector kernels.
struct Lattice {
  int L, dim;
  long long nn;         // nodes per component
  unsigned fmask[3];    // per component face bits, as in CellArgs
};

__device__ __forceinline__ bool constrained_dof(const Lattice& lt, long long dof) {
  const int c = (int)(dof / lt.nn);
  long long n = dof - c * lt.nn;
  const int i = (int)(n % lt.L);
  n /= lt.L;
  const int j = (int)(n % lt.L);
  const int k = (int)(n / lt.L);
  unsigned f = 0;
  f |= (i == 0) ? 1u : 0u;
  f |= (i == lt.L - 1) ? 2u : 0u;
  f |= (j == 0) ? 4u : 0u;
  f |= (j == lt.L - 1) ? 8u : 0u;
  if (lt.dim == 3) {
    f |= (k == 0) ? 16u : 0u;
    f |= (k == lt.L - 1) ? 32u : 0u;
  }
  return (f & lt.fmask[c]) != 0;
}

// Workgroups are dealt round-robin to the 8 XCDs; remap so that every XCD
// receives one contiguous range of logical blocks (neighbouring cells share
// nodes, so this keeps the shared lines in one L2).
__device__ __forceinline__ long long xcd_block(long long b, long long nb) {
  const long long q = nb >> 3, r = nb & 7;
  const long long x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Faces a lattice node lies on: bit (2*axis + side).
__device__ __forceinline__ unsigned node_faces(int i, int j, int k, int L, int dim) {
  unsigned f = 0;
  f |= (i == 0) ? 1u : 0u;
  f |= (i == L - 1) ? 2u : 0u;
  f |= (j == 0) ? 4u : 0u;
  f |= (j == L - 1) ? 8u : 0u;
  if (dim == 3) {
    f |= (k == 0) ? 16u : 0u;
    f |= (k == L - 1) ? 32u : 0u;
  }
  return f;
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  // Compiled with -munsafe-fp-atomics: a single hardware global atomic add.
  atomicAdd(p, v);
}

}  // namespace mfh
