// Vector, transfer and coarse-solve kernels.
#include "vec.hpp"

#include <stdexcept>

namespace mfh {

namespace {

constexpr int kVB = 256;

inline unsigned grid_for(long long n, long long cap = 16384) {
  long long g = (n + kVB - 1) / kVB;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

inline unsigned red_grid(long long n) { return grid_for(n, kRedBlocks); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kVB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename T>
__global__ void k_fill_dirichlet(T* __restrict__ y, const T* __restrict__ x, long long n, Lattice lt) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    y[i] = (x != nullptr && constrained_dof(lt, i)) ? x[i] : T(0);
}

template <typename T>
__global__ void k_fill_dirichlet_batch(const FillItem<T>* __restrict__ items, const long long* __restrict__ off, int n) {
  const long long total = off[n];
  for (long long c = blockIdx.x; c < total; c += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= c)
        lo = mid;
      else
        hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const FillItem<T> it = items[lo];
    const long long b0 = (c - off[lo]) * kFillChunk;
    const long long b1 = b0 + kFillChunk < it.n ? b0 + kFillChunk : it.n;
    for (long long i = b0 + threadIdx.x; i < b1; i += kVB)
      it.y[i] = constrained_dof(it.lt, i) ? it.x[i] : T(0);
  }
}

template <typename T>
__global__ void k_zero_constrained(T* __restrict__ v, long long n, Lattice lt) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    if (constrained_dof(lt, i)) v[i] = T(0);
}

template <typename T>
__global__ void k_fill(T* __restrict__ v, T val, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) v[i] = val;
}

template <typename TI, typename TO>
__global__ void k_cast(const TI* __restrict__ in, TO* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    out[i] = (TO)in[i];
}

template <typename TA, typename TB>
__global__ void k_dot_part(const TA* __restrict__ a, const TB* __restrict__ b, long long n, double* part) {
  __shared__ double sh[kVB];
  double acc = 0;
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    acc += (double)a[i] * (double)b[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_final(const double* __restrict__ part, int np, double* out) {
  __shared__ double sh[kVB];
  double acc = 0;
  for (int i = threadIdx.x; i < np; i += kVB) acc += part[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_min_final(const double* __restrict__ part, int np, double* out) {
  __shared__ double sh[kVB];
  double m = 1e300;
  for (int i = threadIdx.x; i < np; i += kVB) m = part[i] < m ? part[i] : m;
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kVB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x + s] < sh[threadIdx.x] ? sh[threadIdx.x + s] : sh[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_set_scalar(double* p, double v) { *p = v; }

__global__ void k_scalar_div(double* sc, int dst, int num, int den, int copy_to, int copy_from, double* hist,
                             int hidx) {
  const double v = sc[num] / sc[den];
  sc[dst] = v;
  if (hist) hist[hidx] = v;
  if (copy_to >= 0) sc[copy_to] = sc[copy_from];
}

template <typename T>
__global__ void k_cg_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ Ap,
                            long long n, const double* __restrict__ sc, double* part) {
  __shared__ double sh[kVB];
  const T alpha = (T)sc[SC_ALPHA];
  double acc = 0;
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    acc += (double)ri * (double)ri;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ void k_lanczos_update(T* __restrict__ r, T* __restrict__ z, const T* __restrict__ Ap,
                                 const T* __restrict__ dinv, long long n, const double* __restrict__ sc,
                                 double* part) {
  __shared__ double sh[kVB];
  const T alpha = (T)sc[SC_ALPHA];
  double acc = 0;
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    const T ri = r[i] - alpha * Ap[i];
    const T zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    acc += (double)ri * (double)zi;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ void k_cg_pupdate(T* __restrict__ p, const T* __restrict__ z, long long n, const double* __restrict__ sc) {
  const T beta = (T)sc[SC_BETA];
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    p[i] = z[i] + beta * p[i];
}

template <typename T>
__global__ void k_axpby(T* __restrict__ y, const T* __restrict__ x, T a, T b, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    y[i] = a * x[i] + b * y[i];
}

template <typename T>
__global__ void k_lincomb3(T* __restrict__ z, T a, const T* __restrict__ x, T b, const T* __restrict__ y, T c,
                           const T* __restrict__ w, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    T v = 0;
    if (x) v += a * x[i];
    if (y) v += b * y[i];
    if (w) v += c * w[i];
    z[i] = v;
  }
}

template <typename T>
__global__ void k_cheb(const T* __restrict__ f, const T* __restrict__ t, const T* __restrict__ dinv, T* __restrict__ d,
                       T* __restrict__ x, T cd, T cr, int xzero, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    const T r = t ? f[i] - t[i] : f[i];
    const T di = (cd != T(0) ? cd * d[i] : T(0)) + cr * dinv[i] * r;
    d[i] = di;
    x[i] = xzero ? di : x[i] + di;
  }
}

template <typename T>
__global__ void k_set_constrained(T* __restrict__ v, T val, long long n, Lattice lt) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    if (constrained_dof(lt, i)) v[i] = val;
}

template <typename T>
__global__ void k_splitmix(T* __restrict__ v, long long n, unsigned long long seed) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    unsigned long long z = seed + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    v[i] = (T)((double)(z >> 11) * 0x1p-52 - 1.0);
  }
}

template <typename TO>
__global__ void k_reciprocal(const double* __restrict__ in, TO* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB)
    out[i] = (TO)(1.0 / in[i]);
}

// One output entry per thread: blockIdx.y = (component, index along axis 2)
// of the output, the x threads run over its axis-0 x axis-1 plane, so the
// only per-thread division is by the plane's row length (32-bit; the launch
// checks that plane and component sizes fit).  KB > 0: the band width as a
// compile-time constant (loads of the band unrolled and in flight together);
// KB = 0: any width.
template <typename T, int KB>
__global__ void k_sweep(const T* __restrict__ in, T* __restrict__ out, SweepArgs<T> a) {
  const unsigned m0 = a.axis == 0 ? a.band.nout : a.n[0];
  const unsigned m1 = a.axis == 1 ? a.band.nout : a.n[1];
  const unsigned m2 = a.axis == 2 ? a.band.nout : a.n[2];
  const unsigned t = blockIdx.x * kVB + threadIdx.x;
  if (t >= m0 * m1) return;
  const unsigned c = blockIdx.y / m2, i2 = blockIdx.y - c * m2;
  const unsigned i1 = t / m0, i0 = t - i1 * m0;
  const unsigned o = a.axis == 0 ? i0 : a.axis == 1 ? i1 : i2;
  const unsigned st = (unsigned)a.band.start[o];
  const unsigned j0 = a.axis == 0 ? st : i0, j1 = a.axis == 1 ? st : i1, j2 = a.axis == 2 ? st : i2;
  const unsigned n0 = a.n[0], n1 = a.n[1];
  const unsigned stride = a.axis == 0 ? 1u : a.axis == 1 ? n0 : n0 * n1;
  const T* src = in + c * a.in_cs + (j0 + n0 * (j1 + n1 * j2));
  const T* v = a.band.vals + (long long)o * a.band.K;
  T s = 0;
  if constexpr (KB > 0) {
    T w[KB], x[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      w[k] = v[k];
      x[k] = src[k * stride];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) s += w[k] * x[k];
  } else {
    for (int k = 0; k < a.band.K; ++k) s += v[k] * src[k * stride];
  }
  const long long ob = c * a.out_cs + (i0 + m0 * (i1 + m1 * i2));
  if (a.mask && (node_faces((int)i0, (int)i1, (int)i2, a.lt.L, a.lt.dim) & a.lt.fmask[c])) s = T(0);
  out[ob] = a.add ? out[ob] + s : s;
}

struct FaceVals {
  double v[6][3];
};

__device__ __forceinline__ int last_face(const Lattice& lt, long long dof, int& comp) {
  comp = (int)(dof / lt.nn);
  long long n = dof - comp * lt.nn;
  const int i = (int)(n % lt.L);
  n /= lt.L;
  const int j = (int)(n % lt.L);
  const int k = (int)(n / lt.L);
  int f = -1;
  const int lat[3] = {i, j, k};
  for (int ax = 0; ax < lt.dim; ++ax)
    for (int side = 0; side < 2; ++side) {
      const int ff = 2 * ax + side;
      if (lat[ax] == (side ? lt.L - 1 : 0) && ((lt.fmask[comp] >> ff) & 1u)) f = ff;
    }
  return f;
}

__global__ void k_set_dirichlet(double* __restrict__ u, Lattice lt, FaceVals fv, double scale, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    int c;
    const int f = last_face(lt, i, c);
    if (f >= 0) u[i] = scale * fv.v[f][c];
  }
}

// Nodal forces of dead face tractions: f[c, node] = sum over the loaded faces
// f holding the node of t_f[c] * prod over the face's tangential axes a of
// g[index_a], with g the 1-D lattice integrals of the global basis functions.
__global__ void k_traction(double* __restrict__ f, Lattice lt, FaceVals tr, const double* __restrict__ g,
                           long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    const int c = (int)(i / lt.nn);
    long long r = i - c * lt.nn;
    const int ix = (int)(r % lt.L);
    r /= lt.L;
    const int iy = (int)(r % lt.L);
    const int iz = lt.dim == 3 ? (int)(r / lt.L) : 0;
    const int idx[3] = {ix, iy, iz};
    double acc = 0.0;
    for (int axis = 0; axis < lt.dim; ++axis)
      for (int side = 0; side < 2; ++side) {
        if (idx[axis] != (side == 0 ? 0 : lt.L - 1)) continue;
        double w = tr.v[2 * axis + side][c];
        if (w == 0.0) continue;
        for (int a = 0; a < lt.dim; ++a)
          if (a != axis) w *= g[idx[a]];
        acc += w;
      }
    f[i] = acc;
  }
}

// CSR pattern of K_c on the lattice, one thread per row: a free row (c, node)
// lists component-major the nodes of the cells holding the node (per axis the
// range [lo, lo + len) of csr_axis_range, x fastest), a constrained row its
// diagonal only (value 1).  Values of free rows start at zero.
__device__ __forceinline__ void csr_range(int I, int P, int L, int& lo, int& len) {
  if (I % P != 0) {
    lo = I - I % P;
    len = P + 1;
  } else {
    lo = I - P > 0 ? I - P : 0;
    len = (I + P < L - 1 ? I + P : L - 1) - lo + 1;
  }
}

__global__ void k_csr_pattern(const long long* __restrict__ row_ptr, int* __restrict__ col,
                              double* __restrict__ val, Lattice lt, int P, long long n) {
  for (long long r = blockIdx.x * (long long)kVB + threadIdx.x; r < n; r += (long long)gridDim.x * kVB) {
    const long long p0 = row_ptr[r];
    if (constrained_dof(lt, r)) {
      col[p0] = (int)r;
      val[p0] = 1.0;
      continue;
    }
    const int c = (int)(r / lt.nn);
    long long m = r - c * lt.nn;
    const int I = (int)(m % lt.L);
    m /= lt.L;
    const int J = (int)(m % lt.L);
    const int K = lt.dim == 3 ? (int)(m / lt.L) : 0;
    int lo[3] = {0, 0, 0}, len[3] = {1, 1, 1};
    csr_range(I, P, lt.L, lo[0], len[0]);
    csr_range(J, P, lt.L, lo[1], len[1]);
    if (lt.dim == 3) csr_range(K, P, lt.L, lo[2], len[2]);
    long long q = p0;
    for (int k = 0; k < lt.dim; ++k)
      for (int z = lo[2]; z < lo[2] + len[2]; ++z)
        for (int y = lo[1]; y < lo[1] + len[1]; ++y)
          for (int x = lo[0]; x < lo[0] + len[0]; ++x) {
            col[q] = (int)(k * lt.nn + x + (long long)lt.L * (y + (long long)lt.L * z));
            val[q] = 0.0;
            ++q;
          }
  }
}

// y = A x for a CSR matrix (FP64).  A group of G lanes per row (64 / G rows
// per wavefront), U entries per lane loaded before their products are summed
// (loads in flight hide the latency of the dependent x gathers), then a
// butterfly sum inside the group.  Small groups with deep unrolling measured
// fastest on the lattice patterns (mean rows of 80-650 entries); non-temporal
// loads of the matrix were slower.
template <int G, int U>
__global__ void __launch_bounds__(256) k_csr_spmv(const long long* __restrict__ row_ptr, const int* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ x,
                                                  double* __restrict__ y, long long n) {
  constexpr int RPW = 64 / G;   // rows per wavefront
  const int lane = threadIdx.x & 63;
  const long long r = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW + lane / G;
  const int l = lane % G;
  double s = 0.0;
  if (r < n) {
    const long long e = row_ptr[r + 1];
    long long q = row_ptr[r] + l;
    for (; q + (U - 1) * G < e; q += U * G) {
      double v[U];
      int c[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        v[k] = val[q + k * G];
        c[k] = col[q + k * G];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) s += v[k] * x[c[k]];
    }
    for (; q < e; q += G) s += val[q] * x[col[q]];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (r < n && l == 0) y[r] = s;
}

__global__ void k_dirichlet_delta(const double* __restrict__ u, double* __restrict__ dg, Lattice lt, FaceVals fv,
                                  double scale, long long n) {
  for (long long i = blockIdx.x * (long long)kVB + threadIdx.x; i < n; i += (long long)gridDim.x * kVB) {
    int c;
    const int f = last_face(lt, i, c);
    dg[i] = f >= 0 ? scale * fv.v[f][c] - u[i] : 0.0;
  }
}

__global__ void k_material_bits(uint32_t* __restrict__ bits, long long ncells, int N, int dim, int n1,
                                Tables<double> tb, double h, const double* __restrict__ incl, int nincl, int nwords) {
  const int nq = dim == 3 ? n1 * n1 * n1 : n1 * n1;
  const long long total = ncells * nwords;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const long long e = g / nwords;
    const int w = (int)(g - e * nwords);
    const int ex = (int)(e % N), ey = (int)((e / N) % N), ez = dim == 3 ? (int)(e / ((long long)N * N)) : 0;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int q = w * 32 + b;
      if (q >= nq) break;
      const int qx = q % n1, qy = (q / n1) % n1, qz = q / (n1 * n1);
      double X[3] = {h * (ex + tb.xg[qx]), h * (ey + tb.xg[qy]), dim == 3 ? h * (ez + tb.xg[qz]) : 0.0};
      int id = 0;
      for (int s = 0; s < nincl; ++s) {
        const double* row = incl + (long long)s * (dim + 2);
        double d2 = 0;
        for (int k = 0; k < dim; ++k) d2 += (X[k] - row[k]) * (X[k] - row[k]);
        if (d2 <= row[dim] * row[dim]) id = (int)row[dim + 1];
      }
      if (id) word |= 1u << b;
    }
    bits[g] = word;
  }
}

// ---- coarse solve -----------------------------------------------------------------

constexpr int kGJ = 64;

// Coarse inverse by symmetric block Gauss-Jordan.  A plain pass (diagonal
// pivots in order) runs first and is kept when all its pivots are positive
// and above the singularity threshold (a positive definite matrix, for which
// elimination without exchanges is stable).  Otherwise the pass with
// Bunch-Kaufman pivoting described next runs; its launches are gated on the
// device by the plain pass's verdict, so no host round trip decides between
// them.  Each block step of the pivoted pass chooses its (up to) 64 pivots on the current Schur
// complement of the unswept positions [k0, n) (the update kernels keep those
// entries current): the unswept index k of largest |diagonal|, lambda = the
// largest off-diagonal |entry| of its column (row r); k alone when |a_kk| >=
// alpha lambda or |a_kk| sigma >= alpha lambda^2 (sigma: largest off-diagonal
// |entry| of column r), r alone when |a_rr| >= alpha sigma, else the 2x2 block
// {k, r} (alpha = (1 + sqrt 17) / 8).  The columns are formed lazily, from the
// matrix at the step's start minus the updates of the pivots already chosen,
// so the choice sees whole columns, as unblocked Bunch-Kaufman does.  The
// chosen positions are then exchanged (rows and columns, symmetrically, the
// free-DoF permutation following) into the block window [k0, k0 + nb), and
// the block is swept in the chosen order (1x1 and 2x2 pivots).  Sweeps
// commute, so the result is the inverse in the permuted basis; the pivots are
// those of a symmetric block LDL^T elimination, whose signs give the inertia
// (Sylvester).  At the block's last slot a needed 2x2 pivot is replaced by
// the 1x1 pivot of the larger of |a_kk|, |a_rr|.

// Wave-wide argmax of (v, i) over 64 lanes (larger v, then smaller i wins).
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

__device__ __forceinline__ double mag(double x) { return isfinite(x) ? fabs(x) : INFINITY; }   // non-finite first

constexpr int kSel = 1024;   // threads of the pivot-choice kernel
constexpr int kPerMax = (kGJMaxFree + kSel - 1) / kSel;   // positions per thread at the largest size
constexpr int kKeepMax = 5;   // up to this many positions per thread, a formed column also stays in registers

// Block-wide argmax over kSel threads; every thread gets the result.
__device__ __forceinline__ void block_argmax(double& v, int& i, double* sv, int* si) {
  wave_argmax(v, i);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    v = threadIdx.x < kSel / 64 ? sv[threadIdx.x] : -1.0;
    i = threadIdx.x < kSel / 64 ? si[threadIdx.x] : 0x7fffffff;
    wave_argmax(v, i);
    if (threadIdx.x == 0) {
      sv[kSel / 64] = v;
      si[kSel / 64] = i;
    }
  }
  __syncthreads();
  v = sv[kSel / 64];
  i = si[kSel / 64];
  __syncthreads();
}

// Column k (position relative to k0) of the current Schur complement into
// V[slot]: row k of the matrix at the step's start (the unswept block is
// symmetric) minus the updates of the pivot groups chosen so far.  Thread t
// handles positions q = t + j kSel (j < KP) and, when KP <= kKeepMax, keeps
// its entries in cq[j].  Returns to every thread the column's diagonal entry
// ckk and the largest |entry| lam over the unswept positions other than k
// (own bit j of tk set: swept), at position r (lam = -1 when there is none).
template <int KP>
__device__ __forceinline__ void form_column(const double* __restrict__ A, long long n, long long k0, int m, int k, double* V,
                            int slot, int ng, const int* gs, const int* gn, const double (*einv)[3], double* wk,
                            unsigned tk, double* sv, int* si, double* bc, double (&cq)[KP], double& ckk,
                            double& lam, int& r) {
  const int t = threadIdx.x;
  if (t < ng) {
    const int s0 = gs[t];
    if (gn[t] == 1) {
      wk[s0] = einv[t][0] * V[(long long)s0 * m + k];
    } else {
      const double a = V[(long long)s0 * m + k], b = V[(long long)(s0 + 1) * m + k];
      wk[s0] = einv[t][0] * a + einv[t][1] * b;
      wk[s0 + 1] = einv[t][1] * a + einv[t][2] * b;
    }
  }
  __syncthreads();
  const int nv = ng > 0 ? gs[ng - 1] + gn[ng - 1] : 0;
  const double* arow = A + (k0 + k) * n + k0;
  double* vs = V + (long long)slot * m;
  double best = -1.0;
  int bi = 0x7fffffff;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int q = t + j * kSel;
    if (q < m) {
      double c = arow[q];
#pragma unroll 8
      for (int u = 0; u < nv; ++u) c -= V[(long long)u * m + q] * wk[u];
      vs[q] = c;
      if constexpr (KP <= kKeepMax) cq[j] = c;
      if (q == k) {
        bc[0] = c;
      } else if (!((tk >> j) & 1u)) {
        const double a = mag(c);
        if (a > best) {
          best = a;
          bi = q;
        }
      }
    }
  }
  block_argmax(best, bi, sv, si);   // its barriers also publish bc[0] and vs
  ckk = bc[0];
  lam = best;
  r = bi;
}

// Chooses the block's pivots (see above) and writes the exchange and the
// pivot list: sw[0] = number of exchange pairs q, sw[1 + i] / sw[1 + kGJ + i]
// = window / outside position of pair i, sw[1 + 2 kGJ + t] = window-relative
// position of pivot t (after the exchange), sw[1 + 3 kGJ + t] = 1 (1x1 pivot),
// 2 / 3 (first / second index of a 2x2 pivot).  V: nb vectors of n - k0
// doubles (scratch).  One workgroup of kSel threads; thread t keeps the
// current Schur-complement diagonal of its positions t + j kSel (j < KP,
// KP kSel >= n - k0) in registers, and their swept flags in tk.
template <int KP>
__global__ void __launch_bounds__(kSel) k_gj_choose(const double* __restrict__ A, long long n, long long k0, int nb,
                                                    double* __restrict__ V, int* __restrict__ sw,
                                                    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  __shared__ double sv[kSel / 64 + 1];
  __shared__ int si[kSel / 64 + 1];
  __shared__ double wk[kGJ];
  __shared__ double einv[kGJ][3];
  __shared__ double bc[1];
  __shared__ int gs[kGJ], gn[kGJ];
  __shared__ int sel[kGJ], kind[kGJ];
  const double alpha = 0.6403882032022076;   // (1 + sqrt(17)) / 8
  const int t = threadIdx.x;
  const int m = (int)(n - k0);
  double dq[KP], cq[KP];
  unsigned tk = 0u;
  double best = -1.0;
  int k = 0x7fffffff;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int q = t + j * kSel;
    dq[j] = 0.0;
    cq[j] = 0.0;
    if (q < m) {
      dq[j] = A[(k0 + q) * n + k0 + q];
      const double a = mag(dq[j]);
      if (a > best) {
        best = a;
        k = q;
      }
    }
  }
  block_argmax(best, k, sv, si);   // m > 0 unswept positions: k is one of them
  int cnt = 0, ng = 0;
  while (cnt < nb) {
    double ckk, lam, sig, crr;
    int r, ri;
    form_column<KP>(A, n, k0, m, k, V, cnt, ng, gs, gn, einv, wk, tk, sv, si, bc, cq, ckk, lam, r);
    const double akk = mag(ckk);
    double p = ckk;     // 1x1 pivot value
    int pk = k, two = 0;
    bool in_regs = true;   // cq holds the column in slot cnt
    if (lam > 0.0 && akk < alpha * lam) {
      const int slot_r = cnt + (cnt + 1 < nb ? 1 : 0);
      // (at the last slot column r overwrites column k: only r's diagonal and sigma are needed)
      form_column<KP>(A, n, k0, m, r, V, slot_r, ng, gs, gn, einv, wk, tk, sv, si, bc, cq, crr, sig, ri);
      const double arr = mag(crr);
      if (akk * sig >= alpha * lam * lam) {
        pk = k;
      } else if (arr >= alpha * sig) {
        pk = r;
      } else if (cnt + 1 < nb) {
        two = 1;
      } else {
        pk = arr > akk ? r : k;   // last slot: no room for a 2x2 pivot
      }
      if (!two && (pk == r) != (cnt + 1 >= nb)) {   // bring the chosen column into slot cnt
        double c2, l2;
        int r2;
        form_column<KP>(A, n, k0, m, pk, V, cnt, ng, gs, gn, einv, wk, tk, sv, si, bc, cq, c2, l2, r2);
        p = c2;
      } else if (!two && pk == r) {   // last slot: column r already sits in slot cnt (and in cq)
        p = crr;
      } else {   // column k in slot cnt but cq holds column r, or a 2x2 pivot
        in_regs = false;
      }
    }
    // record the group (read by the next form_column after the barriers below)
    const double* c0 = V + (long long)cnt * m;
    const double* c1 = V + (long long)(cnt + 1) * m;
    double e00 = 0.0, e01 = 0.0, e11 = 0.0;
    if (!two) {
      e00 = 1.0 / p;
      if (t == 0) {
        gs[ng] = cnt;
        gn[ng] = 1;
        einv[ng][0] = e00;
        sel[cnt] = pk;
        kind[cnt] = 1;
      }
    } else {
      const double a = ckk, b = c0[r], c = crr;
      const double det = a * c - b * b;
      e00 = c / det;
      e01 = -b / det;
      e11 = a / det;
      if (t == 0) {
        gs[ng] = cnt;
        gn[ng] = 2;
        einv[ng][0] = e00;
        einv[ng][1] = e01;
        einv[ng][2] = e11;
        sel[cnt] = k;
        kind[cnt] = 2;
        sel[cnt + 1] = r;
        kind[cnt + 1] = 3;
      }
    }
    // update the diagonal of the unswept positions and choose the next k
    best = -1.0;
    int kn = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int q = t + j * kSel;
      if (q < m) {
        if (q == pk || (two && (q == k || q == r))) tk |= 1u << j;
        if (!((tk >> j) & 1u)) {
          if (!two) {
            const double v = KP <= kKeepMax && in_regs ? cq[j] : c0[q];
            dq[j] -= v * v * e00;
          } else {
            const double v0 = c0[q], v1 = c1[q];
            dq[j] -= e00 * v0 * v0 + 2.0 * e01 * v0 * v1 + e11 * v1 * v1;
          }
          const double a = mag(dq[j]);
          if (a > best) {
            best = a;
            kn = q;
          }
        }
      }
    }
    cnt += two ? 2 : 1;
    ++ng;
    block_argmax(best, kn, sv, si);   // no unswept position left: kn unused (the loop ends)
    k = kn;
  }
  __shared__ bool in_window[kGJ];
  __shared__ int wpos[kGJ];
  if (t == 0) {   // exchange pairs: window positions not chosen <-> chosen positions outside
    for (int w = 0; w < nb; ++w) in_window[w] = false;
    for (int c = 0; c < nb; ++c)
      if (sel[c] < nb) in_window[sel[c]] = true;
    int q = 0;
    for (int w = 0; w < nb; ++w)
      if (!in_window[w]) wpos[q++] = w;
    int o = 0;
    for (int c = 0; c < nb; ++c) {
      int pos = sel[c];
      if (pos >= nb) {
        sw[1 + o] = (int)(k0 + wpos[o]);
        sw[1 + kGJ + o] = (int)(k0 + pos);
        pos = wpos[o];
        ++o;
      }
      sw[1 + 2 * kGJ + c] = pos;
      sw[1 + 3 * kGJ + c] = kind[c];
    }
    sw[0] = o;
  }
}

// Symmetric exchange of the pairs of sw: rows first (this kernel), then
// columns and the permutation (k_gj_swap_cols), as two launches.
__global__ void k_gj_swap_rows(double* __restrict__ A, long long n, const int* __restrict__ sw,
                               const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const int q = sw[0];
  const long long total = (long long)q * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const int pr = (int)(g / n);
    const long long j = g - (long long)pr * n;
    double* ra = A + (long long)sw[1 + pr] * n + j;
    double* rb = A + (long long)sw[1 + kGJ + pr] * n + j;
    const double va = *ra, vb = *rb;
    *ra = vb;
    *rb = va;
  }
}

__global__ void k_gj_swap_cols(double* __restrict__ A, long long n, const int* __restrict__ sw, int* __restrict__ perm,
                               const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const int q = sw[0];
  const long long total = (long long)q * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const long long i = g / q;
    const int pr = (int)(g - i * q);
    const int ca = sw[1 + pr], cb = sw[1 + kGJ + pr];
    double* ea = A + i * n + ca;
    double* eb = A + i * n + cb;
    const double va = *ea, vb = *eb;
    *ea = vb;
    *eb = va;
    if (i == 0) {
      const int pa = perm[ca];
      perm[ca] = perm[cb];
      perm[cb] = pa;
    }
  }
}

// Inverts the symmetric pivot block [k0, k0 + nb) by Gauss-Jordan sweeps
// (the block held in registers) in the order and grouping k_gj_choose
// recorded (sw).  flag[1] accumulates the negative eigenvalues of the pivots;
// flag[0] is set when a pivot (or a 2x2 determinant against its largest
// entry) is not finite or at most tol * scale[0] in magnitude (numerically
// singular).
constexpr int kPivT = 1024;   // threads of the pivot-block kernel
__global__ void __launch_bounds__(kPivT) k_gj_pivot(double* __restrict__ A, long long n, long long k0, int nb,
                                                  double* __restrict__ Pinv, int* flag, const double* scale,
                                                  double tol, const int* __restrict__ sw,
                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  // thread t keeps column j = t % kGJ of rows i0 + kGroups r (i0 = t / kGJ,
  // r < kPerT) in registers; each step broadcasts the pivot rows and columns
  // through LDS (double-buffered, one barrier per step)
  constexpr int kGroups = kPivT / kGJ, kPerT = kGJ / kGroups;
  __shared__ double bc[2][4][kGJ];      // [buffer][col k, row k, col r, row r][index]
  __shared__ int pos[kGJ], kind[kGJ];   // the pivot list
  const int t = threadIdx.x;
  const int j = t % kGJ, i0 = t / kGJ;
  const double thr = tol * scale[0];
  if (t < nb) {
    pos[t] = sw[1 + 2 * kGJ + t];
    kind[t] = sw[1 + 3 * kGJ + t];
  }
  double m[kPerT];
#pragma unroll
  for (int r = 0; r < kPerT; ++r) {
    const int i = i0 + kGroups * r;
    m[r] = (i < nb && j < nb) ? A[(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  bool bad = false;   // pivot checks of thread 0, written once at the end
  int neg = 0;
  int buf = 0;
  for (int step = 0; step < nb;) {
    const int k = pos[step];
    const bool two = kind[step] != 1;
    const int r2 = two ? pos[step + 1] : k;
    double* ck = bc[buf][0];
    double* rk = bc[buf][1];
    double* cr = bc[buf][2];
    double* rr = bc[buf][3];
    // publish column k (and r) from the threads owning it, row k (and r) likewise
    if (j == k || (two && j == r2)) {
      double* dst = j == k ? ck : cr;
#pragma unroll
      for (int r = 0; r < kPerT; ++r) dst[i0 + kGroups * r] = m[r];
    }
    if (i0 == (k % kGroups) || (two && i0 == (r2 % kGroups))) {
      double vk = 0.0, vr = 0.0;
#pragma unroll
      for (int r = 0; r < kPerT; ++r) {
        vk = r == k / kGroups ? m[r] : vk;
        vr = r == r2 / kGroups ? m[r] : vr;
      }
      if (i0 == (k % kGroups)) rk[j] = vk;
      if (two && i0 == (r2 % kGroups)) rr[j] = vr;
    }
    __syncthreads();
    if (!two) {   // 1x1 pivot
      const double p = rk[k];
      if (t == 0) {
        bad = bad || !(fabs(p) > thr) || !isfinite(p);
        neg += p < 0.0 ? 1 : 0;
      }
      const double pinv = 1.0 / p;
      // branch-free (selects), so that m stays in place in registers
      const double rj = rk[j] * pinv;
      const double rowv = j == k ? pinv : rj;
#pragma unroll
      for (int r = 0; r < kPerT; ++r) {
        const int i = i0 + kGroups * r;
        const double ci = ck[i];
        const double v = i == k ? rowv : (j == k ? -ci * pinv : m[r] - ci * rj);
        m[r] = (i < nb && j < nb) ? v : m[r];
      }
      step += 1;
    } else {   // 2x2 pivot {k, r}: E = [[a, b], [b, c]]
      const double a = rk[k], b = rk[r2], c = rr[r2];
      const double det = a * c - b * b;
      if (t == 0) {
        bad = bad || !(fabs(det) > thr * fmax(fabs(b), fmax(fabs(a), fabs(c)))) || !isfinite(det);
        neg += det < 0.0 ? 1 : (a + c < 0.0 ? 2 : 0);
      }
      const double e00 = c / det, e01 = -b / det, e11 = a / det;   // E^-1
      const bool jb = j == k || j == r2;
      const double sk = e00 * rk[j] + e01 * rr[j];   // (E^-1 M_Bj)_k
      const double sr = e01 * rk[j] + e11 * rr[j];   // (E^-1 M_Bj)_r
      const double ek = j == k ? e00 : e01, er = j == k ? e01 : e11;   // column j of E^-1
#pragma unroll
      for (int r = 0; r < kPerT; ++r) {
        const int i = i0 + kGroups * r;
        const double ci = ck[i], di = cr[i];
        const double inb = jb ? (i == k ? ek : er) : (i == k ? sk : sr);
        const double v = (i == k || i == r2) ? inb : (jb ? -(ci * ek + di * er) : m[r] - (ci * sk + di * sr));
        m[r] = (i < nb && j < nb) ? v : m[r];
      }
      step += 2;
    }
    buf ^= 1;   // the next step writes the other buffer; the one after waits behind its barrier
  }
  if (j < nb) {
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
      const int i = i0 + kGroups * r;
      if (i < nb) Pinv[i * nb + j] = m[r];
    }
  }
  if (t == 0) {
    if (bad) flag[0] = 1;
    flag[1] += neg;
  }
}

// scale[0] = max_i |A[i][i]|
__global__ void k_diag_absmax(const double* __restrict__ A, long long n, double* scale, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  __shared__ double sh[kVB];
  double m = 0;
  for (long long i = threadIdx.x; i < n; i += kVB) m = fmax(m, fabs(A[i * n + i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kVB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[0] = sh[0];
}

// R[t][j] = sum_s Pinv[t][s] A[k0+s][j]
__global__ void k_gj_rowpanel(const double* __restrict__ A, long long n, long long k0, int nb,
                              const double* __restrict__ Pinv, double* __restrict__ R, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long total = (long long)nb * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const int t = (int)(g / n);
    const long long j = g - (long long)t * n;
    double s = 0;
    for (int q = 0; q < nb; ++q) s += Pinv[t * nb + q] * A[(k0 + q) * n + j];
    R[g] = s;
  }
}

// Cb[i][t] = A[i][k0+t]
__global__ void k_gj_colpanel(const double* __restrict__ A, long long n, long long k0, int nb, double* __restrict__ Cb,
                              const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long total = (long long)nb * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const long long i = g / nb;
    const int t = (int)(g - i * nb);
    Cb[g] = A[i * n + k0 + t];
  }
}

// A[i][j] -= sum_t Cb[i][t] R[t][j]   for i, j outside the pivot block
__global__ void __launch_bounds__(256) k_gj_update(double* __restrict__ A, long long n, long long k0, int nb,
                                                   const double* __restrict__ Cb, const double* __restrict__ R,
                                                   const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long bi = blockIdx.y, bj = blockIdx.x;
  const long long kb = k0 / kGJ;
  if (bi == kb || bj == kb) return;
  __shared__ double Cs[kGJ][kGJ + 1];
  __shared__ double Rs[kGJ][kGJ + 1];
  const int t = threadIdx.x;
  const long long i0 = bi * kGJ, j0 = bj * kGJ;
  for (int e = t; e < kGJ * kGJ; e += 256) {
    const int r = e / kGJ, c = e % kGJ;
    Cs[r][c] = (i0 + r < n && c < nb) ? Cb[(i0 + r) * nb + c] : 0.0;
    Rs[r][c] = (r < nb && j0 + c < n) ? R[(long long)r * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int ty = t / 16, tx = t % 16;
  double acc[4][4] = {};
  for (int q = 0; q < nb; ++q) {
    double a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = Cs[ty * 4 + r][q];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = Rs[q][tx * 4 + c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long long i = i0 + ty * 4 + r;
    if (i >= n) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long j = j0 + tx * 4 + c;
      if (j < n) A[i * n + j] -= acc[r][c];
    }
  }
}

// Column k block: A[i][k0+t] = -sum_s Cb[i][s] Pinv[s][t] (i outside), Pinv inside.
__global__ void k_gj_fincol(double* __restrict__ A, long long n, long long k0, int nb, const double* __restrict__ Cb,
                            const double* __restrict__ Pinv, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long total = (long long)nb * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const long long i = g / nb;
    const int t = (int)(g - i * nb);
    double v;
    if (i >= k0 && i < k0 + nb) {
      v = Pinv[(i - k0) * nb + t];
    } else {
      v = 0;
      for (int s = 0; s < nb; ++s) v -= Cb[i * nb + s] * Pinv[s * nb + t];
    }
    A[i * n + k0 + t] = v;
  }
}

// Row k block: A[k0+t][j] = R[t][j] for j outside the pivot block.
__global__ void k_gj_finrow(double* __restrict__ A, long long n, long long k0, int nb, const double* __restrict__ R,
                            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long total = (long long)nb * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const int t = (int)(g / n);
    const long long j = g - (long long)t * n;
    if (j >= k0 && j < k0 + nb) continue;
    A[(k0 + t) * n + j] = R[g];
  }
}

// Pivot list of a block step without pivoting: the window's diagonal in order.
__global__ void k_gj_plain_order(int* __restrict__ sw, int nb) {
  const int t = threadIdx.x;
  if (t == 0) sw[0] = 0;
  if (t < nb) {
    sw[1 + 2 * kGJ + t] = t;
    sw[1 + 3 * kGJ + t] = 1;
  }
}

// dst = src (n entries) when the gate is open.
__global__ void k_copy_gated(const double* __restrict__ src, double* __restrict__ dst, long long n,
                             const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < n; g += (long long)gridDim.x * kVB) dst[g] = src[g];
}

// Accepts the plain pass when every pivot was positive and above the
// singularity threshold: the matrix is then positive definite (Sylvester) and
// elimination without exchanges is stable (no element growth).  Otherwise
// sets flag[2], the gate of the pivoted pass, and clears the plain pass's
// pivot flags.
__global__ void k_plain_decide(int* __restrict__ flag) {
  if (threadIdx.x != 0) return;
  const bool ok = flag[0] == 0 && flag[1] == 0;
  flag[2] = ok ? 0 : 1;
  if (!ok) {
    flag[0] = 0;
    flag[1] = 0;
  }
}

template <typename T>
__global__ void k_coarse_gather(const T* __restrict__ r, const int* __restrict__ dof_of, long long nf,
                                double* __restrict__ rf) {
  for (long long f = blockIdx.x * (long long)kVB + threadIdx.x; f < nf; f += (long long)gridDim.x * kVB)
    rf[f] = (double)r[dof_of[f]];
}

__global__ void k_gemv_rows(const double* __restrict__ K, long long nf, const double* __restrict__ x,
                            double* __restrict__ y) {
  __shared__ double sh[kVB];
  const long long i = blockIdx.x;
  const double* row = K + i * nf;
  double acc = 0;
  for (long long j = threadIdx.x; j < nf; j += kVB) acc += row[j] * x[j];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) y[i] = s;
}

template <typename T>
__global__ void k_coarse_scatter(const double* __restrict__ zf, const int* __restrict__ dof_of, long long nf,
                                 T* __restrict__ z) {
  for (long long f = blockIdx.x * (long long)kVB + threadIdx.x; f < nf; f += (long long)gridDim.x * kVB)
    z[dof_of[f]] = (T)zf[f];
}

}  // namespace

// ---- launch wrappers ------------------------------------------------------------------

template <typename T>
void fill_dirichlet(T* y, const T* x, long long n, const Lattice& lt, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_dirichlet<T>, dim3(grid_for(n)), dim3(kVB), 0, s, y, x, n, lt);
}
template <typename T>
void fill_dirichlet_batch(const FillItem<T>* items, const long long* off, int n, long long chunks, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_dirichlet_batch<T>, dim3(grid_for(chunks * kVB, 8192)), dim3(kVB), 0, s, items, off, n);
}
template <typename T>
void zero_constrained(T* v, long long n, const Lattice& lt, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_constrained<T>, dim3(grid_for(n)), dim3(kVB), 0, s, v, n, lt);
}
template <typename T>
void fill(T* v, T val, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kVB), 0, s, v, val, n);
}
template <typename TI, typename TO>
void cast(const TI* in, TO* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<TI, TO>), dim3(grid_for(n)), dim3(kVB), 0, s, in, out, n);
}
template <typename TA, typename TB>
void dot(const TA* a, const TB* b, long long n, double* part, double* out, hipStream_t s) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL((k_dot_part<TA, TB>), dim3(g), dim3(kVB), 0, s, a, b, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kVB), 0, s, part, (int)g, out);
}
void min_reduce(const double* part, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kVB), 0, s, part, np, out);
}
void set_scalar(double* p, double v, hipStream_t s) { hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, p, v); }
void scalar_div(double* sc, int dst, int num, int den, int copy_to, int copy_from, double* hist, int hidx,
                hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_div, dim3(1), dim3(1), 0, s, sc, dst, num, den, copy_to, copy_from, hist, hidx);
}
template <typename T>
void cg_update(T* x, T* r, const T* p, const T* Ap, long long n, const double* sc, double* part, hipStream_t s) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_cg_update<T>, dim3(g), dim3(kVB), 0, s, x, r, p, Ap, n, sc, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kVB), 0, s, part, (int)g, const_cast<double*>(sc) + SC_RR);
}
template <typename T>
void lanczos_update(T* r, T* z, const T* Ap, const T* dinv, long long n, const double* sc, double* part,
                    hipStream_t s) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_lanczos_update<T>, dim3(g), dim3(kVB), 0, s, r, z, Ap, dinv, n, sc, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kVB), 0, s, part, (int)g, const_cast<double*>(sc) + SC_RZNEW);
}
template <typename T>
void cg_pupdate(T* p, const T* z, long long n, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_pupdate<T>, dim3(grid_for(n)), dim3(kVB), 0, s, p, z, n, sc);
}
template <typename T>
void axpby(T* y, const T* x, T a, T b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n)), dim3(kVB), 0, s, y, x, a, b, n);
}
template <typename T>
void lincomb3(T* z, T a, const T* x, T b, const T* y, T c, const T* w, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb3<T>, dim3(grid_for(n)), dim3(kVB), 0, s, z, a, x, b, y, c, w, n);
}
template <typename T>
void cheb_step(const T* f, const T* t, const T* dinv, T* d, T* x, T cd, T cr, int xzero, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cheb<T>, dim3(grid_for(n)), dim3(kVB), 0, s, f, t, dinv, d, x, cd, cr, xzero, n);
}
template <typename T>
void set_constrained(T* v, T val, long long n, const Lattice& lt, hipStream_t s) {
  hipLaunchKernelGGL(k_set_constrained<T>, dim3(grid_for(n)), dim3(kVB), 0, s, v, val, n, lt);
}
template <typename T>
void splitmix_uniform(T* v, long long n, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_splitmix<T>, dim3(grid_for(n)), dim3(kVB), 0, s, v, n, seed);
}
template <typename TO>
void reciprocal(const double* in, TO* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_reciprocal<TO>, dim3(grid_for(n)), dim3(kVB), 0, s, in, out, n);
}
template <typename T>
void sweep(const T* in, T* out, const SweepArgs<T>& a, hipStream_t s) {
  const long long m0 = a.axis == 0 ? a.band.nout : a.n[0], m1 = a.axis == 1 ? a.band.nout : a.n[1];
  const long long m2 = a.axis == 2 ? a.band.nout : a.n[2];
  const long long in_per = (long long)a.n[0] * a.n[1] * a.n[2];
  if (m0 * m1 >= (1LL << 31) || in_per >= (1LL << 32) || m0 * m1 * m2 >= (1LL << 32) || m2 * a.comps > 65535)
    throw std::runtime_error("transfer sweep: lattice too large for the 32-bit sweep indices");
  const dim3 grid((unsigned)((m0 * m1 + kVB - 1) / kVB), (unsigned)(m2 * a.comps));
  switch (a.band.K) {
#define MFH_SWEEP_K(K) \
  case K:              \
    hipLaunchKernelGGL((k_sweep<T, K>), grid, dim3(kVB), 0, s, in, out, a); \
    break;
    MFH_SWEEP_K(1) MFH_SWEEP_K(2) MFH_SWEEP_K(3) MFH_SWEEP_K(4) MFH_SWEEP_K(5)
    MFH_SWEEP_K(6) MFH_SWEEP_K(7) MFH_SWEEP_K(8) MFH_SWEEP_K(9)
#undef MFH_SWEEP_K
    default:
      hipLaunchKernelGGL((k_sweep<T, 0>), grid, dim3(kVB), 0, s, in, out, a);
  }
}

void set_dirichlet(double* u, const Lattice& lt, const double* fv, double scale, long long n, hipStream_t s) {
  FaceVals f = {};
  for (int face = 0; face < 2 * lt.dim; ++face)
    for (int c = 0; c < lt.dim; ++c) f.v[face][c] = fv[face * lt.dim + c];
  hipLaunchKernelGGL(k_set_dirichlet, dim3(grid_for(n)), dim3(kVB), 0, s, u, lt, f, scale, n);
}
void traction_force(double* f, const Lattice& lt, const double* ft, const double* g, long long n, hipStream_t s) {
  FaceVals t = {};
  for (int face = 0; face < 2 * lt.dim; ++face)
    for (int c = 0; c < lt.dim; ++c) t.v[face][c] = ft[face * lt.dim + c];
  hipLaunchKernelGGL(k_traction, dim3(grid_for(n)), dim3(kVB), 0, s, f, lt, t, g, n);
}
void csr_pattern(const long long* row_ptr, int* col, double* val, const Lattice& lt, int P, long long n,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_csr_pattern, dim3(grid_for(n)), dim3(kVB), 0, s, row_ptr, col, val, lt, P, n);
}
void csr_spmv(const long long* row_ptr, const int* col, const double* val, const double* x, double* y, long long n,
              int group, hipStream_t s) {
  if (n == 0) return;
  const long long rows_per_block = 4 * (64 / group);
  const dim3 grid((unsigned)((n + rows_per_block - 1) / rows_per_block));
  if (group == 16)
    hipLaunchKernelGGL((k_csr_spmv<16, 4>), grid, dim3(256), 0, s, row_ptr, col, val, x, y, n);
  else
    hipLaunchKernelGGL((k_csr_spmv<8, 8>), grid, dim3(256), 0, s, row_ptr, col, val, x, y, n);
}
void dirichlet_delta(const double* u, double* dg, const Lattice& lt, const double* fv, double scale, long long n,
                     hipStream_t s) {
  FaceVals f = {};
  for (int face = 0; face < 2 * lt.dim; ++face)
    for (int c = 0; c < lt.dim; ++c) f.v[face][c] = fv[face * lt.dim + c];
  hipLaunchKernelGGL(k_dirichlet_delta, dim3(grid_for(n)), dim3(kVB), 0, s, u, dg, lt, f, scale, n);
}

void material_bits(uint32_t* bits, long long ncells, int N, int dim, int n1, const Tables<double>& tb, double h,
                   const double* incl, int nincl, int nwords, hipStream_t s) {
  hipLaunchKernelGGL(k_material_bits, dim3(grid_for(ncells * nwords)), dim3(kVB), 0, s, bits, ncells, N, dim, n1, tb,
                     h, incl, nincl, nwords);
}

__global__ void k_unpermute(const double* __restrict__ A, const int* __restrict__ perm, long long n,
                            double* __restrict__ out, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // pivoted pass not needed
  const long long total = n * n;
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < total; g += (long long)gridDim.x * kVB) {
    const long long i = g / n, j = g - i * n;
    out[(long long)perm[i] * n + perm[j]] = A[g];
  }
}
void gj_choose_block(double* A, long long n, long long k0, int nb, double* V, int* sw, int* perm, const int* gate,
                     hipStream_t s) {
  const long long m = n - k0;
  if (m <= 2 * kSel)
    hipLaunchKernelGGL(k_gj_choose<2>, dim3(1), dim3(kSel), 0, s, A, n, k0, nb, V, sw, gate);
  else if (m <= 5 * kSel)
    hipLaunchKernelGGL(k_gj_choose<5>, dim3(1), dim3(kSel), 0, s, A, n, k0, nb, V, sw, gate);
  else if (m <= 10 * kSel)
    hipLaunchKernelGGL(k_gj_choose<10>, dim3(1), dim3(kSel), 0, s, A, n, k0, nb, V, sw, gate);
  else
    hipLaunchKernelGGL(k_gj_choose<kPerMax>, dim3(1), dim3(kSel), 0, s, A, n, k0, nb, V, sw, gate);
  hipLaunchKernelGGL(k_gj_swap_rows, dim3(grid_for((long long)kGJ * n)), dim3(kVB), 0, s, A, n, sw, gate);
  hipLaunchKernelGGL(k_gj_swap_cols, dim3(grid_for((long long)kGJ * n)), dim3(kVB), 0, s, A, n, sw, perm, gate);
}
void gj_pivot(double* A, long long n, long long k0, int nb, double* Pinv, int* flag, const double* scale, double tol,
              const int* sw, const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kPivT), 0, s, A, n, k0, nb, Pinv, flag, scale, tol, sw, gate);
}
void diag_absmax(const double* A, long long n, double* scale, const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_absmax, dim3(1), dim3(kVB), 0, s, A, n, scale, gate);
}
void gj_panels(const double* A, long long n, long long k0, int nb, const double* Pinv, double* Cb, double* R,
               const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_rowpanel, dim3(grid_for((long long)nb * n)), dim3(kVB), 0, s, A, n, k0, nb, Pinv, R, gate);
  hipLaunchKernelGGL(k_gj_colpanel, dim3(grid_for((long long)nb * n)), dim3(kVB), 0, s, A, n, k0, nb, Cb, gate);
}
void gj_update(double* A, long long n, long long k0, int nb, const double* Cb, const double* R, const int* gate,
               hipStream_t s) {
  const unsigned nt = (unsigned)((n + kGJ - 1) / kGJ);
  hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(256), 0, s, A, n, k0, nb, Cb, R, gate);
}
void gj_finish(double* A, long long n, long long k0, int nb, const double* Cb, const double* R, const double* Pinv,
               const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_fincol, dim3(grid_for((long long)nb * n)), dim3(kVB), 0, s, A, n, k0, nb, Cb, Pinv, gate);
  hipLaunchKernelGGL(k_gj_finrow, dim3(grid_for((long long)nb * n)), dim3(kVB), 0, s, A, n, k0, nb, R, gate);
}
// Block Gauss-Jordan sweeps over A in place: pivoted (Bunch-Kaufman choice,
// exchanges, perm following) or in plain diagonal order; every launch of the
// pivoted form is gated.
void gj_blocks(double* A, long long n, int* perm, const DenseInvWork& w, double tol, bool pivoted, const int* gate,
               hipStream_t s) {
  diag_absmax(A, n, w.scale, gate, s);
  for (long long k0 = 0; k0 < n; k0 += kGJ) {
    const int nb = (int)std::min<long long>(kGJ, n - k0);
    if (pivoted)
      gj_choose_block(A, n, k0, nb, w.C, w.sw, perm, gate, s);
    else
      hipLaunchKernelGGL(k_gj_plain_order, dim3(1), dim3(kGJ), 0, s, w.sw, nb);
    gj_pivot(A, n, k0, nb, w.Pinv, w.flag, w.scale, tol, w.sw, gate, s);
    gj_panels(A, n, k0, nb, w.Pinv, w.C, w.R, gate, s);
    gj_update(A, n, k0, nb, w.C, w.R, gate, s);
    gj_finish(A, n, k0, nb, w.C, w.R, w.Pinv, gate, s);
  }
}
void dense_inverse(double* A, double* X, long long n, int* perm, const DenseInvWork& w, double tol, bool natural,
                   hipStream_t s) {
  // plain pass on a copy in X, accepted on the device
  hipLaunchKernelGGL(k_copy_gated, dim3(grid_for(n * n)), dim3(kVB), 0, s, A, X, n * n, nullptr);
  gj_blocks(X, n, perm, w, tol, false, nullptr, s);
  hipLaunchKernelGGL(k_plain_decide, dim3(1), dim3(64), 0, s, w.flag);
  // pivoted pass on A, run only when the plain one was rejected
  const int* gate = w.flag + 2;
  gj_blocks(A, n, perm, w, tol, true, gate, s);
  if (natural)
    hipLaunchKernelGGL(k_unpermute, dim3(grid_for(n * n)), dim3(kVB), 0, s, A, perm, n, X, gate);
  else
    hipLaunchKernelGGL(k_copy_gated, dim3(grid_for(n * n)), dim3(kVB), 0, s, A, X, n * n, gate);
}

__global__ void k_iota(int* __restrict__ v, long long n) {
  for (long long g = blockIdx.x * (long long)kVB + threadIdx.x; g < n; g += (long long)gridDim.x * kVB) v[g] = (int)g;
}
void iota(int* v, long long n, hipStream_t s) { hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kVB), 0, s, v, n); }
template <typename T>
void coarse_apply(const double* Kinv, long long nf, const int* dof_of, const T* r, double* rf, double* zf, T* z,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gather<T>, dim3(grid_for(nf)), dim3(kVB), 0, s, r, dof_of, nf, rf);
  hipLaunchKernelGGL(k_gemv_rows, dim3((unsigned)nf), dim3(kVB), 0, s, Kinv, nf, rf, zf);
  hipLaunchKernelGGL(k_coarse_scatter<T>, dim3(grid_for(nf)), dim3(kVB), 0, s, zf, dof_of, nf, z);
}

#define MFH_INST_T(T)                                                                                          \
  template void fill_dirichlet<T>(T*, const T*, long long, const Lattice&, hipStream_t);                       \
  template void fill_dirichlet_batch<T>(const FillItem<T>*, const long long*, int, long long, hipStream_t);     \
  template void zero_constrained<T>(T*, long long, const Lattice&, hipStream_t);                               \
  template void fill<T>(T*, T, long long, hipStream_t);                                                        \
  template void cg_update<T>(T*, T*, const T*, const T*, long long, const double*, double*, hipStream_t);      \
  template void lanczos_update<T>(T*, T*, const T*, const T*, long long, const double*, double*, hipStream_t); \
  template void cg_pupdate<T>(T*, const T*, long long, const double*, hipStream_t);                            \
  template void axpby<T>(T*, const T*, T, T, long long, hipStream_t);                                          \
  template void lincomb3<T>(T*, T, const T*, T, const T*, T, const T*, long long, hipStream_t);                \
  template void cheb_step<T>(const T*, const T*, const T*, T*, T*, T, T, int, long long, hipStream_t);         \
  template void reciprocal<T>(const double*, T*, long long, hipStream_t);                                      \
  template void set_constrained<T>(T*, T, long long, const Lattice&, hipStream_t);                             \
  template void splitmix_uniform<T>(T*, long long, unsigned long long, hipStream_t);                           \
                                      \
  template void sweep<T>(const T*, T*, const SweepArgs<T>&, hipStream_t);                                      \
  template void coarse_apply<T>(const double*, long long, const int*, const T*, double*, double*, T*, hipStream_t);
MFH_INST_T(float)
MFH_INST_T(double)
#undef MFH_INST_T
template void fill<uint32_t>(uint32_t*, uint32_t, long long, hipStream_t);
template void fill<int>(int*, int, long long, hipStream_t);
template void cast<double, float>(const double*, float*, long long, hipStream_t);
template void cast<float, double>(const float*, double*, long long, hipStream_t);
template void cast<double, double>(const double*, double*, long long, hipStream_t);
template void dot<double, double>(const double*, const double*, long long, double*, double*, hipStream_t);
template void dot<float, float>(const float*, const float*, long long, double*, double*, hipStream_t);

}  // namespace mfh
