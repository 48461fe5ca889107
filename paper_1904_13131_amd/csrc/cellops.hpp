// Cell kernels of the matrix-free operator: gather -> sum factorisation ->
// quadrature-point stage -> transposed sum factorisation -> scatter.
//
// Sec. 5 evaluates eq. (mf_vmult) cell by cell with sum factorisation: every
// reference derivative at the tensor-product Gauss points is a sequence of
// 1-D contractions with the tables S (values) and D (derivatives), and the
// test-function side is the same sequence transposed.
//
// Thread layout (one block = kBlock threads = CPB cells x NP pencils):
//   thread t handles cell t % CPB (consecutive lanes -> neighbouring cells, so
//   the lattice gathers coalesce) and pencil t / CPB.  A pencil is a line of
//   n = p+1 points; 3-D cells have n^2 pencils, 2-D cells n.  The 1-D
//   contraction along a pencil runs in registers; pencils are re-oriented
//   between the x, y and z sweeps through LDS (layout [array][point][cell],
//   cell fastest, so a wave's LDS accesses are consecutive words).  After the
//   forward sweeps each thread owns the Gauss points of one z-line (2-D:
//   y-line) of its cell with all d x d reference derivatives in registers; the
//   quadrature-point stage runs there, and the transposed sweeps return the
//   test-function contributions to the thread's x-line of nodes, which are
//   scattered into the output with hardware float atomics (or plain
//   read-modify-write inside one colour of cells).
#pragma once

#include "common.hpp"

namespace mfh {

enum { POL_R = 0, POL_CF = 1, POL_C2 = 2, POL_C4 = 3 };

// Symmetric second-order tensors in Voigt order: (00, 11, 22, 01, 02, 12) in
// 3-D, (00, 11, 01) in 2-D; a symmetric Voigt matrix is stored as its upper
// triangle, row by row.
template <int DIM>
struct Voigt {
  static constexpr int N = DIM * (DIM + 1) / 2;
  static constexpr int NSYM = N * (N + 1) / 2;
  __device__ static constexpr int row(int a) { return DIM == 3 ? (a < 3 ? a : (a == 5 ? 1 : 0)) : (a < 2 ? a : 0); }
  __device__ static constexpr int col(int a) { return DIM == 3 ? (a < 3 ? a : (a == 3 ? 1 : 2)) : (a < 2 ? a : 1); }
  __device__ static constexpr int of(int i, int j) {   // Voigt index of (i, j)
    return i == j ? i : (DIM == 2 ? 2 : (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)));
  }
  __device__ static constexpr int packed(int a, int b) {   // upper-triangle slot of (a, b)
    return a <= b ? a * N - a * (a - 1) / 2 + (b - a) : b * N - b * (b - 1) / 2 + (a - b);
  }
};

// Cache words per quadrature point.
template <int DIM, int POL>
struct CacheWords {
  static constexpr int value = POL == POL_CF ? DIM * DIM
                              : POL == POL_C2 ? DIM * DIM + 1
                              : POL == POL_C4 ? DIM * DIM + DIM * (DIM + 1) / 2 + Voigt<DIM>::NSYM
                              : 0;
};

template <int DIM, int N1>
struct Geo {
  static constexpr int NP = DIM == 3 ? N1 * N1 : N1;   // pencils per cell
  static constexpr int NV = NP * N1;                   // points per cell
  // cells per block: as many as the block's threads hold, except where the
  // FP64 LDS footprint (DIM * NARR * NV * CPB doubles) would let fewer blocks
  // reside on a CU (160 KB of LDS): 3-D Q2 takes 27 (52.5 KB, three blocks
  // instead of two), 3-D Q4 takes 8 (72 KB, two blocks instead of one); this
  // measured 6-10 % (Q2) and 23-25 % (Q4) faster FP64 vmults at equal FP32 ones.
  static constexpr int CPB = DIM == 3 && N1 == 3 ? 27 : DIM == 3 && N1 == 5 ? 8 : kBlock / NP;
  static constexpr int NARR = DIM == 3 ? 3 : 2;        // LDS arrays per component
};

// Cells per block of the tangent vmult's pencil kernels, two variants that
// the tuned table chooses between per level: V = 0 the length above; V = 1 a
// second one (about half, so two-wave blocks; 3-D Q4 the full 10 cells that
// 256 threads hold).  The element scatter's node-sum kernel must be launched
// with the same variant, as it locates the cell-block ends.
template <int DIM, int N1, int V>
struct CellBlock {
  static constexpr int NP = Geo<DIM, N1>::NP;
  static constexpr int value = V == 0 ? Geo<DIM, N1>::CPB : DIM == 3 && N1 == 5 ? 10 : DIM == 3 && N1 == 3 ? 14
                                                                                               : kBlock / NP / 2;
  static constexpr int threads = (value * NP + 63) / 64 * 64;
  static_assert(value * NP <= kBlock, "a cell block fits the block's threads");
};

// LDS words (of T) of the tangent kernels' block: the sweeps' DIM * NARR
// arrays of NV points per cell, also used for the element-buffer handover.
template <int DIM, int N1, typename T, int CPB = Geo<DIM, N1>::CPB>
struct TangentLdsSize {
  static constexpr int value = DIM * Geo<DIM, N1>::NARR * Geo<DIM, N1>::NV * CPB;
};

// Element buffer of the ELEMENT scatter for a level of `cells` cells (T words,
// each array cell-fastest, so that a block's cells store and load coalesced):
//   [0, DIM * NX * cells): component c, slot s = x + P * line at
//     (c * NX + s) * cells + e, for the x-nodes x = 0..P-1 of each x-line
//     (line = y + N1 * z in cell-local node indices);
//   then the overflow part, (c * NP + line) * cells + e: the sums of the last
//     x-node (x = P) of the cells that could not hand them to their
//     x-neighbour (last cell of a block, cells on the x = 1 face).
// Together DIM * NV * cells words, the size of one value per cell node.
template <int DIM, int N1>
struct ElemLayout {
  static constexpr int NP = Geo<DIM, N1>::NP;
  static constexpr int NX = (N1 - 1) * NP;
};

// Even-odd form of the 1-D products.  The support and Gauss points are
// symmetric about the cell centre, so S and S^T are centro-symmetric
// (M[n-1-r][n-1-c] = M[r][c]) and D and D^T skew (= -M[r][c]).  A line v is
// folded into e[c] = v[c] + v[n-1-c], o[c] = v[c] - v[n-1-c] (c < h = n/2)
// and, for odd n, its middle value vm; products are accumulated as P and Q
// with y[r] = P[r] + Q[r], y[n-1-r] = P[r] - Q[r] (r < h), y[h] = P[h]: a
// symmetric M adds its even half times e and its middle column times vm to
// P and its odd half times o to Q, a skew M its odd half times o to P and its
// even half times e and middle column times vm to Q.  At n = 5 one product
// takes 13 (symmetric) or 12 (skew) multiply-adds instead of 25, plus four
// additions to fold each input line and four to unfold each output line,
// shared by the products of a sweep.
template <int N1, typename T>
struct EvenOdd {
  static constexpr int H = N1 / 2, NPQ = H + (N1 & 1);
  struct Fold {
    T e[H], o[H], m;
  };
  struct Acc {
    T P[NPQ], Q[H];
    __device__ Acc() {
#pragma unroll
      for (int r = 0; r < NPQ; ++r) P[r] = 0;
#pragma unroll
      for (int r = 0; r < H; ++r) Q[r] = 0;
    }
  };
  __device__ static __forceinline__ Fold fold(const T (&v)[N1]) {
    Fold f;
#pragma unroll
    for (int c = 0; c < H; ++c) {
      f.e[c] = v[c] + v[N1 - 1 - c];
      f.o[c] = v[c] - v[N1 - 1 - c];
    }
    f.m = (N1 & 1) ? v[H] : T(0);
    return f;
  }
  // acc += M v for M = S, D, S^T, D^T (M = 0..3; 1 and 3 are skew)
  template <int M>
  __device__ static __forceinline__ void add(Acc& acc, const Fold& f, const Tables<T>& tb) {
    constexpr bool skew = M & 1;
#pragma unroll
    for (int r = 0; r < NPQ; ++r)
#pragma unroll
      for (int c = 0; c < H; ++c) acc.P[r] += tb.eo[M][skew ? 1 : 0][r][c] * (skew ? f.o[c] : f.e[c]);
#pragma unroll
    for (int r = 0; r < H; ++r)
#pragma unroll
      for (int c = 0; c < H; ++c) acc.Q[r] += tb.eo[M][skew ? 0 : 1][r][c] * (skew ? f.e[c] : f.o[c]);
    if constexpr (N1 & 1) {
      if constexpr (skew) {
#pragma unroll
        for (int r = 0; r < H; ++r) acc.Q[r] += tb.mid[M][r] * f.m;
      } else {
#pragma unroll
        for (int r = 0; r < NPQ; ++r) acc.P[r] += tb.mid[M][r] * f.m;
      }
    }
  }
  __device__ static __forceinline__ void unfold(const Acc& acc, T (&y)[N1]) {
#pragma unroll
    for (int r = 0; r < H; ++r) {
      y[r] = acc.P[r] + acc.Q[r];
      y[N1 - 1 - r] = acc.P[r] - acc.Q[r];
    }
    if constexpr (N1 & 1) y[H] = acc.P[H];
  }
};

// Sum-factorisation sweeps over the LDS of a block of NCELL cells (the
// pencil kernels' cells per block by default; the tile kernel's tile).  In
// 3-D from n = 4 the sweeps take the even-odd form (EvenOdd): measured
// 3-11 % faster vmults at Q4 and 2-8 % at Q3 (except Q3 FP64 with cached
// F^-1, within noise), no gain at Q2, where a product of 9 multiply-adds
// becomes 7 or 6 plus the folds.
template <int DIM, int N1, typename T, int NCELL = Geo<DIM, N1>::CPB>
struct SumFact {
  static constexpr int NV = Geo<DIM, N1>::NV, CPB = NCELL;
  static constexpr bool kEO = DIM == 3 && N1 >= 4;
  using EO = EvenOdd<N1, T>;

  __device__ static __forceinline__ int pt(int x, int y, int z) { return x + N1 * (y + N1 * z); }
  __device__ static __forceinline__ T& at(T* lds, int arr, int p, int cl) {
    return lds[(arr * NV + p) * CPB + cl];
  }

  // Nodal values v[c][a] on the thread's x-line -> reference gradients
  // g[c][I][q] (I = derivative direction) at the Gauss points of the thread's
  // final line (3-D: z-line (qx,qy) = (pen%n, pen/n); 2-D: y-line qx = pen).
  template <int NC>
  __device__ static void forward(const T (&v)[NC][N1], T (&g)[NC][DIM][N1], T* lds,
                                 int pen, int cl, bool act, const Tables<T>& tb) {
    if constexpr (kEO) {
      forward_eo<NC>(v, g, lds, pen, cl, act, tb);
    } else if constexpr (DIM == 3) {
      const int p0 = pen % N1, p1 = pen / N1;
      if (act) {   // x-sweep: line (b, c) = (p0, p1)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            T s = 0, d = 0;
#pragma unroll
            for (int a = 0; a < N1; ++a) {
              s += tb.S[q][a] * v[c][a];
              d += tb.D[q][a] * v[c][a];
            }
            at(lds, 3 * c + 0, pt(q, p0, p1), cl) = s;
            at(lds, 3 * c + 1, pt(q, p0, p1), cl) = d;
          }
      }
      __syncthreads();
      if (act) {   // y-sweep: line (qx, c) = (p0, p1)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T s[N1], d[N1];
#pragma unroll
          for (int b = 0; b < N1; ++b) {
            s[b] = at(lds, 3 * c + 0, pt(p0, b, p1), cl);
            d[b] = at(lds, 3 * c + 1, pt(p0, b, p1), cl);
          }
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            T ss = 0, sd = 0, ds = 0;
#pragma unroll
            for (int b = 0; b < N1; ++b) {
              ss += tb.S[q][b] * s[b];
              sd += tb.D[q][b] * s[b];
              ds += tb.S[q][b] * d[b];
            }
            at(lds, 3 * c + 0, pt(p0, q, p1), cl) = ss;   // S_y S_x
            at(lds, 3 * c + 1, pt(p0, q, p1), cl) = sd;   // D_y S_x
            at(lds, 3 * c + 2, pt(p0, q, p1), cl) = ds;   // S_y D_x
          }
        }
      }
      __syncthreads();
      if (act) {   // z-sweep: line (qx, qy) = (p0, p1)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T ss[N1], sd[N1], ds[N1];
#pragma unroll
          for (int k = 0; k < N1; ++k) {
            ss[k] = at(lds, 3 * c + 0, pt(p0, p1, k), cl);
            sd[k] = at(lds, 3 * c + 1, pt(p0, p1, k), cl);
            ds[k] = at(lds, 3 * c + 2, pt(p0, p1, k), cl);
          }
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            T gx = 0, gy = 0, gz = 0;
#pragma unroll
            for (int k = 0; k < N1; ++k) {
              gx += tb.S[q][k] * ds[k];
              gy += tb.S[q][k] * sd[k];
              gz += tb.D[q][k] * ss[k];
            }
            g[c][0][q] = gx;
            g[c][1][q] = gy;
            g[c][2][q] = gz;
          }
        }
      }
      __syncthreads();
    } else {
      const int b = pen;
      if (act) {   // x-sweep: line b
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            T s = 0, d = 0;
#pragma unroll
            for (int a = 0; a < N1; ++a) {
              s += tb.S[q][a] * v[c][a];
              d += tb.D[q][a] * v[c][a];
            }
            at(lds, 2 * c + 0, pt(q, b, 0), cl) = s;
            at(lds, 2 * c + 1, pt(q, b, 0), cl) = d;
          }
      }
      __syncthreads();
      if (act) {   // y-sweep: line qx = pen
        const int qx = pen;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T s[N1], d[N1];
#pragma unroll
          for (int j = 0; j < N1; ++j) {
            s[j] = at(lds, 2 * c + 0, pt(qx, j, 0), cl);
            d[j] = at(lds, 2 * c + 1, pt(qx, j, 0), cl);
          }
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            T gx = 0, gy = 0;
#pragma unroll
            for (int j = 0; j < N1; ++j) {
              gx += tb.S[q][j] * d[j];
              gy += tb.D[q][j] * s[j];
            }
            g[c][0][q] = gx;
            g[c][1][q] = gy;
          }
        }
      }
      __syncthreads();
    }
  }

  // Transposed sweeps: quadrature values P[c][I][q] on the thread's final line
  // (weights already applied) -> out[c][a] = sum_q sum_I dphi_a/dxi_I(q) P[c][I][q]
  // on the thread's x-line of nodes.
  template <int NC>
  __device__ static void backward(const T (&P)[NC][DIM][N1], T (&out)[NC][N1], T* lds,
                                  int pen, int cl, bool act, const Tables<T>& tb) {
    if constexpr (kEO) {
      backward_eo<NC>(P, out, lds, pen, cl, act, tb);
    } else if constexpr (DIM == 3) {
      const int p0 = pen % N1, p1 = pen / N1;
      if (act) {   // z: line (qx, qy)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int k = 0; k < N1; ++k) {
            T z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
            for (int q = 0; q < N1; ++q) {
              z0 += tb.S[q][k] * P[c][0][q];
              z1 += tb.S[q][k] * P[c][1][q];
              z2 += tb.D[q][k] * P[c][2][q];
            }
            at(lds, 3 * c + 0, pt(p0, p1, k), cl) = z0;
            at(lds, 3 * c + 1, pt(p0, p1, k), cl) = z1;
            at(lds, 3 * c + 2, pt(p0, p1, k), cl) = z2;
          }
      }
      __syncthreads();
      if (act) {   // y: line (qx, c)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T z0[N1], z1[N1], z2[N1];
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            z0[q] = at(lds, 3 * c + 0, pt(p0, q, p1), cl);
            z1[q] = at(lds, 3 * c + 1, pt(p0, q, p1), cl);
            z2[q] = at(lds, 3 * c + 2, pt(p0, q, p1), cl);
          }
#pragma unroll
          for (int b = 0; b < N1; ++b) {
            T yd = 0, ys = 0;
#pragma unroll
            for (int q = 0; q < N1; ++q) {
              yd += tb.S[q][b] * z0[q];
              ys += tb.D[q][b] * z1[q] + tb.S[q][b] * z2[q];
            }
            at(lds, 3 * c + 0, pt(p0, b, p1), cl) = yd;   // still needs D_x
            at(lds, 3 * c + 1, pt(p0, b, p1), cl) = ys;   // still needs S_x
          }
        }
      }
      __syncthreads();
      if (act) {   // x: line (b, c)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T yd[N1], ys[N1];
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            yd[q] = at(lds, 3 * c + 0, pt(q, p0, p1), cl);
            ys[q] = at(lds, 3 * c + 1, pt(q, p0, p1), cl);
          }
#pragma unroll
          for (int a = 0; a < N1; ++a) {
            T s = 0;
#pragma unroll
            for (int q = 0; q < N1; ++q) s += tb.D[q][a] * yd[q] + tb.S[q][a] * ys[q];
            out[c][a] = s;
          }
        }
      }
      __syncthreads();
    } else {
      if (act) {   // y: line qx = pen
        const int qx = pen;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int j = 0; j < N1; ++j) {
            T yd = 0, ys = 0;
#pragma unroll
            for (int q = 0; q < N1; ++q) {
              yd += tb.S[q][j] * P[c][0][q];
              ys += tb.D[q][j] * P[c][1][q];
            }
            at(lds, 2 * c + 0, pt(qx, j, 0), cl) = yd;
            at(lds, 2 * c + 1, pt(qx, j, 0), cl) = ys;
          }
      }
      __syncthreads();
      if (act) {   // x: line b = pen
        const int b = pen;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T yd[N1], ys[N1];
#pragma unroll
          for (int q = 0; q < N1; ++q) {
            yd[q] = at(lds, 2 * c + 0, pt(q, b, 0), cl);
            ys[q] = at(lds, 2 * c + 1, pt(q, b, 0), cl);
          }
#pragma unroll
          for (int a = 0; a < N1; ++a) {
            T s = 0;
#pragma unroll
            for (int q = 0; q < N1; ++q) s += tb.D[q][a] * yd[q] + tb.S[q][a] * ys[q];
            out[c][a] = s;
          }
        }
      }
      __syncthreads();
    }
  }

  // 3-D sweeps in the even-odd form: the same products, stages and LDS
  // traffic as the direct form above.
  template <int NC>
  __device__ static void forward_eo(const T (&v)[NC][N1], T (&g)[NC][DIM][N1], T* lds,
                                    int pen, int cl, bool act, const Tables<T>& tb) {
    const int p0 = pen % N1, p1 = pen / N1;
    if (act) {   // x-sweep: line (b, c) = (p0, p1)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const typename EO::Fold f = EO::fold(v[c]);
        typename EO::Acc as, ad;
        EO::template add<0>(as, f, tb);
        EO::template add<1>(ad, f, tb);
        T s[N1], d[N1];
        EO::unfold(as, s);
        EO::unfold(ad, d);
#pragma unroll
        for (int q = 0; q < N1; ++q) {
          at(lds, 3 * c + 0, pt(q, p0, p1), cl) = s[q];
          at(lds, 3 * c + 1, pt(q, p0, p1), cl) = d[q];
        }
      }
    }
    __syncthreads();
    if (act) {   // y-sweep: line (qx, c) = (p0, p1)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T s[N1], d[N1];
#pragma unroll
        for (int b = 0; b < N1; ++b) {
          s[b] = at(lds, 3 * c + 0, pt(p0, b, p1), cl);
          d[b] = at(lds, 3 * c + 1, pt(p0, b, p1), cl);
        }
        const typename EO::Fold fs = EO::fold(s), fd = EO::fold(d);
        typename EO::Acc ass, asd, ads;
        EO::template add<0>(ass, fs, tb);   // S_y S_x
        EO::template add<1>(asd, fs, tb);   // D_y S_x
        EO::template add<0>(ads, fd, tb);   // S_y D_x
        T ss[N1], sd[N1], ds[N1];
        EO::unfold(ass, ss);
        EO::unfold(asd, sd);
        EO::unfold(ads, ds);
#pragma unroll
        for (int q = 0; q < N1; ++q) {
          at(lds, 3 * c + 0, pt(p0, q, p1), cl) = ss[q];
          at(lds, 3 * c + 1, pt(p0, q, p1), cl) = sd[q];
          at(lds, 3 * c + 2, pt(p0, q, p1), cl) = ds[q];
        }
      }
    }
    __syncthreads();
    if (act) {   // z-sweep: line (qx, qy) = (p0, p1)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T ss[N1], sd[N1], ds[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          ss[k] = at(lds, 3 * c + 0, pt(p0, p1, k), cl);
          sd[k] = at(lds, 3 * c + 1, pt(p0, p1, k), cl);
          ds[k] = at(lds, 3 * c + 2, pt(p0, p1, k), cl);
        }
        const typename EO::Fold fss = EO::fold(ss), fsd = EO::fold(sd), fds = EO::fold(ds);
        typename EO::Acc ax, ay, az;
        EO::template add<0>(ax, fds, tb);
        EO::template add<0>(ay, fsd, tb);
        EO::template add<1>(az, fss, tb);
        EO::unfold(ax, g[c][0]);
        EO::unfold(ay, g[c][1]);
        EO::unfold(az, g[c][2]);
      }
    }
    __syncthreads();
  }

  template <int NC>
  __device__ static void backward_eo(const T (&P)[NC][DIM][N1], T (&out)[NC][N1], T* lds,
                                     int pen, int cl, bool act, const Tables<T>& tb) {
    const int p0 = pen % N1, p1 = pen / N1;
    if (act) {   // z: line (qx, qy)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const typename EO::Fold f0 = EO::fold(P[c][0]), f1 = EO::fold(P[c][1]), f2 = EO::fold(P[c][2]);
        typename EO::Acc a0, a1, a2;
        EO::template add<2>(a0, f0, tb);
        EO::template add<2>(a1, f1, tb);
        EO::template add<3>(a2, f2, tb);
        T z0[N1], z1[N1], z2[N1];
        EO::unfold(a0, z0);
        EO::unfold(a1, z1);
        EO::unfold(a2, z2);
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          at(lds, 3 * c + 0, pt(p0, p1, k), cl) = z0[k];
          at(lds, 3 * c + 1, pt(p0, p1, k), cl) = z1[k];
          at(lds, 3 * c + 2, pt(p0, p1, k), cl) = z2[k];
        }
      }
    }
    __syncthreads();
    if (act) {   // y: line (qx, c)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T z0[N1], z1[N1], z2[N1];
#pragma unroll
        for (int q = 0; q < N1; ++q) {
          z0[q] = at(lds, 3 * c + 0, pt(p0, q, p1), cl);
          z1[q] = at(lds, 3 * c + 1, pt(p0, q, p1), cl);
          z2[q] = at(lds, 3 * c + 2, pt(p0, q, p1), cl);
        }
        const typename EO::Fold f0 = EO::fold(z0), f1 = EO::fold(z1), f2 = EO::fold(z2);
        typename EO::Acc ad, as;
        EO::template add<2>(ad, f0, tb);   // still needs D_x
        EO::template add<3>(as, f1, tb);   // still needs S_x
        EO::template add<2>(as, f2, tb);
        T yd[N1], ys[N1];
        EO::unfold(ad, yd);
        EO::unfold(as, ys);
#pragma unroll
        for (int b = 0; b < N1; ++b) {
          at(lds, 3 * c + 0, pt(p0, b, p1), cl) = yd[b];
          at(lds, 3 * c + 1, pt(p0, b, p1), cl) = ys[b];
        }
      }
    }
    __syncthreads();
    if (act) {   // x: line (b, c)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T yd[N1], ys[N1];
#pragma unroll
        for (int q = 0; q < N1; ++q) {
          yd[q] = at(lds, 3 * c + 0, pt(q, p0, p1), cl);
          ys[q] = at(lds, 3 * c + 1, pt(q, p0, p1), cl);
        }
        const typename EO::Fold fd = EO::fold(yd), fs = EO::fold(ys);
        typename EO::Acc a;
        EO::template add<3>(a, fd, tb);
        EO::template add<2>(a, fs, tb);
        EO::unfold(a, out[c]);
      }
    }
    __syncthreads();
  }
};

// ---------------------------------------------------------------------------
// Per-thread cell geometry.
template <int DIM, int N1>
struct CellPos {
  long long e;          // linear cell index on the level
  int i0, j0, k0;       // lattice origin of the thread's x-line of nodes
  unsigned fjk;         // faces touched by the line's (j, k)
  bool first_i, last_i; // the cell touches x = 0 / x = 1
  long long base;       // node index of the line's first node

  template <typename T>
  __device__ void init(const CellArgs<T>& a, long long lin, int pen) {
    constexpr int P = N1 - 1;
    int ex, ey, ez;
    if (a.color < 0) {   // cells of a level < 2^32 (lattice of at most 1600^3 nodes)
      e = lin;
      const unsigned ul = (unsigned)lin, un = (unsigned)a.N;
      const unsigned r = ul / un;
      ex = (int)(ul - r * un);
      const unsigned r2 = r / un;
      ey = (int)(r - r2 * un);
      ez = (int)r2;
    } else {
      const int cx = a.color & 1, cy = (a.color >> 1) & 1, cz = (a.color >> 2) & 1;
      const int nx = (a.N - cx + 1) / 2, ny = (a.N - cy + 1) / 2;
      const int ix = (int)(lin % nx);
      const long long r = lin / nx;
      const int iy = (int)(r % ny), iz = (int)(r / ny);
      ex = 2 * ix + cx;
      ey = 2 * iy + cy;
      ez = DIM == 3 ? 2 * iz + cz : 0;
      e = ex + (long long)a.N * (ey + (long long)a.N * ez);
    }
    const int b = DIM == 3 ? pen % N1 : pen;
    const int c = DIM == 3 ? pen / N1 : 0;
    i0 = ex * P;
    j0 = ey * P + b;
    k0 = DIM == 3 ? ez * P + c : 0;
    fjk = node_faces(1, j0, k0, a.L, DIM);     // i = 1 is never a face node
    first_i = (ex == 0);
    last_i = (ex == a.N - 1);
    base = i0 + (long long)a.L * (j0 + (long long)a.L * k0);
  }

  __device__ __forceinline__ unsigned faces(int a_, int L) const {
    unsigned f = fjk;
    if (a_ == 0 && first_i) f |= 1u;
    if (a_ == N1 - 1 && last_i) f |= 2u;
    return f;
  }
};

template <int DIM, int N1, typename T>
__device__ __forceinline__ void gather(const T* __restrict__ src, const CellArgs<T>& a,
                                       const CellPos<DIM, N1>& cp, bool act, bool masked,
                                       T (&v)[DIM][N1]) {
  // all loads first (inactive lanes read the valid line of cell 0), then the masking,
  // so that the loads of every component are in flight together
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < N1; ++k) v[c][k] = src[c * a.nn + cp.base + k];
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const bool zero = !act || (masked && a.mask_in && (cp.faces(k, a.L) & a.fmask[c]));
      v[c][k] = zero ? T(0) : v[c][k];
    }
}

template <int DIM, int N1, typename T>
__device__ __forceinline__ void scatter(T* __restrict__ dst, const CellArgs<T>& a,
                                        const CellPos<DIM, N1>& cp, bool act,
                                        const T (&v)[DIM][N1]) {
  if (!act) return;
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      if (cp.faces(k, a.L) & a.fmask[c]) continue;
      T* p = dst + c * a.nn + cp.base + k;
      if (a.color < 0)
        atomic_add(p, v[c][k]);
      else
        *p += v[c][k];
    }
}

// Atomic scatter that leaves the last x-node to the next lane (skip_last).
template <int DIM, int N1, typename T>
__device__ __forceinline__ void scatter_merged(T* __restrict__ dst, const CellArgs<T>& a,
                                               const CellPos<DIM, N1>& cp, bool act, const T (&v)[DIM][N1],
                                               bool skip_last) {
  if (!act) return;
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      if (k == N1 - 1 && skip_last) continue;
      if (cp.faces(k, a.L) & a.fmask[c]) continue;
      atomic_add(dst + c * a.nn + cp.base + k, v[c][k]);
    }
}

// ---------------------------------------------------------------------------
// Quadrature-point algebra (Sec. 2.3).  All gradients are physical (1/h
// applied).  Referential route used by the device:
//   F = I + Grad u, J = det F, c1 = mu - 2 lambda ln J,
//   S = mu I - c1 C^-1   (C^-1 = F^-1 F^-T),
//   g = Grad x F^-1 (spatial gradient of the trial field),
//   sigma = 2 c1 sym(g) + 2 lambda tr(g) I        (J c : sym g, Sec. 2.3)
//   P_x = sigma F^-T + Grad x S                    (tangent, eq. tangent
//                                                   pulled back: g tau F^-T = Grad x S)
//       = mu Grad x + (c1 g^T + 2 lambda tr(g) I) F^-T   (evaluated form, no S)
// and the residual stress P = mu F - c1 F^-T (= tau F^-T with tau = mu b - c1 I).

template <typename T> __device__ __forceinline__ T log1p_t(T x);
template <> __device__ __forceinline__ double log1p_t<double>(double x) { return log1p(x); }
template <> __device__ __forceinline__ float log1p_t<float>(float x) { return log1pf(x); }

// J - 1 of F = I + H without cancellation: tr H + second invariant + det H.
template <int DIM, typename T>
__device__ __forceinline__ T det_minus_one(const T (&H)[DIM][DIM]) {
  if constexpr (DIM == 3) {
    const T tr = H[0][0] + H[1][1] + H[2][2];
    const T i2 = H[0][0] * H[1][1] - H[0][1] * H[1][0] + H[0][0] * H[2][2] - H[0][2] * H[2][0]
               + H[1][1] * H[2][2] - H[1][2] * H[2][1];
    const T dt = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1])
               - H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0])
               + H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
    return tr + i2 + dt;
  } else {
    return H[0][0] + H[1][1] + (H[0][0] * H[1][1] - H[0][1] * H[1][0]);
  }
}

// F = I + H; returns J and writes F^-1 (Fi[I][j]).
template <int DIM, typename T>
__device__ __forceinline__ T kinematics(const T (&H)[DIM][DIM], T (&F)[DIM][DIM], T (&Fi)[DIM][DIM], T& jm1) {
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) F[i][j] = H[i][j] + (i == j ? T(1) : T(0));
  jm1 = det_minus_one<DIM, T>(H);
  const T J = T(1) + jm1;
  const T r = T(1) / J;
  if constexpr (DIM == 3) {
    Fi[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * r;
    Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * r;
    Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * r;
    Fi[1][0] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * r;
    Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * r;
    Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * r;
    Fi[2][0] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * r;
    Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * r;
    Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * r;
  } else {
    Fi[0][0] = F[1][1] * r;
    Fi[0][1] = -F[0][1] * r;
    Fi[1][0] = -F[1][0] * r;
    Fi[1][1] = F[0][0] * r;
  }
  return J;
}

// Tangent action at one quadrature point for the Neo-Hookean law:
// Hx (Grad x) -> P_x * wt, in place.  With g = Grad x F^-1 and
// S = mu I - c1 C^-1 the geometric part is Grad x S = mu Grad x - c1 g F^-T,
// so that P_x = sigma F^-T + Grad x S collapses to
//   P_x = mu Grad x + (c1 g^T + 2 lambda tr(g) I) F^-T
// (2 c1 sym g - c1 g = c1 g^T): the stress is never formed, and the cached
// policies need only F^-1 and c1 besides the material's (mu, lambda).
template <int DIM, typename T>
__device__ __forceinline__ void tangent_qp(T (&Hx)[DIM][DIM], const T (&Fi)[DIM][DIM], T c1, T mu, T lam, T wt) {
  T g[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T s = 0;
#pragma unroll
      for (int I = 0; I < DIM; ++I) s += Hx[i][I] * Fi[I][j];
      g[i][j] = s;
    }
  T tr = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) tr += g[i][i];
  const T l2t = T(2) * lam * tr;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int I = 0; I < DIM; ++I) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s += g[j][i] * Fi[I][j];
      Hx[i][I] = (mu * Hx[i][I] + c1 * s + l2t * Fi[I][i]) * wt;
    }
}

// ---------------------------------------------------------------------------
// General route (any law; Algorithm 3 of Sec. 5 and the setup kernels of the
// Mooney-Rivlin law).  The compressible Mooney-Rivlin energy
//   psi = mu/2 [I1 - 3 - 2 ln J] + mu2/2 [I2 - 3 - 4 ln J] + lambda ln^2 J
// is the Neo-Hookean law of Sec. 2.3 for mu2 = 0.  Its stresses:
//   S = mu (I - C^-1) + mu2 (I1 I - C - 2 C^-1) + 2 lambda ln J C^-1,
// and the material part of the spatial tangent (J times the push-forward of
// 4 d2psi/dC2):
//   J c = 2 c1' Ssym + 2 lambda I (x) I + 2 mu2 (b (x) b - I_b),
//   c1' = mu + 2 mu2 - 2 lambda ln J,  (I_b)_ijkl = 1/2 (b_ik b_jl + b_il b_jk).
// I1 and I2 are invariants of the 3-D tensors (plane strain: C_33 = 1).

// S of the general law from F, F^-1 and J - 1 (FP64).
template <int DIM, typename T>
__device__ __forceinline__ void mr_stress(const T (&F)[DIM][DIM], const T (&Fi)[DIM][DIM], T jm1, T mu, T mu2, T lam,
                                          T (&S)[DIM][DIM]) {
  T C[DIM][DIM], Ci[DIM][DIM];
#pragma unroll
  for (int I = 0; I < DIM; ++I)
#pragma unroll
    for (int J = 0; J < DIM; ++J) {
      T c = 0, ci = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        c += F[k][I] * F[k][J];
        ci += Fi[I][k] * Fi[J][k];
      }
      C[I][J] = c;
      Ci[I][J] = ci;
    }
  T I1 = T(3 - DIM);
#pragma unroll
  for (int I = 0; I < DIM; ++I) I1 += C[I][I];
  const T l2 = T(2) * lam * log1p_t<T>(jm1);
#pragma unroll
  for (int I = 0; I < DIM; ++I)
#pragma unroll
    for (int J = 0; J < DIM; ++J) {
      const T d = I == J ? T(1) : T(0);
      S[I][J] = mu * (d - Ci[I][J]) + mu2 * (I1 * d - C[I][J] - T(2) * Ci[I][J]) + l2 * Ci[I][J];
    }
}

// J c of the general law in packed Voigt form (see Voigt).
template <int DIM, typename T>
__device__ __forceinline__ void mr_spatial_tangent(const T (&F)[DIM][DIM], T jm1, T mu, T mu2, T lam,
                                                   T (&Cv)[Voigt<DIM>::NSYM]) {
  using V = Voigt<DIM>;
  T b[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T s = 0;
#pragma unroll
      for (int K = 0; K < DIM; ++K) s += F[i][K] * F[j][K];
      b[i][j] = s;
    }
  const T c1p = mu + T(2) * mu2 - T(2) * lam * log1p_t<T>(jm1);
#pragma unroll
  for (int A = 0; A < V::N; ++A)
#pragma unroll
    for (int B = A; B < V::N; ++B) {
      const int i = V::row(A), j = V::col(A), k = V::row(B), l = V::col(B);
      const T dik = i == k ? T(1) : T(0), djl = j == l ? T(1) : T(0);
      const T dil = i == l ? T(1) : T(0), djk = j == k ? T(1) : T(0);
      const T dij = i == j ? T(1) : T(0), dkl = k == l ? T(1) : T(0);
      Cv[V::packed(A, B)] = c1p * (dik * djl + dil * djk) + T(2) * lam * dij * dkl +
                            mu2 * (T(2) * b[i][j] * b[k][l] - b[i][k] * b[j][l] - b[i][l] * b[j][k]);
    }
}

// Per-lane arrays at a wave-uniform base (caches, element buffer): with O32
// the lane's offset is a 32-bit byte count, so the loads and stores take the
// base from scalar registers and need no 64-bit address arithmetic per
// access; the launcher picks O32 when every offset of the level fits, also
// those of arrays of T pairs (NV * cells * 2 * sizeof(T) < 2^32), else the
// 64-bit form.
template <bool O32, typename T>
__device__ __forceinline__ T lane_load(const T* ubase, long long lane, unsigned lane_bytes) {
  if constexpr (O32)
    return *(const T*)((const char*)ubase + lane_bytes);
  else
    return ubase[lane];
}
template <bool O32, typename T>
__device__ __forceinline__ void lane_store(T* ubase, long long lane, unsigned lane_bytes, T v) {
  if constexpr (O32)
    *(T*)((char*)ubase + lane_bytes) = v;
  else
    ubase[lane] = v;
}

// cache_T2 data of a quadrature point: F^-1 (row-major) and c1.  In 3-D the
// ten words are five pairs (words 2k, 2k+1): pair k of the point with element
// index `at` (qp * cells + e) is element k * stride + at of the cache read as
// an array of T pairs (stride = NV * cells), one 16-byte load per pair in
// FP64.  In 2-D word w is element w * stride + at of the plain array.
template <typename T> struct Vec2Of;
template <> struct Vec2Of<double> { using type = double2; };
template <> struct Vec2Of<float> { using type = float2; };

// Reader: `base` is the wave-uniform part of `at`, `lane` the per-lane part.
template <int DIM, typename T, bool O32>
__device__ __forceinline__ void c2_load(const T* __restrict__ cache, long long base, long long stride, long long lane,
                                        T (&Fi)[DIM][DIM], T& c1) {
  if constexpr (DIM == 3) {
    using V2 = typename Vec2Of<T>::type;
    const V2* pb = reinterpret_cast<const V2*>(cache) + base;
    const unsigned lb = O32 ? (unsigned)lane * (unsigned)sizeof(V2) : 0u;
    T wv[10];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const V2 v = lane_load<O32>(pb + k * stride, lane, lb);
      wv[2 * k] = v.x;
      wv[2 * k + 1] = v.y;
    }
#pragma unroll
    for (int I = 0; I < 3; ++I)
#pragma unroll
      for (int j = 0; j < 3; ++j) Fi[I][j] = wv[3 * I + j];
    c1 = wv[9];
  } else {
    const T* wb = cache + base;
    const unsigned lb = O32 ? (unsigned)lane * (unsigned)sizeof(T) : 0u;
#pragma unroll
    for (int I = 0; I < DIM; ++I)
#pragma unroll
      for (int j = 0; j < DIM; ++j) Fi[I][j] = lane_load<O32>(wb + (I * DIM + j) * stride, lane, lb);
    c1 = lane_load<O32>(wb + DIM * DIM * stride, lane, lb);
  }
}

// Writer (from the FP64 quadrature-point data, rounded to T).
template <int DIM, typename T>
__device__ __forceinline__ void c2_store(T* __restrict__ cache, long long at, long long stride,
                                         const double (&Fi)[DIM][DIM], double c1) {
  if constexpr (DIM == 3) {
    using V2 = typename Vec2Of<T>::type;
    V2* pb = reinterpret_cast<V2*>(cache) + at;
    const double wv[10] = {Fi[0][0], Fi[0][1], Fi[0][2], Fi[1][0], Fi[1][1], Fi[1][2], Fi[2][0], Fi[2][1], Fi[2][2], c1};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      V2 v;
      v.x = (T)wv[2 * k];
      v.y = (T)wv[2 * k + 1];
      pb[k * stride] = v;
    }
  } else {
#pragma unroll
    for (int I = 0; I < DIM; ++I)
#pragma unroll
      for (int j = 0; j < DIM; ++j) cache[(I * DIM + j) * stride + at] = (T)Fi[I][j];
    cache[DIM * DIM * stride + at] = (T)c1;
  }
}

// Tangent action with a cached general tangent (Algorithm 3, referential
// form): g = Grad x F^-1, sigma = J c : sym g, P_x = sigma F^-T + Grad x S.
// Hx (Grad x) -> P_x * wt, in place.  Word w of this quadrature point's C4
// cache (F^-1, S upper triangle, J c packed Voigt) is lane element `lane` of
// the array at qb + w * stride; J c is streamed word by word into the
// symmetric product so that only sym g and sigma stay live.  The law enters
// only through the cached data.
template <int DIM, typename T, bool O32>
__device__ __forceinline__ void tangent_qp_c4(T (&Hx)[DIM][DIM], const T* __restrict__ qb, long long stride,
                                              long long lane, unsigned lane_bytes, T wt) {
  using V = Voigt<DIM>;
  T Fi[DIM][DIM];
#pragma unroll
  for (int I = 0; I < DIM; ++I)
#pragma unroll
    for (int j = 0; j < DIM; ++j) Fi[I][j] = lane_load<O32>(qb + (I * DIM + j) * stride, lane, lane_bytes);
  T gam[V::N];   // sym g in Voigt form, shear entries doubled
#pragma unroll
  for (int A = 0; A < V::N; ++A) {
    const int i = V::row(A), j = V::col(A);
    T gij = 0, gji = 0;
#pragma unroll
    for (int I = 0; I < DIM; ++I) {
      gij += Hx[i][I] * Fi[I][j];
      gji += Hx[j][I] * Fi[I][i];
    }
    gam[A] = i == j ? gij : gij + gji;
  }
  const T* cv = qb + (DIM * DIM + V::N) * stride;
  T sv[V::N] = {};
#pragma unroll
  for (int A = 0; A < V::N; ++A)
#pragma unroll
    for (int B = A; B < V::N; ++B) {
      const T c = lane_load<O32>(cv + V::packed(A, B) * stride, lane, lane_bytes);
      sv[A] += c * gam[B];
      if (B != A) sv[B] += c * gam[A];
    }
  T sig[DIM][DIM];
#pragma unroll
  for (int A = 0; A < V::N; ++A) {
    sig[V::row(A)][V::col(A)] = sv[A];
    sig[V::col(A)][V::row(A)] = sv[A];
  }
  T S[DIM][DIM];
  {
    int w = DIM * DIM;
#pragma unroll
    for (int I = 0; I < DIM; ++I)
#pragma unroll
      for (int J = I; J < DIM; ++J) {
        const T v = lane_load<O32>(qb + (w++) * stride, lane, lane_bytes);
        S[I][J] = v;
        S[J][I] = v;
      }
  }
  T P[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int I = 0; I < DIM; ++I) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s += sig[i][j] * Fi[I][j];
#pragma unroll
      for (int J = 0; J < DIM; ++J) s += Hx[i][J] * S[J][I];
      P[i][I] = s;
    }
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int I = 0; I < DIM; ++I) Hx[i][I] = P[i][I] * wt;
}

// arr[i] for a thread-dependent i by compare-and-select over the N1 entries:
// indexing a kernel-argument array with a runtime index makes the compiler
// copy the whole argument block to scratch memory first.
template <int N1, typename T>
__device__ __forceinline__ T pick(const T (&arr)[kMaxN1], int i) {
  T v = arr[0];
#pragma unroll
  for (int k = 1; k < N1; ++k) v = (i == k) ? arr[k] : v;
  return v;
}

template <int DIM, int N1, typename T>
__device__ __forceinline__ T qp_weight(const Tables<T>& tb, int p0, int p1, int q) {
  if constexpr (DIM == 3)
    return pick<N1>(tb.w, p0) * pick<N1>(tb.w, p1) * tb.w[q];
  else
    return pick<N1>(tb.w, p0) * tb.w[q];
}

template <int DIM, int N1>
__device__ __forceinline__ int qp_index(int p0, int p1, int q) {
  return DIM == 3 ? p0 + N1 * (p1 + N1 * q) : p0 + N1 * q;
}

template <typename T>
__device__ __forceinline__ int material_of(const CellArgs<T>& a, long long e, int qp) {
  return (a.matbits[e * a.nwords + (qp >> 5)] >> (qp & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// Tangent vmult body for cell block `blk` of one level: y += K x over the
// block's cells (y pre-filled).  Shared by the single-problem kernel and the
// batched work-list kernel.
template <int DIM, int P, typename T, int POL, bool O32, int CPB = Geo<DIM, P + 1>::CPB>
__device__ __forceinline__ void tangent_block(const CellArgs<T>& a, const T* __restrict__ x, T* __restrict__ y,
                                              long long blk, T* lds) {
  constexpr int N1 = P + 1;
  using G = Geo<DIM, N1>;
  using SF = SumFact<DIM, N1, T, CPB>;
  constexpr int NW = CacheWords<DIM, POL>::value;

  const int t = threadIdx.x;
  const int cl = t % CPB, pen = t / CPB;
  const long long lin = blk * CPB + cl;
  const bool act = pen < G::NP && lin < a.nlaunch;
  CellPos<DIM, N1> cp;
  cp.init(a, act ? lin : 0, act ? pen : 0);
  const int p0 = DIM == 3 ? pen % N1 : pen;
  const int p1 = DIM == 3 ? pen / N1 : 0;

  T gx[DIM][DIM][N1];
  {
    T v[DIM][N1];
    gather<DIM, N1, T>(x, a, cp, act, true, v);
    SF::template forward<DIM>(v, gx, lds, pen, cl, act, a.tb);
  }
  T gu[DIM][DIM][N1];
  if constexpr (POL == POL_R) {
    T v[DIM][N1];
    gather<DIM, N1, T>(a.u, a, cp, act, false, v);
    SF::template forward<DIM>(v, gu, lds, pen, cl, act, a.tb);
  }

  // cache word w of quadrature point (p0, p1, q): lane element qp(p0, p1, 0) *
  // cells + e of the array at cache + (w * NV + q * NP) * cells
  const long long lane_c = (long long)qp_index<DIM, N1>(p0, p1, 0) * a.ncells + cp.e;
  const unsigned lane_cb = O32 ? (unsigned)lane_c * (unsigned)sizeof(T) : 0u;
  const long long wstride = (long long)G::NV * a.ncells;
  if (act) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      const int qp = qp_index<DIM, N1>(p0, p1, q);
      const int mid = material_of(a, cp.e, qp);
      const T* qb = a.cache + (long long)q * G::NP * a.ncells;
      const T mu = mid ? a.mu[1] : a.mu[0];
      const T lam = mid ? a.lam[1] : a.lam[0];
      // the action is linear in Grad x: the 1/h of the trial gradient joins the weight
      const T wt = qp_weight<DIM, N1, T>(a.tb, p0, p1, q) * a.wscale * a.invh;
      T Hx[DIM][DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) Hx[i][I] = gx[i][I][q];
      if constexpr (POL == POL_C4) {
        tangent_qp_c4<DIM, T, O32>(Hx, qb, wstride, lane_c, lane_cb, wt);
      } else {
        T Fi[DIM][DIM], c1;
        if constexpr (POL == POL_R || POL == POL_CF) {
          T H[DIM][DIM];
          if constexpr (POL == POL_R) {
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int I = 0; I < DIM; ++I) H[i][I] = gu[i][I][q] * a.invh;
          } else {
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int I = 0; I < DIM; ++I)
                H[i][I] = lane_load<O32>(qb + (i * DIM + I) * wstride, lane_c, lane_cb) - (i == I ? T(1) : T(0));
          }
          T F[DIM][DIM], jm1;
          kinematics<DIM, T>(H, F, Fi, jm1);
          c1 = mu - T(2) * lam * log1p_t<T>(jm1);
        } else {
          c2_load<DIM, T, O32>(a.cache, (long long)q * G::NP * a.ncells, wstride, lane_c, Fi, c1);
        }
        tangent_qp<DIM, T>(Hx, Fi, c1, mu, lam, wt);
      }
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) gx[i][I][q] = Hx[i][I];
    }
  }
  (void)NW;

  T out[DIM][N1];
  SF::template backward<DIM>(gx, out, lds, pen, cl, act, a.tb);
  if (a.elem != nullptr) {
    // Element buffer (layout at ElemLayout): x-nodes 0..P-1 of every line, one
    // coalesced store per (component, node) across the block's cells.  The
    // last x-node of a line is the first one of the x-neighbour's line: when
    // that neighbour is the next cell of this block, its thread adds the sums
    // (through LDS, free after the transposed sweeps' last barrier); otherwise
    // (block end, x = 1 face) they go to the overflow part.
    using EL = ElemLayout<DIM, N1>;
    const int line = DIM == 3 ? p0 + N1 * p1 : p0;
    if (act) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) lds[(c * G::NP + line) * CPB + cl] = out[c][N1 - 1];
    }
    __syncthreads();
    if (act) {
      if (cl > 0 && !cp.first_i) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c][0] += lds[(c * G::NP + line) * CPB + cl - 1];
      }
      const long long lane_e = (long long)(P * line) * a.ncells + cp.e;
      const unsigned lane_eb = O32 ? (unsigned)lane_e * (unsigned)sizeof(T) : 0u;
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int k = 0; k < P; ++k)
          lane_store<O32>(a.elem + ((long long)c * EL::NX + k) * a.ncells, lane_e, lane_eb, out[c][k]);
      if (cl + 1 == CPB || cp.last_i || lin + 1 >= a.nlaunch) {
        const long long lane_o = (long long)line * a.ncells + cp.e;
        const unsigned lane_ob = O32 ? (unsigned)lane_o * (unsigned)sizeof(T) : 0u;
#pragma unroll
        for (int c = 0; c < DIM; ++c)
          lane_store<O32>(a.elem + ((long long)DIM * EL::NX + c * G::NP) * a.ncells, lane_o, lane_ob, out[c][N1 - 1]);
      }
    }
  } else if (a.color < 0) {
    // The x-neighbour of this cell (same pencil) sits in the previous lane when
    // both are in one wave: its last x-node is this cell's first one.  Pass it
    // over and let one lane add the sum, saving a third of the atomics.
    const int lane = t & 63;
    const bool from_prev = act && cl > 0 && lane > 0 && !cp.first_i;
    const bool to_next = act && cl + 1 < CPB && lane < 63 && lin + 1 < a.nlaunch && !cp.last_i;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const T v = __shfl_up(out[c][N1 - 1], 1);
      if (from_prev) out[c][0] += v;
    }
    scatter_merged<DIM, N1, T>(y, a, cp, act, out, to_next);
  } else {
    scatter<DIM, N1, T>(y, a, cp, act, out);
  }
}

// Second pass of the ELEMENT scatter: y at every node is the sum of the
// element-buffer entries (ElemLayout) of the cells containing it, in a fixed
// order; constrained entries take x (mask_in = 1) or 0.  Along x a node has
// one entry: the slot of the cell it starts (x-node 0..P-1), which for a node
// shared by cells q - 1 and q already holds both cells' sums, unless cell
// q - 1 ended its cell block (then its share sits in the overflow part, a
// second entry); the node on the x = 1 face reads the overflow of cell N - 1.
// Along y and z, one or two cells each.  One thread per node of an (i, j)
// plane and all its components (the loads are in flight together);
// blockIdx.y is the plane k.  j = t / L comes from a multiply-high by
// magic = ceil(2^32 / L), exact for t < L^2 while L^3 < 2^32.
template <int DIM, int P, typename T, typename Out, int CPB = Geo<DIM, P + 1>::CPB>
__device__ __forceinline__ void elem_gather_node(const CellArgs<T>& a, const T* __restrict__ x, const Out& out,
                                                 int t, int k, unsigned magic) {
  constexpr int N1 = P + 1;
  using EL = ElemLayout<DIM, N1>;
  const int N = a.N, L = a.L;
  if (t >= L * L) return;
  const int j = (int)__umulhi((unsigned)t, magic);
  const int i = t - j * L;
  const unsigned fc = node_faces(i, j, k, L, DIM);
  int ce[3][2], cn[3][2], m[3];
  const int idx[3] = {i, j, k};
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    if (d >= DIM) {
      ce[d][0] = ce[d][1] = 0;
      cn[d][0] = cn[d][1] = 0;
      m[d] = 1;
      continue;
    }
    const int q = idx[d] / P, rem = idx[d] - q * P;
    const bool inner = rem != 0;
    const bool has_lo = !inner && q > 0, has_hi = inner || q < N;
    ce[d][0] = has_lo ? q - 1 : q;
    cn[d][0] = has_lo ? P : rem;
    ce[d][1] = q;
    cn[d][1] = 0;
    m[d] = (has_lo && has_hi) ? 2 : 1;
  }
  const int qx = i / P, rx = i - qx * P;
  const bool last = qx == N;                    // i = L - 1
  const int ex0 = last ? N - 1 : qx;
  const bool shared = rx == 0 && qx > 0 && qx < N;
  // the entries of every component: loads first, then the sums
  T v[DIM][DIM == 3 ? 8 : 4];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T* eb = a.elem + (long long)c * EL::NX * a.ncells;
    const T* ob = a.elem + ((long long)DIM * EL::NX + (long long)c * EL::NP) * a.ncells;
#pragma unroll
    for (int zz = 0; zz < (DIM == 3 ? 2 : 1); ++zz)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        const int s = yy + 2 * zz;
        const bool on = yy < m[1] && zz < m[2];
        const int eyz = N * (ce[1][yy] + N * ce[2][zz]);
        const int line = cn[1][yy] + N1 * cn[2][zz];
        const int e0 = ex0 + eyz, e1 = qx - 1 + eyz;
        const bool on1 = on && shared && (unsigned)e1 % (unsigned)CPB == (unsigned)(CPB - 1);
        const long long i0 = (long long)(last ? line : rx + P * line) * a.ncells + e0;
        // only the entries that exist are loaded (the others read as zero, so
        // the fixed summation order below is kept)
        T v0 = T(0), v1 = T(0);
        if (on) v0 = (last ? ob : eb)[i0];
        if (on1) v1 = ob[(long long)line * a.ncells + e1];
        v[c][2 * s] = v0;
        v[c][2 * s + 1] = v1;
      }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const long long gi = c * a.nn + t + (long long)L * L * k;
    T acc = 0;
#pragma unroll
    for (int s = 0; s < (DIM == 3 ? 8 : 4); ++s) acc += v[c][s];
    if (fc & a.fmask[c]) acc = a.mask_in ? x[gi] : T(0);
    out(gi, acc);
  }
}

template <int DIM, int P, typename T, int CPB>
__global__ void __launch_bounds__(kBlock) k_elem_gather(CellArgs<T> arg, unsigned magic) {
  const CellArgs<T>& a = kernel_args(arg);
  elem_gather_node<DIM, P, T, StoreOut<T>, CPB>(a, a.x, StoreOut<T>{a.y}, blockIdx.x * kBlock + threadIdx.x,
                                                 blockIdx.y, magic);
}

// Node sums fused with one Chebyshev step (the smoother's vmult on a level
// with the ELEMENT scatter).
template <int DIM, int P, typename T, int CPB>
__global__ void __launch_bounds__(kBlock) k_elem_gather_cheb(CellArgs<T> arg, unsigned magic, ChebOut<T> out) {
  const CellArgs<T>& a = kernel_args(arg);
  elem_gather_node<DIM, P, T, ChebOut<T>, CPB>(a, a.x, out, blockIdx.x * kBlock + threadIdx.x, blockIdx.y, magic);
}

// Batched second pass: one workgroup per item (problem, plane k, block of the
// plane) of the problems that use the ELEMENT scatter.

template <int DIM, int P, typename T>
__global__ void __launch_bounds__(kBlock) k_elem_gather_batch(const CellArgs<T>* __restrict__ args,
                                                              const GatherItem* __restrict__ items,
                                                              const T* const* __restrict__ xs,
                                                              T* const* __restrict__ ys) {
  using CArgs = const CellArgs<T> __attribute__((address_space(4)));
  using CInt = const int __attribute__((address_space(4)));
  using CPtrX = const T* const __attribute__((address_space(4)));
  using CPtrY = T* const __attribute__((address_space(4)));
  const CInt* it = (CInt*)(items + blockIdx.x);
  const int p = it[0], k = it[1], blk = it[2];
  const unsigned magic = (unsigned)it[3];
  const CellArgs<T>& a = *(const CellArgs<T>*)((CArgs*)args + p);
  elem_gather_node<DIM, P, T>(a, ((CPtrX*)xs)[p], StoreOut<T>{((CPtrY*)ys)[p]}, blk * kBlock + threadIdx.x, k, magic);
}

// Tangent vmult: y += K x over the cells of this launch (y pre-filled).
template <int DIM, int P, typename T, int POL, bool O32, int CPB>
__global__ void __launch_bounds__(kBlock) k_tangent(CellArgs<T> arg) {
  __shared__ T lds[TangentLdsSize<DIM, P + 1, T, CPB>::value];
  const CellArgs<T>& a = kernel_args(arg);
  const long long blk = a.color < 0 ? xcd_block(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
  tangent_block<DIM, P, T, POL, O32, CPB>(a, a.x, a.y, blk, lds);
}

// Batched tangent vmult over many independent problems of one degree: one
// workgroup per (problem, cell block) item of the bin's work list, item i
// being cell block item[i].y of problem item[i].x.  The item index is
// XCD-aware (neighbouring cell blocks of a problem share an L2) and
// wave-uniform, so the item and the problem's arguments come in through
// scalar loads; the block body is the single-problem one.
template <int DIM, int P, typename T, int POL, bool O32>
__global__ void __launch_bounds__(kBlock) k_tangent_batch(const CellArgs<T>* __restrict__ args,
                                                          const int2* __restrict__ items,
                                                          const T* const* __restrict__ xs, T* const* __restrict__ ys) {
  __shared__ T lds[TangentLdsSize<DIM, P + 1, T>::value];
  // The tables are read through the constant address space, where
  // wave-uniform addresses become scalar loads; the arguments are used in
  // place (no private copy), as kernel arguments are.
  using CArgs = const CellArgs<T> __attribute__((address_space(4)));
  using CInt = const int __attribute__((address_space(4)));
  using CPtrX = const T* const __attribute__((address_space(4)));
  using CPtrY = T* const __attribute__((address_space(4)));
  const long long i = xcd_block(blockIdx.x, gridDim.x);
  const int p = ((CInt*)items)[2 * i];
  const int blk = ((CInt*)items)[2 * i + 1];
  const CellArgs<T>& a = *(const CellArgs<T>*)((CArgs*)args + p);
  tangent_block<DIM, P, T, POL, O32>(a, ((CPtrX*)xs)[p], ((CPtrY*)ys)[p], blk, lds);
}

// ---------------------------------------------------------------------------
// Tile variant of the tangent vmult (atomic scatter).  One block owns a tile of
// TX x TY x TZ cells (2-D: TX x TY).  The tile's lattice nodes are loaded once,
// coalesced, into LDS; each (cell, pencil) thread reads its x-line from there,
// runs the same sweeps and quadrature-point stage as k_tangent, and adds its
// results into an LDS copy of the tile's nodes (ds_add).  Nodes inside the
// tile, or on a tile face that is the domain boundary, receive all their
// contributions from this block and are written with plain stores; nodes on a
// face shared with a neighbouring tile are added with global atomics.  Compared
// with one atomic per cell node this divides the global atomics by ~3 for
// Q2 tiles of 4x4x2 and replaces the per-cell gathers with one coalesced
// load per tile node.
template <int DIM, int P, int TX, int TY, int TZ>
struct TileGeo {
  static constexpr int N1 = P + 1;
  static constexpr int NP = DIM == 3 ? N1 * N1 : N1;
  static constexpr int NCELL = TX * TY * (DIM == 3 ? TZ : 1);
  static constexpr int ACTIVE = NCELL * NP;
  static constexpr int BLOCK = (ACTIVE + 63) / 64 * 64;
  static constexpr int GX = TX * P + 1, GY = TY * P + 1, GZ = DIM == 3 ? TZ * P + 1 : 1;
  static constexpr int NG = GX * GY * GZ;
  static constexpr int NV = NP * N1;
};

// Tile origin and extent of block b.
template <int DIM, int TX, int TY, int TZ>
struct TilePos {
  int cx0, cy0, cz0;    // first cell of the tile
  int ex, ey, ez;       // cells of the tile inside the domain along each axis
  __device__ void init(long long b, int N) {
    const int ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY;
    const int tx = (int)(b % ntx);
    const long long r = b / ntx;
    const int ty = (int)(r % nty);
    const int tz = DIM == 3 ? (int)(r / nty) : 0;
    cx0 = tx * TX;
    cy0 = ty * TY;
    cz0 = tz * TZ;
    ex = min(TX, N - cx0);
    ey = min(TY, N - cy0);
    ez = DIM == 3 ? min(TZ, N - cz0) : 1;
  }
};

template <int DIM, int P, typename T, int POL, int TX, int TY, int TZ, int NC>
__global__ void __launch_bounds__((TileGeo<DIM, P, TX, TY, TZ>::BLOCK))
k_tangent_tile(CellArgs<T> a) {
  using TG = TileGeo<DIM, P, TX, TY, TZ>;
  constexpr int N1 = P + 1, NCELL = TG::NCELL, NG = TG::NG, GX = TG::GX, GY = TG::GY;
  constexpr int NARR = DIM == 3 ? 3 : 2;
  using SF = SumFact<DIM, N1, T, NCELL>;
  __shared__ T xs[DIM * NG];                                   // x tile, then y accumulator
  __shared__ T us[POL == POL_R ? DIM * NG : 1];                // displacement tile (recompute)
  __shared__ T sf[NC * NARR * TG::NV * NCELL];

  const int t = threadIdx.x;
  const long long nb = gridDim.x;
  TilePos<DIM, TX, TY, TZ> tp;
  tp.init(xcd_block(blockIdx.x, nb), a.N);
  const int L = a.L;

  // 1. tile nodes -> LDS (x masked on constrained DoFs)
  for (int idx = t; idx < DIM * NG; idx += TG::BLOCK) {
    const int c = idx / NG, g = idx - c * NG;
    const int gi = g % GX, gj = (g / GX) % GY, gk = DIM == 3 ? g / (GX * GY) : 0;
    const int I = tp.cx0 * P + gi, J = tp.cy0 * P + gj, K = tp.cz0 * P + gk;
    T xv = 0, uv = 0;
    if (I < L && J < L && (DIM == 2 || K < L)) {
      const long long node = I + (long long)L * (J + (long long)L * K);
      xv = a.x[c * a.nn + node];
      if (a.mask_in && (node_faces(I, J, K, L, DIM) & a.fmask[c])) xv = 0;
      if constexpr (POL == POL_R) uv = a.u[c * a.nn + node];
    }
    xs[idx] = xv;
    if constexpr (POL == POL_R) us[idx] = uv;
  }
  __syncthreads();

  // 2. per (cell, pencil) thread
  const int cl = t % NCELL, pen = t / NCELL;
  const int lx = cl % TX, ly = (cl / TX) % TY, lz = DIM == 3 ? cl / (TX * TY) : 0;
  const bool act = pen < TG::NP && lx < tp.ex && ly < tp.ey && lz < tp.ez;
  const int pb = DIM == 3 ? pen % N1 : pen, pc = DIM == 3 ? pen / N1 : 0;
  const int p0 = pb, p1 = pc;
  const int g0 = lx * P + GX * ((ly * P + pb) + GY * (lz * P + pc));   // tile node of the line's first node
  const long long e = (tp.cx0 + lx) + (long long)a.N * ((tp.cy0 + ly) + (long long)a.N * (tp.cz0 + lz));

  T gx[DIM][DIM][N1];
  T gu[POL == POL_R ? DIM : 1][DIM][N1];
  if constexpr (POL == POL_R) {
#pragma unroll
    for (int c0 = 0; c0 < DIM; c0 += NC) {
      T v[NC][N1];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < N1; ++k) v[c][k] = act ? us[(c0 + c) * NG + g0 + k] : T(0);
      SF::template forward<NC>(v, reinterpret_cast<T(&)[NC][DIM][N1]>(gu[c0]), sf, pen, cl, act, a.tb);
    }
  }
#pragma unroll
  for (int c0 = 0; c0 < DIM; c0 += NC) {
    T v[NC][N1];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int k = 0; k < N1; ++k) v[c][k] = act ? xs[(c0 + c) * NG + g0 + k] : T(0);
    SF::template forward<NC>(v, reinterpret_cast<T(&)[NC][DIM][N1]>(gx[c0]), sf, pen, cl, act, a.tb);
  }
  // x is consumed: the tile buffer becomes the accumulator
  for (int idx = t; idx < DIM * NG; idx += TG::BLOCK) xs[idx] = T(0);

  if (act) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      const int qp = qp_index<DIM, N1>(p0, p1, q);
      const int mid = material_of(a, e, qp);
      const T mu = mid ? a.mu[1] : a.mu[0];
      const T lam = mid ? a.lam[1] : a.lam[0];
      const T wt = qp_weight<DIM, N1, T>(a.tb, p0, p1, q) * a.wscale;
      T Hx[DIM][DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) Hx[i][I] = gx[i][I][q] * a.invh;
      if constexpr (POL == POL_C4) {
        tangent_qp_c4<DIM, T, false>(Hx, a.cache, (long long)TG::NV * a.ncells, (long long)qp * a.ncells + e, 0u, wt);
      } else {
        T Fi[DIM][DIM], c1;
        if constexpr (POL == POL_R || POL == POL_CF) {
          T H[DIM][DIM];
          if constexpr (POL == POL_R) {
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int I = 0; I < DIM; ++I) H[i][I] = gu[i][I][q] * a.invh;
          } else {
            const T* cq = a.cache + (long long)qp * a.ncells + e;
            const long long stride = (long long)TG::NV * a.ncells;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int I = 0; I < DIM; ++I) H[i][I] = cq[(i * DIM + I) * stride] - (i == I ? T(1) : T(0));
          }
          T F[DIM][DIM], jm1;
          kinematics<DIM, T>(H, F, Fi, jm1);
          c1 = mu - T(2) * lam * log1p_t<T>(jm1);
        } else {
          c2_load<DIM, T, false>(a.cache, 0, (long long)TG::NV * a.ncells, (long long)qp * a.ncells + e, Fi, c1);
        }
        tangent_qp<DIM, T>(Hx, Fi, c1, mu, lam, wt);
      }
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) gx[i][I][q] = Hx[i][I];
    }
  }

#pragma unroll
  for (int c0 = 0; c0 < DIM; c0 += NC) {
    T out[NC][N1];
    SF::template backward<NC>(reinterpret_cast<const T(&)[NC][DIM][N1]>(gx[c0]), out, sf, pen, cl, act, a.tb);
    if (act) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < N1; ++k) atomicAdd(&xs[(c0 + c) * NG + g0 + k], out[c][k]);
    }
  }
  __syncthreads();

  // 3. tile nodes -> global: exclusive nodes stored, shared tile faces added atomically
  for (int idx = t; idx < DIM * NG; idx += TG::BLOCK) {
    const int c = idx / NG, g = idx - c * NG;
    const int gi = g % GX, gj = (g / GX) % GY, gk = DIM == 3 ? g / (GX * GY) : 0;
    const int I = tp.cx0 * P + gi, J = tp.cy0 * P + gj, K = tp.cz0 * P + gk;
    if (!(I < L && J < L && (DIM == 2 || K < L))) continue;
    if (node_faces(I, J, K, L, DIM) & a.fmask[c]) continue;
    const bool shx = (gi == 0 && I != 0) || (gi == tp.ex * P && I != L - 1);
    const bool shy = (gj == 0 && J != 0) || (gj == tp.ey * P && J != L - 1);
    const bool shz = DIM == 3 && ((gk == 0 && K != 0) || (gk == tp.ez * P && K != L - 1));
    const long long node = I + (long long)L * (J + (long long)L * K);
    T* p = a.y + c * a.nn + node;
    if (shx || shy || shz)
      atomic_add(p, xs[idx]);
    else
      *p = xs[idx];
  }
}

// Residual of the weak form: y += sum_q w P(F) : Grad N (FP64).
template <int DIM, int P>
__global__ void __launch_bounds__(kBlock) k_residual(CellArgs<double> arg) {
  const CellArgs<double>& a = kernel_args(arg);
  using T = double;
  constexpr int N1 = P + 1;
  using G = Geo<DIM, N1>;
  using SF = SumFact<DIM, N1, T>;
  __shared__ T lds[DIM * G::NARR * G::NV * G::CPB];
  const int t = threadIdx.x;
  const int cl = t % G::CPB, pen = t / G::CPB;
  const long long blk = a.color < 0 ? xcd_block(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
  const long long lin = blk * G::CPB + cl;
  const bool act = pen < G::NP && lin < a.nlaunch;
  CellPos<DIM, N1> cp;
  cp.init(a, act ? lin : 0, act ? pen : 0);
  const int p0 = DIM == 3 ? pen % N1 : pen;
  const int p1 = DIM == 3 ? pen / N1 : 0;

  T gu[DIM][DIM][N1];
  {
    T v[DIM][N1];
    gather<DIM, N1, T>(a.u, a, cp, act, false, v);
    SF::template forward<DIM>(v, gu, lds, pen, cl, act, a.tb);
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      const int qp = qp_index<DIM, N1>(p0, p1, q);
      const int mid = material_of(a, cp.e, qp);
      const T mu = mid ? a.mu[1] : a.mu[0];
      const T lam = mid ? a.lam[1] : a.lam[0];
      const T wt = qp_weight<DIM, N1, T>(a.tb, p0, p1, q) * a.wscale;
      T H[DIM][DIM], F[DIM][DIM], Fi[DIM][DIM], jm1;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) H[i][I] = gu[i][I][q] * a.invh;
      kinematics<DIM, T>(H, F, Fi, jm1);
      if (a.law) {   // general law: P = F S
        const T mu2 = mid ? a.mu2[1] : a.mu2[0];
        T S[DIM][DIM];
        mr_stress<DIM, T>(F, Fi, jm1, mu, mu2, lam, S);
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int I = 0; I < DIM; ++I) {
            T v = 0;
#pragma unroll
            for (int J = 0; J < DIM; ++J) v += F[i][J] * S[J][I];
            gu[i][I][q] = v * wt;
          }
      } else {
        const T c1 = mu - T(2) * lam * log1p_t<T>(jm1);
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int I = 0; I < DIM; ++I) gu[i][I][q] = (mu * F[i][I] - c1 * Fi[I][i]) * wt;
      }
    }
  }
  T out[DIM][N1];
  SF::template backward<DIM>(gu, out, lds, pen, cl, act, a.tb);
  scatter<DIM, N1, T>(a.y, a, cp, act, out);
}

// Quadrature data of a level: min J per block, and the policy cache
// (CF: F;  C2: F^-1, c1;  C4: F^-1, S (upper triangle, row major), J c of the
// general law in packed Voigt form) in precision T.
// The displacement is read in FP64 and everything is evaluated in FP64.
template <int DIM, int P, typename T, int POL>
__global__ void __launch_bounds__(kBlock) k_qpdata(CellArgs<double> arg, T* __restrict__ cache) {
  const CellArgs<double>& a = kernel_args(arg);
  using D = double;
  constexpr int N1 = P + 1;
  using G = Geo<DIM, N1>;
  using SF = SumFact<DIM, N1, D>;
  __shared__ D lds[DIM * G::NARR * G::NV * G::CPB];
  __shared__ D red[kBlock];
  const int t = threadIdx.x;
  const int cl = t % G::CPB, pen = t / G::CPB;
  const long long lin = (long long)blockIdx.x * G::CPB + cl;
  const bool act = pen < G::NP && lin < a.nlaunch;
  CellPos<DIM, N1> cp;
  cp.init(a, act ? lin : 0, act ? pen : 0);
  const int p0 = DIM == 3 ? pen % N1 : pen;
  const int p1 = DIM == 3 ? pen / N1 : 0;
  D gu[DIM][DIM][N1];
  {
    D v[DIM][N1];
    gather<DIM, N1, D>(a.u, a, cp, act, false, v);
    SF::template forward<DIM>(v, gu, lds, pen, cl, act, a.tb);
  }
  D jmin = 1e300;
  if (act) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      const int qp = qp_index<DIM, N1>(p0, p1, q);
      const int mid = material_of(a, cp.e, qp);
      const D mu = mid ? a.mu[1] : a.mu[0];
      const D lam = mid ? a.lam[1] : a.lam[0];
      D H[DIM][DIM], F[DIM][DIM], Fi[DIM][DIM], jm1;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int I = 0; I < DIM; ++I) H[i][I] = gu[i][I][q] * a.invh;
      const D J = kinematics<DIM, D>(H, F, Fi, jm1);
      jmin = J < jmin ? J : jmin;
      if constexpr (POL != POL_R) {
        T* cq = cache + (long long)qp * a.ncells + cp.e;
        const long long stride = (long long)G::NV * a.ncells;
        if constexpr (POL == POL_CF) {
#pragma unroll
          for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int I = 0; I < DIM; ++I) cq[(i * DIM + I) * stride] = (T)F[i][I];
        } else if constexpr (POL == POL_C4) {
          const D mu2 = mid ? a.mu2[1] : a.mu2[0];
          D S[DIM][DIM], Cv[Voigt<DIM>::NSYM];
          mr_stress<DIM, D>(F, Fi, jm1, mu, mu2, lam, S);
          mr_spatial_tangent<DIM, D>(F, jm1, mu, mu2, lam, Cv);
          int w = 0;
#pragma unroll
          for (int I = 0; I < DIM; ++I)
#pragma unroll
            for (int j = 0; j < DIM; ++j) cq[(w++) * stride] = (T)Fi[I][j];
#pragma unroll
          for (int I = 0; I < DIM; ++I)
#pragma unroll
            for (int J = I; J < DIM; ++J) cq[(w++) * stride] = (T)S[I][J];
#pragma unroll
          for (int k = 0; k < Voigt<DIM>::NSYM; ++k) cq[(w++) * stride] = (T)Cv[k];
        } else {
          const D c1 = mu - 2.0 * lam * log1p(jm1);
          c2_store<DIM, T>(cache, (long long)qp * a.ncells + cp.e, stride, Fi, c1);
        }
      }
    }
  }
  red[t] = jmin;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = red[t] < red[t + s] ? red[t] : red[t + s];
    __syncthreads();
  }
  if (t == 0) a.blockmin[blockIdx.x] = red[0];
}

// Operator diagonal (FP64).  For DoF (node a, component al) of a cell the
// tangent entry reduces, with v = F^-T Grad N_a, to
//   sum_q w_q |cell| [ (c1 + 2 lambda) v_al^2 + mu |Grad N_a|^2 ]
// (material part 2 c1 sym g : sym g + 2 lambda tr(g)^2 plus geometric part
// v . tau v with tau = mu b - c1 I).  One thread per (cell, node); the cell's
// displacement and per-qp data are staged in LDS.  LAW = 1: the general
// law, entry sum_q w_q |cell| [ v_j (J c)_(al j al l) v_l + Grad N_a . S Grad N_a ].
template <int DIM, int P, int LAW>
struct DiagShape {
  static constexpr int NV = DIM == 3 ? (P + 1) * (P + 1) * (P + 1) : (P + 1) * (P + 1);
  // F^-1, c1 + 2 lambda, mu;  LAW = 1: F^-1, S (upper triangle), J c (packed Voigt)
  static constexpr int NQD = LAW ? DIM * DIM + Voigt<DIM>::N + Voigt<DIM>::NSYM : DIM * DIM + 2;
  static constexpr int BYTES = NV * (DIM + NQD) * 8;   // LDS per cell
  static constexpr int CPB_LDS = (48 * 1024) / BYTES;
  static constexpr int CPB = LAW ? (CPB_LDS < kBlock / NV ? CPB_LDS : kBlock / NV) : kBlock / NV;
  static_assert(CPB >= 1, "one cell's quadrature data must fit in LDS");
};

template <int DIM, int P, int LAW>
__global__ void __launch_bounds__(kBlock) k_diag(CellArgs<double> a) {
  using D = double;
  using V = Voigt<DIM>;
  constexpr int N1 = P + 1;
  constexpr int NV = DiagShape<DIM, P, LAW>::NV;
  constexpr int CPB = DiagShape<DIM, P, LAW>::CPB;
  constexpr int NQD = DiagShape<DIM, P, LAW>::NQD;
  __shared__ D su[CPB][DIM][NV];
  __shared__ D sq[CPB][NV][NQD];
  const int t = threadIdx.x;
  const int cl = t / NV, loc = t % NV;
  const long long e = (long long)blockIdx.x * CPB + cl;
  const bool act = cl < CPB && e < a.ncells;
  int ex = 0, ey = 0, ez = 0;
  if (act) {
    ex = (int)(e % a.N);
    ey = (int)((e / a.N) % a.N);
    ez = DIM == 3 ? (int)(e / ((long long)a.N * a.N)) : 0;
  }
  const int ax = loc % N1, ay = (loc / N1) % N1, az = DIM == 3 ? loc / (N1 * N1) : 0;
  const int I = ex * P + ax, J = ey * P + ay, K = ez * P + az;
  const long long node = I + (long long)a.L * (J + (long long)a.L * K);
  if (act) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) su[cl][c][loc] = a.u[c * a.nn + node];
  }
  __syncthreads();
  if (act) {   // quadrature point qp = loc: Grad u by direct summation over the cell's nodes
    const int qx = ax, qy = ay, qz = az;
    D H[DIM][DIM] = {};
    for (int b = 0; b < NV; ++b) {
      const int bx = b % N1, by = (b / N1) % N1, bz = DIM == 3 ? b / (N1 * N1) : 0;
      D gr[DIM];
      if constexpr (DIM == 3) {
        gr[0] = a.tb.D[qx][bx] * a.tb.S[qy][by] * a.tb.S[qz][bz];
        gr[1] = a.tb.S[qx][bx] * a.tb.D[qy][by] * a.tb.S[qz][bz];
        gr[2] = a.tb.S[qx][bx] * a.tb.S[qy][by] * a.tb.D[qz][bz];
      } else {
        gr[0] = a.tb.D[qx][bx] * a.tb.S[qy][by];
        gr[1] = a.tb.S[qx][bx] * a.tb.D[qy][by];
      }
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int d = 0; d < DIM; ++d) H[c][d] += su[cl][c][b] * gr[d] * a.invh;
    }
    D F[DIM][DIM], Fi[DIM][DIM], jm1;
    kinematics<DIM, D>(H, F, Fi, jm1);
    const int mid = material_of(a, e, loc);
    const D mu = mid ? a.mu[1] : a.mu[0];
    const D lam = mid ? a.lam[1] : a.lam[0];
    int w = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) sq[cl][loc][w++] = Fi[i][j];
    if constexpr (LAW) {
      const D mu2 = mid ? a.mu2[1] : a.mu2[0];
      D S[DIM][DIM], Cv[V::NSYM];
      mr_stress<DIM, D>(F, Fi, jm1, mu, mu2, lam, S);
      mr_spatial_tangent<DIM, D>(F, jm1, mu, mu2, lam, Cv);
#pragma unroll
      for (int I = 0; I < DIM; ++I)
#pragma unroll
        for (int J = I; J < DIM; ++J) sq[cl][loc][w++] = S[I][J];
#pragma unroll
      for (int k = 0; k < V::NSYM; ++k) sq[cl][loc][w++] = Cv[k];
    } else {
      const D c1 = mu - 2.0 * lam * log1p(jm1);
      sq[cl][loc][w++] = c1 + 2.0 * lam;
      sq[cl][loc][w] = mu;
    }
  }
  __syncthreads();
  if (!act) return;
  D acc[DIM] = {};
  for (int q = 0; q < NV; ++q) {
    const int qx = q % N1, qy = (q / N1) % N1, qz = DIM == 3 ? q / (N1 * N1) : 0;
    D gr[DIM], wq;
    if constexpr (DIM == 3) {
      gr[0] = a.tb.D[qx][ax] * a.tb.S[qy][ay] * a.tb.S[qz][az] * a.invh;
      gr[1] = a.tb.S[qx][ax] * a.tb.D[qy][ay] * a.tb.S[qz][az] * a.invh;
      gr[2] = a.tb.S[qx][ax] * a.tb.S[qy][ay] * a.tb.D[qz][az] * a.invh;
      wq = a.tb.w[qx] * a.tb.w[qy] * a.tb.w[qz];
    } else {
      gr[0] = a.tb.D[qx][ax] * a.tb.S[qy][ay] * a.invh;
      gr[1] = a.tb.S[qx][ax] * a.tb.D[qy][ay] * a.invh;
      wq = a.tb.w[qx] * a.tb.w[qy];
    }
    wq *= a.wscale / a.invh;   // w_q h^d
    const D* s = sq[cl][q];
    if constexpr (LAW) {
      D v[DIM], geo = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        D t = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) t += gr[d] * s[d * DIM + j];
        v[j] = t;
      }
      const D* sS = s + DIM * DIM;
      const D* cv = sS + V::N;
#pragma unroll
      for (int I = 0; I < DIM; ++I)
#pragma unroll
        for (int J = 0; J < DIM; ++J) {
          const int lo = I < J ? I : J, hi = I < J ? J : I;
          geo += gr[I] * sS[lo * DIM - lo * (lo - 1) / 2 + (hi - lo)] * gr[J];
        }
#pragma unroll
      for (int al = 0; al < DIM; ++al) {
        D m = 0;
#pragma unroll
        for (int j = 0; j < DIM; ++j)
#pragma unroll
          for (int l = 0; l < DIM; ++l) m += v[j] * cv[V::packed(V::of(al, j), V::of(al, l))] * v[l];
        acc[al] += wq * (m + geo);
      }
    } else {
      D gg = 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) gg += gr[d] * gr[d];
#pragma unroll
      for (int al = 0; al < DIM; ++al) {
        D v = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) v += gr[d] * s[d * DIM + al];
        acc[al] += wq * (s[DIM * DIM] * v * v + s[DIM * DIM + 1] * gg);
      }
    }
  }
  const unsigned f = node_faces(I, J, K, a.L, DIM);
#pragma unroll
  for (int al = 0; al < DIM; ++al)
    if (!(f & a.fmask[al])) atomic_add(a.y + al * a.nn + node, acc[al]);
}

// Destination of assembled element-matrix entries: the dense coarse matrix
// over free DoFs, K[fi * nf + fj] with fi / fj the free indices of the two
// DoFs (fmap = -1 on constrained DoFs).
struct DenseSink {
  const int* fmap;
  long long nf;
  double* K;
  long long fi[3];
  template <int DIM>
  __device__ void begin(const CellArgs<double>& a, long long node, int, int, int) {
    for (int i = 0; i < DIM; ++i) fi[i] = fmap[i * a.nn + node];
  }
  template <int DIM>
  __device__ void add(const CellArgs<double>& a, long long nodeb, int, int, int, const double (&acc)[DIM][DIM]) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int fj = fmap[k * a.nn + nodeb];
      if (fj < 0) continue;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
        if (fi[i] >= 0) atomic_add(K + fi[i] * nf + fj, acc[i][k]);
    }
  }
};

// Destination for the CSR form of K_c.  Row (i, node a) of a free DoF holds
// the columns (k, node b) for every component k and every node b of the
// cells that contain a, component-major and lexicographic within a
// component; per axis the node range of those cells is [lo, lo + len), so the
// position of a column is computed, not searched.  Rows of constrained DoFs
// hold their diagonal only and are skipped here, as are constrained columns.
__device__ __forceinline__ void csr_axis_range(int I, int P, int L, int& lo, int& len) {
  if (I % P != 0) {
    lo = I - I % P;
    len = P + 1;
  } else {
    lo = I - P > 0 ? I - P : 0;
    len = (I + P < L - 1 ? I + P : L - 1) - lo + 1;
  }
}

struct CsrSink {
  const long long* row_ptr;
  double* val;
  int P;
  long long base[3];   // row start of (i, a); -1 for a constrained row
  int lo[3], len[3];
  long long blk;       // columns per component
  template <int DIM>
  __device__ void begin(const CellArgs<double>& a, long long node, int I, int J, int K) {
    const unsigned f = node_faces(I, J, K, a.L, DIM);
    csr_axis_range(I, P, a.L, lo[0], len[0]);
    csr_axis_range(J, P, a.L, lo[1], len[1]);
    lo[2] = 0;
    len[2] = 1;
    if (DIM == 3) csr_axis_range(K, P, a.L, lo[2], len[2]);
    blk = (long long)len[0] * len[1] * len[2];
    for (int i = 0; i < DIM; ++i) base[i] = (f & a.fmask[i]) ? -1 : row_ptr[i * a.nn + node];
  }
  template <int DIM>
  __device__ void add(const CellArgs<double>& a, long long, int Ib, int Jb, int Kb, const double (&acc)[DIM][DIM]) {
    const unsigned fb = node_faces(Ib, Jb, Kb, a.L, DIM);
    const long long off = ((long long)(Kb - lo[2]) * len[1] + (Jb - lo[1])) * len[0] + (Ib - lo[0]);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if (fb & a.fmask[k]) continue;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
        if (base[i] >= 0) atomic_add(val + base[i] + k * blk + off, acc[i][k]);
    }
  }
};

// Element tangent of one cell (FP64), one block per cell and one thread per
// cell node a, added into a Sink.  With v = F^-T Grad N (spatial gradient of a
// shape function) the tangent entry of eq. (algebraic_tangent) between DoFs
// (a, i) and (b, k) is, for this material law,
//   sum_q w_q |cell| [ c1 v_a,k v_b,i + 2 lambda v_a,i v_b,k + mu delta_ik Grad N_a . Grad N_b ]
// (material part with J c = 2 c1 Ssym + 2 lambda I (x) I, geometric part with
// tau = mu b - c1 I).  LAW = 1: the general law, entry
//   sum_q w_q |cell| [ v_a,j (J c)_ijkl v_b,l + delta_ik Grad N_a . S Grad N_b ].
template <int DIM, int P, typename Sink, int LAW>
__global__ void __launch_bounds__(kBlock) k_cell_matrix(CellArgs<double> a, Sink sink) {
  using D = double;
  using V = Voigt<DIM>;
  constexpr int N1 = P + 1;
  constexpr int NV = DIM == 3 ? N1 * N1 * N1 : N1 * N1;
  // F^-1, c1, 2 lambda, mu;  LAW = 1: F^-1, S (upper triangle), J c (packed Voigt)
  constexpr int NQD = LAW ? DIM * DIM + V::N + V::NSYM : DIM * DIM + 3;
  __shared__ D su[DIM][NV];
  __shared__ D sq[NV][NQD];
  const long long e = blockIdx.x;
  const int t = threadIdx.x;
  const bool act = t < NV;
  const int ex = (int)(e % a.N), ey = (int)((e / a.N) % a.N);
  const int ez = DIM == 3 ? (int)(e / ((long long)a.N * a.N)) : 0;
  const int ax = t % N1, ay = (t / N1) % N1, az = DIM == 3 ? t / (N1 * N1) : 0;
  const long long node = (ex * P + ax) + (long long)a.L * ((ey * P + ay) + (long long)a.L * (ez * P + az));
  if (act) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) su[c][t] = a.u[c * a.nn + node];
  }
  __syncthreads();
  if (act) {   // quadrature data at qp t
    D H[DIM][DIM] = {};
    for (int b = 0; b < NV; ++b) {
      const int bx = b % N1, by = (b / N1) % N1, bz = DIM == 3 ? b / (N1 * N1) : 0;
      D gr[DIM];
      if constexpr (DIM == 3) {
        gr[0] = a.tb.D[ax][bx] * a.tb.S[ay][by] * a.tb.S[az][bz];
        gr[1] = a.tb.S[ax][bx] * a.tb.D[ay][by] * a.tb.S[az][bz];
        gr[2] = a.tb.S[ax][bx] * a.tb.S[ay][by] * a.tb.D[az][bz];
      } else {
        gr[0] = a.tb.D[ax][bx] * a.tb.S[ay][by];
        gr[1] = a.tb.S[ax][bx] * a.tb.D[ay][by];
      }
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int d = 0; d < DIM; ++d) H[c][d] += su[c][b] * gr[d] * a.invh;
    }
    D F[DIM][DIM], Fi[DIM][DIM], jm1;
    kinematics<DIM, D>(H, F, Fi, jm1);
    const int mid = material_of(a, e, t);
    const D mu = mid ? a.mu[1] : a.mu[0];
    const D lam = mid ? a.lam[1] : a.lam[0];
    int w = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) sq[t][w++] = Fi[i][j];
    if constexpr (LAW) {
      const D mu2 = mid ? a.mu2[1] : a.mu2[0];
      D S[DIM][DIM], Cv[V::NSYM];
      mr_stress<DIM, D>(F, Fi, jm1, mu, mu2, lam, S);
      mr_spatial_tangent<DIM, D>(F, jm1, mu, mu2, lam, Cv);
#pragma unroll
      for (int I = 0; I < DIM; ++I)
#pragma unroll
        for (int J = I; J < DIM; ++J) sq[t][w++] = S[I][J];
#pragma unroll
      for (int k = 0; k < V::NSYM; ++k) sq[t][w++] = Cv[k];
    } else {
      sq[t][w++] = mu - 2.0 * lam * log1p(jm1);
      sq[t][w++] = 2.0 * lam;
      sq[t][w] = mu;
    }
  }
  __syncthreads();
  if (!act) return;
  sink.template begin<DIM>(a, node, ex * P + ax, ey * P + ay, ez * P + az);
  const D hd = a.wscale / a.invh;   // h^d
  for (int b = 0; b < NV; ++b) {
    const int bx = b % N1, by = (b / N1) % N1, bz = DIM == 3 ? b / (N1 * N1) : 0;
    D acc[DIM][DIM] = {};
    for (int q = 0; q < NV; ++q) {
      const int qx = q % N1, qy = (q / N1) % N1, qz = DIM == 3 ? q / (N1 * N1) : 0;
      D ga[DIM], gb[DIM], wq;
      if constexpr (DIM == 3) {
        ga[0] = a.tb.D[qx][ax] * a.tb.S[qy][ay] * a.tb.S[qz][az];
        ga[1] = a.tb.S[qx][ax] * a.tb.D[qy][ay] * a.tb.S[qz][az];
        ga[2] = a.tb.S[qx][ax] * a.tb.S[qy][ay] * a.tb.D[qz][az];
        gb[0] = a.tb.D[qx][bx] * a.tb.S[qy][by] * a.tb.S[qz][bz];
        gb[1] = a.tb.S[qx][bx] * a.tb.D[qy][by] * a.tb.S[qz][bz];
        gb[2] = a.tb.S[qx][bx] * a.tb.S[qy][by] * a.tb.D[qz][bz];
        wq = a.tb.w[qx] * a.tb.w[qy] * a.tb.w[qz] * hd;
      } else {
        ga[0] = a.tb.D[qx][ax] * a.tb.S[qy][ay];
        ga[1] = a.tb.S[qx][ax] * a.tb.D[qy][ay];
        gb[0] = a.tb.D[qx][bx] * a.tb.S[qy][by];
        gb[1] = a.tb.S[qx][bx] * a.tb.D[qy][by];
        wq = a.tb.w[qx] * a.tb.w[qy] * hd;
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        ga[d] *= a.invh;
        gb[d] *= a.invh;
      }
      const D* s = sq[q];
      D va[DIM], vb[DIM], gg = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        D sa = 0, sb = 0;
#pragma unroll
        for (int I = 0; I < DIM; ++I) {
          sa += ga[I] * s[I * DIM + j];
          sb += gb[I] * s[I * DIM + j];
        }
        va[j] = sa;
        vb[j] = sb;
        gg += ga[j] * gb[j];
      }
      if constexpr (LAW) {
        const D* sS = s + DIM * DIM;
        const D* cv = sS + V::N;
        D geo = 0;   // Grad N_a . S Grad N_b (S stored as its upper triangle, row by row)
#pragma unroll
        for (int I = 0; I < DIM; ++I)
#pragma unroll
          for (int J = 0; J < DIM; ++J) {
            const int lo = I < J ? I : J, hi = I < J ? J : I;
            geo += ga[I] * sS[lo * DIM - lo * (lo - 1) / 2 + (hi - lo)] * gb[J];
          }
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            D m = 0;
#pragma unroll
            for (int j = 0; j < DIM; ++j)
#pragma unroll
              for (int l = 0; l < DIM; ++l) m += va[j] * cv[V::packed(V::of(i, j), V::of(k, l))] * vb[l];
            acc[i][k] += wq * (m + (i == k ? geo : 0.0));
          }
      } else {
        const D c1 = s[DIM * DIM], l2 = s[DIM * DIM + 1], mu = s[DIM * DIM + 2];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int k = 0; k < DIM; ++k)
            acc[i][k] += wq * (c1 * va[k] * vb[i] + l2 * va[i] * vb[k] + (i == k ? mu * gg : 0.0));
      }
    }
    const long long nodeb = (ex * P + bx) + (long long)a.L * ((ey * P + by) + (long long)a.L * (ez * P + bz));
    sink.template add<DIM>(a, nodeb, ex * P + bx, ey * P + by, ez * P + bz, acc);
  }
}

}  // namespace mfh
