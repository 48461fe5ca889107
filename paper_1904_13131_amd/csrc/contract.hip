// The 1-D contraction stage of the sum factorisation (Sec. 5) in two forms,
// for the autotuner's VALU-against-MFMA decision at degrees 3 and 4 in FP32.
// One workgroup holds 256 lines of n = p + 1 values in LDS (the layout of the
// tangent kernels' sweeps: value a of line l at X[a][l]) and applies, sweep
// after sweep, the pair (S, D) of n x n Gauss-point tables: Y_S = S X,
// Y_D = D X, then X <- Y_S + Y_D (so that every sweep depends on the last).
//   VALU: thread l owns line l: n LDS reads, 2 n^2 FMAs, n LDS writes.
//   MFMA: a wave takes 16 lines per v_mfma_f32_16x16x4f32: A (16 x 4) holds
//   the stacked tables [S; D] (2n of 16 rows used) for 4 values of a, B (4 x
//   16) the lines' values (one LDS read per lane), ceil(n / 4) instructions per
//   16 lines; the 16 x 16 result gives S X and D X of the 16 lines.
// The tables are the same n x n matrices in both forms, passed as kernel
// arguments (runtime values read through scalar loads, as in the tangent
// kernels, so that the compiler cannot fold zero entries away); both forms
// write their final X for comparison.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "fused.hpp"

namespace mfh {
namespace {

constexpr int kLines = 256;
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct Tab {
  float S[5][5], D[5][5];
};

template <int N1>
__global__ void __launch_bounds__(kLines) k_contract_valu(Tab tab, int sweeps, float* __restrict__ out) {
  __shared__ float X[N1][kLines];
  const int l = threadIdx.x;
#pragma unroll
  for (int a = 0; a < N1; ++a) X[a][l] = 0.01f * (a + 1) + 1e-4f * (l + blockIdx.x);
  __syncthreads();
  for (int s = 0; s < sweeps; ++s) {
    float v[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) v[a] = X[a][l];
    float y[N1];
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      float ys = 0.f, yd = 0.f;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        ys += tab.S[q][a] * v[a];
        yd += tab.D[q][a] * v[a];
      }
      y[q] = ys + yd;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N1; ++q) X[q][l] = y[q];
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < N1; ++a) out[((long long)blockIdx.x * N1 + a) * kLines + l] = X[a][l];
}

template <int N1>
__global__ void __launch_bounds__(kLines) k_contract_mfma(Tab tab, int sweeps, float* __restrict__ out) {
  __shared__ float X[N1][kLines];
  constexpr int KC = (N1 + 3) / 4;   // K chunks of 4
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int row = lane & 15, kq = lane >> 4;   // A: (row, k); B: (k, column = row)
#pragma unroll
  for (int a = 0; a < N1; ++a) X[a][t] = 0.01f * (a + 1) + 1e-4f * (t + blockIdx.x);
  // A operand per K chunk: [S; D] stacked, rows 0..N1-1 S, N1..2N1-1 D
  float A[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int a = kq + 4 * c;
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < N1; ++q)
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        v = (row == q && a == b) ? tab.S[q][b] : v;
        v = (row == N1 + q && a == b) ? tab.D[q][b] : v;
      }
    A[c] = v;
  }
  __syncthreads();
  for (int s = 0; s < sweeps; ++s) {
    floatx4 D[4];   // 4 groups of 16 lines per wave (64 lines)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int line = wave * 64 + g * 16 + row;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int a = kq + 4 * c;
        const float b = a < N1 ? X[a][line] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[c], b, acc, 0, 0, 0);
      }
      D[g] = acc;
    }
    __syncthreads();
    // lane holds result rows 4 kq .. 4 kq + 3 of column `row`: S rows q < N1,
    // D rows N1 + q; X[q] = S X + D X, summed through LDS by two passes
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int line = wave * 64 + g * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 4 * kq + r;
        if (rr < N1) X[rr][line] = D[g][r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int line = wave * 64 + g * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 4 * kq + r;
        if (rr >= N1 && rr < 2 * N1) X[rr - N1][line] += D[g][r];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < N1; ++a) out[((long long)blockIdx.x * N1 + a) * kLines + t] = X[a][t];
}

template <int N1>
void launch(int mfma, int sweeps, int blocks, float* out, hipStream_t s) {
  Tab tab{};   // S_qa = 1 / (1 + q + 2a), D_qa = (q - a) / 8: spectral radius of S + D near 1
  for (int q = 0; q < N1; ++q)
    for (int a = 0; a < N1; ++a) {
      tab.S[q][a] = 1.0f / (1.0f + q + 2 * a);
      tab.D[q][a] = (q - a) * 0.125f;
    }
  if (mfma)
    hipLaunchKernelGGL(k_contract_mfma<N1>, dim3(blocks), dim3(kLines), 0, s, tab, sweeps, out);
  else
    hipLaunchKernelGGL(k_contract_valu<N1>, dim3(blocks), dim3(kLines), 0, s, tab, sweeps, out);
}

}  // namespace

void contraction_stage(int degree, int mfma, int sweeps, int blocks, float* out, hipStream_t s) {
  if (degree == 3)
    launch<4>(mfma, sweeps, blocks, out, s);
  else
    launch<5>(mfma, sweeps, blocks, out, s);
}

}  // namespace mfh
