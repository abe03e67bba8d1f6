// FP64 contractions on matrix cores (ladder and ring intermediates).
#include <hip/hip_runtime.h>

#include <math.h>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// FP64 matrix-core GEMM  C[M][N] += sum_k A[m][k] B[n][k]
//
// v_mfma_f64_16x16x4f64 operand layout (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] (k = l/16), and holds D[l/16 + 4*i][l%16] in element i.
// A workgroup of four waves owns 64 rows and up to 176 columns (blockIdx.z
// selects the column block); each wave computes 16 rows x 176 columns.  The K range is split in two halves over
// blockIdx.y; both halves add into C (zeroed beforehand), and since exactly
// two terms are added to zero the result does not depend on their order.
// ---------------------------------------------------------------------------

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGemmBM = 64;
constexpr int kGemmBK = 16;
constexpr int kGemmNT = 11;   // column tiles of 16 -> N <= 176

__global__ __launch_bounds__(256) void k_gemm_nt_f64(const double* __restrict__ A,
                                                     const double* __restrict__ B, double* C,
                                                     int M, int N, int K, int kchunk,
                                                     int to_slices) {
  __shared__ double As[kGemmBM][kGemmBK + 1];
  __shared__ double Bs[kGemmNT * 16][kGemmBK + 1];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int m0 = blockIdx.x * kGemmBM;
  const int n0 = blockIdx.z * kGemmNT * 16;
  const int ks = blockIdx.y * kchunk;
  const int ke = min(K, ks + kchunk);
  const int ntiles = min(kGemmNT, (N - n0 + 15) / 16);
  d4 acc[kGemmNT];
#pragma unroll
  for (int t = 0; t < kGemmNT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = ks; k0 < ke; k0 += kGemmBK) {
    for (int e = threadIdx.x; e < kGemmBM * kGemmBK; e += 256) {
      const int r = e / kGemmBK, c = e % kGemmBK;
      const int gm = m0 + r, gk = k0 + c;
      As[r][c] = (gm < M && gk < ke) ? A[(size_t)gm * K + gk] : 0.0;
    }
    for (int e = threadIdx.x; e < ntiles * 16 * kGemmBK; e += 256) {
      const int r = e / kGemmBK, c = e % kGemmBK;
      const int gk = k0 + c;
      Bs[r][c] = (n0 + r < N && gk < ke) ? B[(size_t)(n0 + r) * K + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 4) {
      const double a = As[wave * 16 + lane % 16][kk + lane / 16];
#pragma unroll
      for (int t = 0; t < kGemmNT; ++t) {
        if (t < ntiles) {
          const double b = Bs[t * 16 + lane % 16][kk + lane / 16];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kGemmNT; ++t) {
    if (t >= ntiles) continue;
    const int col = n0 + t * 16 + lane % 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = m0 + wave * 16 + lane / 16 + 4 * i;
      if (row >= M || col >= N) continue;
      if (to_slices)
        C[((size_t)blockIdx.y * M + row) * N + col] = acc[t][i];
      else
        atomicAdd(&C[(size_t)row * N + col], acc[t][i]);
    }
  }
}

__global__ __launch_bounds__(256) void k_sum_slices(const double* __restrict__ part, int splits,
                                                    size_t count, double scale, double* C) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int i = 0; i < splits; ++i) s += part[(size_t)i * count + e];
  C[e] = scale * s;
}

}  // namespace

void launch_gemm_nt_f64_splitk(const double* A, const double* B, double* part, double* C, int M,
                               int N, int K, double scale, hipStream_t st) {
  int kchunk = (K + kMaxSplits - 1) / kMaxSplits;
  kchunk = (kchunk + kGemmBK - 1) / kGemmBK * kGemmBK;
  const int splits = (K + kchunk - 1) / kchunk;
  dim3 grid((M + kGemmBM - 1) / kGemmBM, splits, (N + kGemmNT * 16 - 1) / (kGemmNT * 16));
  k_gemm_nt_f64<<<grid, 256, 0, st>>>(A, B, part, M, N, K, kchunk, 1);
  const size_t count = (size_t)M * N;
  k_sum_slices<<<grid_for(count), kBlock, 0, st>>>(part, splits, count, scale, C);
}

void launch_gemm_nt_f64(const double* A, const double* B, double* C, int M, int N, int K,
                        hipStream_t st) {
  int kchunk = (K + 1) / 2;
  kchunk = (kchunk + kGemmBK - 1) / kGemmBK * kGemmBK;
  const int splits = (K + kchunk - 1) / kchunk;
  dim3 grid((M + kGemmBM - 1) / kGemmBM, splits, (N + kGemmNT * 16 - 1) / (kGemmNT * 16));
  k_gemm_nt_f64<<<grid, 256, 0, st>>>(A, B, C, M, N, K, kchunk, 0);
}

}  // namespace qf
