// FP64 contractions on matrix cores (ladder, ring and one-body ring
// intermediates): C[M][N] = scale * sum_k A[m][k] B[n][k], both operands
// K-contiguous (row-major A[M][K], B[N][K]).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kcommon.h"
#include "kernels.h"

namespace qf {

namespace {

// ---------------------------------------------------------------------------
// v_mfma_f64_16x16x4f64 operand layout (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] (k = l/16), and holds D[l/16 + 4*i][l%16] in element i.
//
// A workgroup of four waves (2 x 2) owns a (32*TM) x (32*TN) tile of C; each
// wave computes TM x TN MFMA tiles of 16 x 16.  K advances in steps of 16:
// the next step's operands are loaded into registers while the matrix cores
// work on the current one from LDS.  Rows of the LDS tiles are padded to 18
// doubles, which keeps the operand reads of a half-wave on distinct banks.
//
// blockIdx.x = column tile (fastest, so the workgroups that share a row tile
// of A run together), blockIdx.y = row tile, blockIdx.z = K split.  With one
// split C is written directly; with several, split z writes slice z of C
// (C + z*M*N) and k_sum_slices adds the slices in order.
// ---------------------------------------------------------------------------

GemmTuning g_tune{};
constexpr int kComputeUnits = 256;
long split_target_workgroups() { return (long)g_tune.split_target * kComputeUnits; }
// FP64 tile: 128 x 96 when it pads N less than 128 x 128 (f64_tile 0)
bool f64_tile_4x3(int N) {
  if (g_tune.f64_tile == 1) return true;
  if (g_tune.f64_tile == 2) return false;
  return (long)((N + 95) / 96) * 96 < (long)((N + 127) / 128) * 128;
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 16;
constexpr int kLD = kBK + 2;

// Up to kMaxBatch products of one shape in one launch: blockIdx.z = batch
// entry * splits + K split.
constexpr int kMaxBatch = 4;
struct GemmBatch {
  const double* A[kMaxBatch];
  const double* B[kMaxBatch];
  double* C[kMaxBatch];
};

template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(GemmBatch gb, double* __restrict__ part,
                                                  int M, int N, int K, int kchunk, int splits,
                                                  int to_slices, double scale) {
  const int bz = blockIdx.z / splits;
  const double* __restrict__ A = gb.A[bz];
  const double* __restrict__ B = gb.B[bz];
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int LA = BM * kBK / 256, LB = BN * kBK / 256;
  __shared__ double As[BM * kLD];
  __shared__ double Bs[BN * kLD];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const int ks = (blockIdx.z % splits) * kchunk;
  const int ke = min(K, ks + kchunk);
  double ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gm = m0 + e / kBK, gk = k0 + e % kBK;
      ra[i] = (gm < M && gk < ke) ? A[(size_t)gm * K + gk] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gn = n0 + e / kBK, gk = k0 + e % kBK;
      rb[i] = (gn < N && gk < ke) ? B[(size_t)gn * K + gk] : 0.0;
    }
  };
  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (ks < ke) load(ks);
  for (int k0 = ks; k0 < ke; k0 += kBK) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = threadIdx.x + 256 * i;
      As[(e / kBK) * kLD + e % kBK] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = threadIdx.x + 256 * i;
      Bs[(e / kBK) * kLD + e % kBK] = rb[i];
    }
    __syncthreads();
    if (k0 + kBK < ke) load(k0 + kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = As[(wm * 16 * TM + i * 16 + lane % 16) * kLD + kk + lane / 16];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = Bs[(wn * 16 * TN + j * 16 + lane % 16) * kLD + kk + lane / 16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = to_slices ? part + (size_t)blockIdx.z * M * N : gb.C[bz];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * 16 * TN + j * 16 + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 16 * TM + i * 16 + lane / 16 + 4 * r;
        if (row < M && col < N) out[(size_t)row * N + col] = scale * acc[i][j][r];
      }
    }
}

// FP32 operands: v_mfma_f32_16x16x4f32 has the same A/B lane layout, and
// lane l holds D[4*(l/16) + i][l%16] in element i.  Products are summed in
// FP32 over 64 consecutive k (four K steps), then added into FP64
// accumulators, so the rounding of long sums stays at the FP64 level.
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kFlush = 4;   // K steps per FP32 partial sum

template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_gemm_f32(const float* __restrict__ A,
                                                     const float* __restrict__ B,
                                                     double* __restrict__ C, int M, int N, int K,
                                                     int kchunk, int to_slices, double scale) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int LA = BM * kBK / 256, LB = BN * kBK / 256;
  __shared__ float As[BM * kLD];
  __shared__ float Bs[BN * kLD];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const int ks = blockIdx.z * kchunk;
  const int ke = min(K, ks + kchunk);
  float ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gm = m0 + e / kBK, gk = k0 + e % kBK;
      ra[i] = (gm < M && gk < ke) ? A[(size_t)gm * K + gk] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gn = n0 + e / kBK, gk = k0 + e % kBK;
      rb[i] = (gn < N && gk < ke) ? B[(size_t)gn * K + gk] : 0.f;
    }
  };
  f4 acc[TM][TN];
  d4 acc64[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
        acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  if (ks < ke) load(ks);
  int step = 0;
  for (int k0 = ks; k0 < ke; k0 += kBK) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = threadIdx.x + 256 * i;
      As[(e / kBK) * kLD + e % kBK] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = threadIdx.x + 256 * i;
      Bs[(e / kBK) * kLD + e % kBK] = rb[i];
    }
    __syncthreads();
    if (k0 + kBK < ke) load(k0 + kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      float a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = As[(wm * 16 * TM + i * 16 + lane % 16) * kLD + kk + lane / 16];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = Bs[(wn * 16 * TN + j * 16 + lane % 16) * kLD + kk + lane / 16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (++step == kFlush) {
      flush();
      step = 0;
    }
    __syncthreads();
  }
  flush();
  double* out = to_slices ? C + (size_t)blockIdx.z * M * N : C;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * 16 * TN + j * 16 + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 16 * TM + i * 16 + 4 * (lane / 16) + r;
        if (row < M && col < N) out[(size_t)row * N + col] = scale * acc64[i][j][r];
      }
    }
}

__global__ void k_cvt_f32(const double* __restrict__ src, float* __restrict__ dst, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// BF16x3 operands: every value is split as x = hi + lo (both bf16; lo =
// bf16(x - hi)), stored as two arrays of rows padded to a multiple of 32 k
// with zeros.  v_mfma_f32_16x16x32_bf16 takes eight consecutive k per lane
// (lane l: row l%16, k = 8*(l/16) .. +7) and returns D[4*(l/16) + i][l%16].
// Each 32-k step adds lo*hi, hi*lo and hi*hi (the lo*lo term, 2^-16 of the
// product, is dropped) in FP32; the FP32 sums go into FP64 every 64 k.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
constexpr int kBK3 = 32;
constexpr int kLD3 = kBK3 + 8;   // bf16 per LDS row: 80 bytes keeps a half-wave on distinct banks

template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_gemm_bf16x3(
    const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al, const __bf16* __restrict__ Bh,
    const __bf16* __restrict__ Bl, double* __restrict__ C, int M, int N, int Kp, int kchunk,
    int to_slices, double scale) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  // 16-byte groups (8 k) of a tile row-slice: BM*4 and BN*4 per step, per thread
  constexpr int NGA = BM * kBK3 / 8, NGB = BN * kBK3 / 8;
  constexpr int GA = (NGA + 255) / 256, GB = (NGB + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 Ash[BM * kLD3];
  __shared__ __attribute__((aligned(16))) __bf16 Asl[BM * kLD3];
  __shared__ __attribute__((aligned(16))) __bf16 Bsh[BN * kLD3];
  __shared__ __attribute__((aligned(16))) __bf16 Bsl[BN * kLD3];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wm = wave / 2, wn = wave % 2;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const int ks = blockIdx.z * kchunk;
  const int ke = min(Kp, ks + kchunk);
  s8v rah[GA], ral[GA], rbh[GB], rbl[GB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < GA; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gm = m0 + e / 4, gk = k0 + 8 * (e % 4);
      const bool ok = e < NGA && gm < M && gk < ke;
      const size_t off = (size_t)gm * Kp + gk;
      rah[i] = ok ? *reinterpret_cast<const s8v*>(Ah + off) : s8v(0);
      ral[i] = ok ? *reinterpret_cast<const s8v*>(Al + off) : s8v(0);
    }
#pragma unroll
    for (int i = 0; i < GB; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int gn = n0 + e / 4, gk = k0 + 8 * (e % 4);
      const bool ok = e < NGB && gn < N && gk < ke;
      const size_t off = (size_t)gn * Kp + gk;
      rbh[i] = ok ? *reinterpret_cast<const s8v*>(Bh + off) : s8v(0);
      rbl[i] = ok ? *reinterpret_cast<const s8v*>(Bl + off) : s8v(0);
    }
  };
  f4 acc[TM][TN];
  d4 acc64[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
        acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  if (ks < ke) load(ks);
  int step = 0;
  for (int k0 = ks; k0 < ke; k0 += kBK3) {
#pragma unroll
    for (int i = 0; i < GA; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e >= NGA) break;
      const int o = (e / 4) * kLD3 + 8 * (e % 4);
      *reinterpret_cast<s8v*>(Ash + o) = rah[i];
      *reinterpret_cast<s8v*>(Asl + o) = ral[i];
    }
#pragma unroll
    for (int i = 0; i < GB; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e >= NGB) break;
      const int o = (e / 4) * kLD3 + 8 * (e % 4);
      *reinterpret_cast<s8v*>(Bsh + o) = rbh[i];
      *reinterpret_cast<s8v*>(Bsl + o) = rbl[i];
    }
    __syncthreads();
    if (k0 + kBK3 < ke) load(k0 + kBK3);
    // all B fragments of the step held, A's streamed one row tile ahead, so
    // that each A read has the previous tile's 3 TN MFMAs to land behind
    bf8 bh[TN], bl[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int o = (wn * 16 * TN + j * 16 + lane % 16) * kLD3 + 8 * (lane / 16);
      bh[j] = *reinterpret_cast<const bf8*>(Bsh + o);
      bl[j] = *reinterpret_cast<const bf8*>(Bsl + o);
    }
    const int oa = (wm * 16 * TM + lane % 16) * kLD3 + 8 * (lane / 16);
    bf8 ah = *reinterpret_cast<const bf8*>(Ash + oa);
    bf8 al = *reinterpret_cast<const bf8*>(Asl + oa);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      bf8 nh, nl;
      if (i + 1 < TM) {
        nh = *reinterpret_cast<const bf8*>(Ash + oa + (i + 1) * 16 * kLD3);
        nl = *reinterpret_cast<const bf8*>(Asl + oa + (i + 1) * 16 * kLD3);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
      }
      if (i + 1 < TM) {
        ah = nh;
        al = nl;
      }
    }
    if (++step == 2) {
      flush();
      step = 0;
    }
    __syncthreads();
  }
  flush();
  double* out = to_slices ? C + (size_t)blockIdx.z * M * N : C;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * 16 * TN + j * 16 + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 16 * TM + i * 16 + 4 * (lane / 16) + r;
        if (row < M && col < N) out[(size_t)row * N + col] = scale * acc64[i][j][r];
      }
    }
}

// hi/lo bf16 split of a row-major [rows][K] FP64 matrix into [rows][Kp]
// (Kp >= K, zero padded).
__global__ void k_split_bf16(const double* __restrict__ src, int rows, int K, int Kp,
                             __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  const size_t tot = (size_t)rows * Kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / Kp;
    const int k = (int)(e % Kp);
    const double x = k < K ? src[r * K + k] : 0.0;
    store_bf16_split(x, hi, lo, e);
  }
}

__global__ __launch_bounds__(256) void k_sum_slices(const double* __restrict__ part, int splits,
                                                    size_t count, double* C) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int i = 0; i < splits; ++i) s += part[(size_t)i * count + e];
  C[e] = s;
}

// the same for the entries of a batch: entry b's slices at part + b*splits*count
__global__ __launch_bounds__(256) void k_sum_slices_batch(const double* __restrict__ part,
                                                          int splits, size_t count, GemmBatch gb,
                                                          int nb) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= count * nb) return;
  const int b = (int)(e / count);
  const size_t i0 = e % count;
  const double* src = part + (size_t)b * splits * count;
  double s = 0.0;
  for (int i = 0; i < splits; ++i) s += src[(size_t)i * count + i0];
  gb.C[b][i0] = s;
}

template <int TM, int TN, class T>
void launch_tiles(const T* A, const T* B, double* C, double* part, size_t part_cap,
                  int M, int N, int K, double scale, hipStream_t st) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  const int tiles_n = (N + BN - 1) / BN, tiles_m = (M + BM - 1) / BM;
  const long tiles = (long)tiles_n * tiles_m;
  // split K until about four workgroups per compute unit are available,
  // keeping at least eight K steps per split and the slices within `part`
  const long kTarget = split_target_workgroups();
  const size_t mn = (size_t)M * N;
  int splits = 1;
  if (tiles < kTarget && part != nullptr) {
    splits = (int)((kTarget + tiles - 1) / tiles);
    splits = std::min(splits, std::max(1, K / (8 * kBK)));
    splits = (int)std::min<size_t>((size_t)splits, part_cap / mn);
    splits = std::min(splits, kMaxSplits);
    splits = std::max(splits, 1);
  }
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  splits = (K + kchunk - 1) / kchunk;
  GemmBatch one{};
  if constexpr (sizeof(T) == 8) {
    one.A[0] = A;
    one.B[0] = B;
    one.C[0] = C;
  }
  if (splits <= 1) {
    dim3 grid(tiles_n, tiles_m, 1);
    if constexpr (sizeof(T) == 8)
      k_gemm_f64<TM, TN><<<grid, 256, 0, st>>>(one, nullptr, M, N, K, K > 0 ? K : kBK, 1, 0,
                                               scale);
    else
      k_gemm_f32<TM, TN><<<grid, 256, 0, st>>>(A, B, C, M, N, K, K > 0 ? K : kBK, 0, scale);
    return;
  }
  dim3 grid(tiles_n, tiles_m, splits);
  if constexpr (sizeof(T) == 8)
    k_gemm_f64<TM, TN><<<grid, 256, 0, st>>>(one, part, M, N, K, kchunk, splits, 1, scale);
  else
    k_gemm_f32<TM, TN><<<grid, 256, 0, st>>>(A, B, part, M, N, K, kchunk, 1, scale);
  k_sum_slices<<<grid_for(mn), kBlock, 0, st>>>(part, splits, mn, C);
}

// nb <= kMaxBatch FP64 products of one shape in one launch (K split as in
// launch_tiles, counting the workgroups of all entries)
template <int TM, int TN>
void launch_tiles_batch(const GemmBatch& gb, int nb, double* part, size_t part_cap, int M,
                        int N, int K, double scale, hipStream_t st) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  const int tiles_n = (N + BN - 1) / BN, tiles_m = (M + BM - 1) / BM;
  const long tiles = (long)tiles_n * tiles_m * nb;
  const long kTarget = split_target_workgroups();
  const size_t mn = (size_t)M * N;
  int splits = 1;
  if (tiles < kTarget && part != nullptr) {
    splits = (int)((kTarget + tiles - 1) / tiles);
    splits = std::min(splits, std::max(1, K / (8 * kBK)));
    splits = (int)std::min<size_t>((size_t)splits, part_cap / (mn * nb));
    splits = std::min(splits, kMaxSplits);
    splits = std::max(splits, 1);
  }
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  splits = (K + kchunk - 1) / kchunk;
  if (splits <= 1) {
    dim3 grid(tiles_n, tiles_m, nb);
    k_gemm_f64<TM, TN><<<grid, 256, 0, st>>>(gb, nullptr, M, N, K, K > 0 ? K : kBK, 1, 0, scale);
    return;
  }
  dim3 grid(tiles_n, tiles_m, nb * splits);
  k_gemm_f64<TM, TN><<<grid, 256, 0, st>>>(gb, part, M, N, K, kchunk, splits, 1, scale);
  k_sum_slices_batch<<<grid_for(mn * nb), kBlock, 0, st>>>(part, splits, mn, gb, nb);
}

template <class T>
void launch_gemm(const T* A, const T* B, double* C, int M, int N, int K, double scale,
                 double* part, size_t part_cap, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  // 128 x 96 or 128 x 128 tiles (f64_tile_4x3)
  // (FP32 operands always take 128 x 96: the wider tile does not fit the
  // registers with its FP64 accumulators)
  if constexpr (sizeof(T) == 4) {
    launch_tiles<4, 3>(A, B, C, part, part_cap, M, N, K, scale, st);
  } else {
    if (f64_tile_4x3(N))
      launch_tiles<4, 3>(A, B, C, part, part_cap, M, N, K, scale, st);
    else
      launch_tiles<4, 4>(A, B, C, part, part_cap, M, N, K, scale, st);
  }
}

template <int TM, int TN>
void launch_tiles_bf16x3(const __bf16* Ah, const __bf16* Al, const __bf16* Bh, const __bf16* Bl,
                         double* C, double* part, size_t part_cap, int M, int N, int Kp,
                         double scale, hipStream_t st) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  const int tiles_n = (N + BN - 1) / BN, tiles_m = (M + BM - 1) / BM;
  const long tiles = (long)tiles_n * tiles_m;
  const long kTarget = split_target_workgroups();
  const size_t mn = (size_t)M * N;
  int splits = 1;
  if (tiles < kTarget && part != nullptr) {
    splits = (int)((kTarget + tiles - 1) / tiles);
    splits = std::min(splits, std::max(1, Kp / (8 * kBK3)));
    splits = (int)std::min<size_t>((size_t)splits, part_cap / mn);
    splits = std::min(splits, kMaxSplits);
    splits = std::max(splits, 1);
  }
  int kchunk = (Kp + splits - 1) / splits;
  kchunk = (kchunk + kBK3 - 1) / kBK3 * kBK3;
  splits = (Kp + kchunk - 1) / kchunk;
  if (splits <= 1) {
    dim3 grid(tiles_n, tiles_m, 1);
    k_gemm_bf16x3<TM, TN><<<grid, 256, 0, st>>>(Ah, Al, Bh, Bl, C, M, N, Kp,
                                                Kp > 0 ? Kp : kBK3, 0, scale);
    return;
  }
  dim3 grid(tiles_n, tiles_m, splits);
  k_gemm_bf16x3<TM, TN><<<grid, 256, 0, st>>>(Ah, Al, Bh, Bl, part, M, N, Kp, kchunk, 1, scale);
  k_sum_slices<<<grid_for(mn), kBlock, 0, st>>>(part, splits, mn, C);
}

}  // namespace

void launch_gemm_nt_bf16x3(const __bf16* Ah, const __bf16* Al, const __bf16* Bh, const __bf16* Bl,
                           double* C, int M, int N, int Kp, double scale, double* part,
                           size_t part_cap, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  launch_tiles_bf16x3<4, 3>(Ah, Al, Bh, Bl, C, part, part_cap, M, N, Kp, scale, st);
}

void set_gemm_tuning(const GemmTuning& t) { g_tune = t; }

void launch_split_bf16(const double* src, int rows, int K, int Kp, __bf16* hi, __bf16* lo,
                       hipStream_t st) {
  k_split_bf16<<<grid_for((size_t)rows * Kp, kBlock, 65536), kBlock, 0, st>>>(src, rows, K, Kp,
                                                                              hi, lo);
}

void launch_gemm_nt_f64(const double* A, const double* B, double* C, int M, int N, int K,
                        double scale, double* part, size_t part_cap, hipStream_t st) {
  launch_gemm(A, B, C, M, N, K, scale, part, part_cap, st);
}

int launch_gemm_nt_f64_batch(const double* const* A, const double* const* B, double* const* C,
                             int nb, int M, int N, int K, double scale, double* part,
                             size_t part_cap, hipStream_t st) {
  if (nb < 1 || nb > kMaxBatch) return -1;
  if (M <= 0 || N <= 0) return 0;
  GemmBatch gb{};
  for (int b = 0; b < nb; ++b) {
    gb.A[b] = A[b];
    gb.B[b] = B[b];
    gb.C[b] = C[b];
  }
  if (f64_tile_4x3(N))
    launch_tiles_batch<4, 3>(gb, nb, part, part_cap, M, N, K, scale, st);
  else
    launch_tiles_batch<4, 4>(gb, nb, part, part_cap, M, N, K, scale, st);
  return 0;
}

void launch_gemm_nt_f32(const float* A, const float* B, double* C, int M, int N, int K,
                        double scale, double* part, size_t part_cap, hipStream_t st) {
  launch_gemm(A, B, C, M, N, K, scale, part, part_cap, st);
}

void launch_cvt_f32(const double* src, float* dst, size_t count, hipStream_t st) {
  k_cvt_f32<<<grid_for(count, kBlock, 65536), kBlock, 0, st>>>(src, dst, count);
}

}  // namespace qf
