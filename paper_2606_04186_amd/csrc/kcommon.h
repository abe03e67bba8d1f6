// Helpers shared by the libqflow kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>

namespace qf {

constexpr int kBlock = 256;

inline unsigned grid_for(size_t work, int block = kBlock, size_t cap = 1u << 20) {
  size_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// through FP32), stored at element i of the two planes
__device__ inline void store_bf16_split(double x, __bf16* hi, __bf16* lo, size_t i) {
  const __bf16 h = (__bf16)(float)x;
  hi[i] = h;
  lo[i] = (__bf16)(float)(x - (double)(float)h);
}

__device__ inline double wave_max(double x) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// Operands of the global commutator evaluations.
struct GlobalOps {
  const double *f, *V, *y1, *y2, *L, *LY, *t1, *t2;
  int n, o;
  const double *ga_h, *g22_h, *j1_h, *j2_h, *ga_y, *g22_y, *j1_y, *j2_y;
  const double *zv, *zo;     // [v][v][o][o], [o][o][v][v]: sigma1 x two-body pieces (residual)
  const double *u_h;         // [x1, sigma_2]_2 of H_N (= two-body of Yg), dense
  const double *s2p, *s2q;   // compact parts of [y1, sigma_2]_2 (Sigma2Lazy)
  const double *c1_h, *c1_y; // [n][n] one-body parts of [H_N, sigma] and [Yg, sigma]
  const double *lo_h, *lo_y; // [v*v][o*o] occupied-occupied ladders
  const double *pf;          // compact parts P1..P4 of [F, sigma_2] (launch_sigma2)
  const double* zc = nullptr;   // dense sigma1 (H_N + Yg/2) (heff), or NULL
  const double* qf = nullptr;   // compact parts Q1, Q2 of [F, sigma_2] (launch_sigma2)
  const double* fs1 = nullptr;  // [2][n][n] one-body external sums of the D1 tables
};

}  // namespace qf
