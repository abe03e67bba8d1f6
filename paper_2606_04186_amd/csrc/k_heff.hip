// Per-space downfolded Hamiltonians in CAS form.
//
// For space A with tau = the amplitudes inside A and s = sigma - tau,
//   Hbar|_A = H + [H,sigma] - [H,tau]
//           + 1/2 ([Yg,sigma] - [Yg,tau] - [Ft,sigma] + [Ft,tau]),
// Yg = [F,sigma], Ft = [F,tau].  Three kernels accumulate the H, Yg and Ft
// groups of terms into the normal-ordered block (x0, x1[na^2], x2[na^4]) of
// each space, held in the output slot itself; a fourth rewrites the slot in
// CAS form (Ec, h, g) relative to the empty active space.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "kcommon.h"
#include "kernels.h"
#include "qflow_cas.h"
#include "qflow_eval.h"

namespace qf {

namespace {

// Per-space tables of the marked [E,sigma] evaluation (see MarkTables), for
// a size class of NA orbitals (NA/2 occupied):
//   tau1[a][b], tau2[a][b][c][d]           sigma restricted to the space;
//   D1[j][t][a] = sum_{x external} f[x][t] sigma1(x in slot j, a in the other)
//     = fs1[j][t][a] (the sum over every orbital, k_fs1) less the active x;
//   D_j(t;a,b,c) = sum_{x external} f[x][t] sigma(.. x in slot j ..), j = 0, 1,
//     which vanish unless b and c share a class and a is in the other one; x
//     then runs over the externals of a's class: the sums over all orbitals of
//     that class are [F, sigma_2]'s P3/P4 (a virtual) or Q1/Q2 (a occupied),
//     less the active ones.  D_2(t;a,b,c) = -D_0(t;c,a,b) and
//     D_3(t;a,b,c) = -D_1(t;c,a,b) by anti-Hermiticity, so they are not stored;
// then H_N and Yg restricted to the space: [f_A | V_A | y1_A | y2_A].
template <int NA>
__global__ __launch_bounds__(256) void k_heff_tab(GlobalOps g,
                                                  const SpaceDev* __restrict__ spaces,
                                                  const int32_t* __restrict__ idx, double* tab,
                                                  int64_t tab_stride) {
  constexpr int NO = NA / 2, N2 = NA * NA, N3 = N2 * NA, N4 = N3 * NA;
  constexpr int S1 = N2, S2 = N4, S3 = 2 * N2, S4 = 2 * N4;
  __shared__ int orb[NA];
  const int k = idx[blockIdx.x];
  if (threadIdx.x < NA) orb[threadIdx.x] = spaces[k].orb[threadIdx.x];
  __syncthreads();
  const int n = g.n, o = g.o, v = n - o;
  const Sigma s{g.t1, g.t2, n, o, v};
  double* out = tab + (int64_t)k * tab_stride;
  for (int e = threadIdx.x; e < N2; e += blockDim.x) out[e] = s.one(orb[e / NA], orb[e % NA]);
  for (int e = threadIdx.x; e < N4; e += blockDim.x)
    out[S1 + e] = s.two(orb[e / N3], orb[e / N2 % NA], orb[e / NA % NA], orb[e % NA]);
  for (int e = threadIdx.x; e < 2 * N2; e += blockDim.x) {
    const int j = e / N2, ft = orb[e / NA % NA], pa = orb[e % NA];
    double acc = g.fs1[((size_t)j * n + ft) * n + pa];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int x = orb[i];
      acc -= g.f[x * n + ft] * (j == 0 ? s.one(x, pa) : s.one(pa, x));
    }
    out[S1 + S2 + e] = acc;
  }
  // D_0, D_1 (D_2 and D_3 are read from them with permuted indices)
  for (int e = threadIdx.x; e < 2 * N4; e += blockDim.x) {
    const int j = e / N4, t = e / N3 % NA, a = e / N2 % NA, b = e / NA % NA, c = e % NA;
    const bool ao = a < NO, bo = b < NO, co = c < NO;
    double acc = 0.0;
    if (bo == co && ao != bo) {
      const int ft = orb[t], pa = orb[a], pb = orb[b], pc = orb[c];
      if (ao) {
        // x over all occupied orbitals is Q1 (slot 0) / Q2 (slot 1) of
        // [F, sigma_2] (-sum_x f[t][x] t2[x][a][b][c] and -sum_x f[t][x]
        // t2[a][x][b][c]; f symmetric), less the active occupied orbitals
        const size_t ovv = (size_t)o * v * v;
        acc = g.qf[(size_t)j * n * ovv + (size_t)ft * ovv + ((size_t)pa * v + (pb - o)) * v +
                   (pc - o)];
#pragma unroll
        for (int i = 0; i < NO; ++i) {
          const int x = orb[i];
          acc -= g.f[x * n + ft] * (j == 0 ? s.two(x, pa, pb, pc) : s.two(pa, x, pb, pc));
        }
      } else {
        // x over all virtuals is P3 (slot 0) / P4 (slot 1) of [F, sigma_2]
        // (sum_x f[x][t] t2[b][c][x][a] and sum_x f[x][t] t2[b][c][a][x]),
        // less the active virtuals
        const size_t ov2 = (size_t)o * o * v, nv = (size_t)n * ov2;
        acc = g.pf[(2 + j) * nv + (size_t)ft * ov2 + ((size_t)pb * o + pc) * v + (pa - o)];
#pragma unroll
        for (int i = NO; i < NA; ++i) {
          const int x = orb[i];
          acc -= g.f[x * n + ft] * (j == 0 ? s.two(x, pa, pb, pc) : s.two(pa, x, pb, pc));
        }
      }
    }
    out[S1 + S2 + S3 + e] = acc;
  }
  double* xo = out + S1 + S2 + S3 + S4;
  for (int e = threadIdx.x; e < N2; e += blockDim.x) {
    const int p = orb[e / NA], q = orb[e % NA];
    xo[e] = g.f[p * n + q];
    xo[N2 + N4 + e] = g.y1[p * n + q];
  }
  for (int e = threadIdx.x; e < N4; e += blockDim.x) {
    const int a = e / N3, b = e / N2 % NA, c = e / NA % NA, d = e % NA;
    const size_t i4 = (((size_t)orb[a] * n + orb[b]) * n + orb[c]) * n + orb[d];
    xo[N2 + e] = g.V[i4];
    // Yg's two-body part is an exact zero unless the class pattern lies
    // within one index of (v,v,o,o) or (o,o,v,v): not read there
    const int pat = (a < NO) << 3 | (b < NO) << 2 | (c < NO) << 1 | (d < NO);
    const bool y_on = __builtin_popcount(pat ^ 0x3) <= 1 || __builtin_popcount(pat ^ 0xC) <= 1;
    xo[2 * N2 + N4 + e] = y_on ? g.y2[i4] : 0.0;
  }
}

// Rows of the dense occupied-pair ladder's operand: xp[tri(p,q)][(t,u)] =
// (H_N + Yg/2)(p,q,t,u) for p <= q, t, u occupied.
__global__ void k_pack_x_pairs(const double* __restrict__ Xh, const double* __restrict__ Xy,
                               int n, int o, double* xp) {
  const size_t oo = (size_t)o * o, tot = (size_t)n * (n + 1) / 2 * oo;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t pr = e / oo;
    const int tu = (int)(e % oo), t = tu / o, u = tu % o;
    int p = 0;   // row pr = tri_row(p, q, n)
    while (tri_row(p + 1, p + 1, n) <= pr) ++p;
    const int q = p + (int)(pr - tri_row(p, p, n));
    const size_t x = (((size_t)p * n + q) * n + t) * n + u;
    xp[e] = Xh[x] + 0.5 * Xy[x];
  }
}

// fs1[j][t][a] = sum_x f[x][t] sigma1(x, a) (j = 0) or sigma1(a, x) (j = 1),
// over every orbital x: the external sums of the D1 tables before the
// active orbitals are taken out.  One thread per entry.
__global__ void k_fs1(const double* __restrict__ f, const double* __restrict__ t1, int n, int o,
                      double* fs1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * n * n) return;
  const int j = e / (n * n), t = e / n % n, a = e % n;
  const Sigma s{t1, nullptr, n, o, n - o};
  double acc = 0.0;
  for (int x = 0; x < n; ++x) acc += f[x * n + t] * (j == 0 ? s.one(x, a) : s.one(a, x));
  fs1[e] = acc;
}

// Slot layout while accumulating: [x0, x1 (na^2), x2 (na^4)].
// part 0: H + [H,sigma] - [H,tau]         (initialises the slot)
// part 1: + 1/2 ([Yg,sigma] - [Yg,tau])
// ([X,tau] from X and tau restricted to the space, staged in LDS, local indices)
// part 2: + 1/2 ([Ft,tau] - [Ft,sigma]) = - 1/2 [E,sigma], marked evaluation
//
// Workgroups of BLK threads; workgroup (x, y) takes space idx[x] and the
// task slots [y * BLK, (y + 1) * BLK).  NA: the size class's orbital count
// (compile-time shape of the marked evaluation of part 2; 0 for parts 0, 1).
// (Parts 0 and 1 wait on scattered global lookups: their 256-thread form is
// held to seven workgroups' worth of registers per compute unit.)
template <int PART, int BLK, int NA>
__global__ __launch_bounds__(BLK, (PART < 2 && BLK == 256) ? 7 : 1) void k_heff_part(GlobalOps g, const double* __restrict__ scal,
                                                   const SpaceDev* __restrict__ spaces,
                                                   const int32_t* __restrict__ idx,
                                                   const int64_t* __restrict__ heff_off,
                                                   const int32_t* __restrict__ tasks,
                                                   int task_stride, const double* __restrict__ tab,
                                                   int64_t tab_stride, double* heff) {
  __shared__ int orb[kMaxAct];   // the space's orbitals (synchronised below)
  extern __shared__ double tl[];
  const int k = idx[blockIdx.x];
  const SpaceDev& sp = spaces[k];
  if (threadIdx.x < sp.na) orb[threadIdx.x] = sp.orb[threadIdx.x];
  MarkTables T{};
  const int na = sp.na, n = g.n, o = g.o, v = n - o;
  const int n2 = na * na, n4 = n2 * n2;
  int s1, s2, s3, s4;
  const int tot = mark_sizes(na, &s1, &s2, &s3, &s4);
  const double* src = tab + (int64_t)k * tab_stride;
  if constexpr (PART == 2) {
    for (int e = threadIdx.x; e < tot; e += blockDim.x) tl[e] = src[e];
    T = MarkTables{tl, tl + s1, tl + s1 + s2, tl + s1 + s2 + s3, na};
  } else {
    // [x1_A | x2_A | tau1 | tau2] of the space (local indices)
    const double* xa = src + tot + (PART == 0 ? 0 : n2 + n4);
    for (int e = threadIdx.x; e < n2 + n4; e += blockDim.x) {
      tl[e] = xa[e];
      tl[n2 + n4 + e] = src[e];
    }
  }
  __syncthreads();
  const LocalOp XA{tl, tl + n2, na, sp.nocc};
  const LocalOp tauA{tl + n2 + n4, tl + 2 * n2 + n4, na, sp.nocc};
  double* slot = heff + heff_off[k];
  const Sigma s{g.t1, g.t2, n, o, v};
  const int slot_idx = (int)blockIdx.y * BLK + (int)threadIdx.x;
  if (slot_idx >= task_stride) return;
  const int32_t code = tasks[(sp.nocc - 2) * task_stride + slot_idx];
  if (code < 0) return;
  const int kind = code >> 24;
  const int la = (code >> 18) & 63, lb = (code >> 12) & 63, lc = (code >> 6) & 63, ld = code & 63;
  const int p = orb[la], q = orb[lb], r = orb[lc], t = orb[ld];
  // distinct slot positions of the task's symmetry orbit (see build_tasks)
  int d0, d1 = -1, d2 = -1, d3 = -1;
  if (kind == 2) {
    d0 = ((la * na + lb) * na + lc) * na + ld;
    const int i1 = ((lb * na + la) * na + ld) * na + lc;
    const int i2 = ((lc * na + ld) * na + la) * na + lb;
    const int i3 = ((ld * na + lc) * na + lb) * na + la;
    if (i1 != d0) d1 = i1;
    if (i2 != d0 && i2 != i1) d2 = i2;
    if (i3 != d0 && i3 != i1 && i3 != i2) d3 = i3;
    d0 += 1 + n2;
    if (d1 >= 0) d1 += 1 + n2;
    if (d2 >= 0) d2 += 1 + n2;
    if (d3 >= 0) d3 += 1 + n2;
  } else if (kind == 1) {
    d0 = 1 + la * na + lb;
    if (la != lb) d1 = 1 + lb * na + la;
  } else {
    d0 = 0;
  }
  auto emit = [&](double x, double scale, bool init) {
    const int ds[4] = {d0, d1, d2, d3};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (ds[i] >= 0) slot[ds[i]] = init ? x : slot[ds[i]] + scale * x;
  };
  if constexpr (PART == 0) {
    DenseOp H{g.f, g.V, g.L, n, o, g.ga_h, g.g22_h, g.j1_h, g.j2_h, g.u_h, g.lo_h};
    H.Z = g.zc;   // Z of H_N + Yg/2 (dense mode; else k_heff_z adds this part)
    auto cs = make_comm(H, s, n, o);
    cs.pp_loops = false;   // k_heff_pp
    const auto ct = make_comm(XA, tauA, na, sp.nocc);
    double x;
    if (kind == 2)
      x = XA.two(la, lb, lc, ld) + cs.c2(p, q, r, t) - ct.c2(la, lb, lc, ld);
    else if (kind == 1)
      x = XA.one(la, lb) + g.c1_h[p * n + q] - ct.c1(la, lb);
    else
      x = scal[3] + scal[0] - ct.c0();
    emit(x, 1.0, true);
  } else if constexpr (PART == 1) {
    const DenseOp Y{g.y1, g.y2, g.LY, n, o, g.ga_y, g.g22_y, g.j1_y, g.j2_y, nullptr, g.lo_y,
                   Sigma2Lazy{g.y1, g.t2, g.s2p, g.s2q, n, o}};
    auto cs = make_comm(Y, s, n, o);
    cs.pp_loops = false;   // k_heff_pp
    const auto ct = make_comm(XA, tauA, na, sp.nocc);
    double x;
    if (kind == 2)
      x = cs.c2(p, q, r, t) - ct.c2(la, lb, lc, ld);
    else if (kind == 1)
      x = g.c1_y[p * n + q] - ct.c1(la, lb);
    else
      x = scal[1] - ct.c0();
    emit(x, 0.5, false);
  } else {
    // two-body elements only; the one- and zero-body ones (k_heff_low) take
    // a wavefront each
    static_assert(PART != 2 || NA > 0, "the marked evaluation needs the space size");
    if (kind != 2) return;
    const MarkedE<NA> E{T};
    const MarkedSigma<NA> D{T};
    const MarkedShape<NA> shape;
    const CommE<MarkedE<NA>, MarkedSigma<NA>, true, MarkedShape<NA>> ce{E, D, shape, n, o};
    emit(ce.c2(la, lb, lc, ld), -0.5, false);   // (local indices)
  }
}

// The sigma1 x two-body part of [H_N, sigma] + [Yg, sigma]/2 on the space's
// two-body block: with X = H_N + Yg/2 (two-body parts, Hermitian and pair
// symmetric, so X(t,q,r,s) = X[s][r][q][t]),
//   Z[a][(b,c,d)] = sum_t sigma1(p_a, t) X[p_d][p_c][p_b][t]      (all t)
//   heff2[a][b][c][d] -= Z[a][bcd] + Z[b][adc] + Z[c][dab] + Z[d][cba].
// The contraction runs on the matrix cores (v_mfma_f64_16x16x4f64): rows
// (b,c,d) of X gathered 16 at a time, the space's sigma1 rows as the other
// operand (columns a, padded to 16); each wavefront takes row tiles in turn.
// A lane loads W consecutive t of its row at once (W = 2 when n is even:
// 16-byte loads) and feeds them to W MFMAs, whose k slots then hold
// t = t0 + W*kq + w; the sigma1 operand follows the same order.
// Dynamic LDS: sigma1 rows [NA][np] (np = n rounded up to 4W) and Z [NA][NA^3].
// With zs the block writes the negated sum to zs[blockIdx.x][NA^4] instead
// (k_heff_cas adds it), so that it may run beside the element kernels.
template <int NA, int W>
__global__ __launch_bounds__(256) void k_heff_z(const double* __restrict__ Xh,
                                                const double* __restrict__ Xy,
                                                const double* __restrict__ t1,
                                                const SpaceDev* __restrict__ spaces,
                                                const int32_t* __restrict__ idx,
                                                const int64_t* __restrict__ heff_off, int n,
                                                int o, double* heff, double* zs) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  typedef double dw __attribute__((ext_vector_type(W)));
  constexpr int N2 = NA * NA, N3 = N2 * NA, NT = (N3 + 15) / 16, NO = NA / 2;
  extern __shared__ double zl[];
  const int np = (n + 4 * W - 1) / (4 * W) * (4 * W), v = n - o;
  double* S = zl;             // [NA][np]
  double* Z = zl + NA * np;   // [NA][N3]
  __shared__ int orb[NA];
  const int k = idx[blockIdx.x];
  if (threadIdx.x < NA) orb[threadIdx.x] = spaces[k].orb[threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < NA * np; e += blockDim.x) {
    const int a = e / np, t = e % np, p = orb[a];
    double s = 0.0;   // sigma1(p,t)
    if (t < n) {
      if (p < o && t >= o) s = -t1[p * v + (t - o)];
      if (p >= o && t < o) s = t1[t * v + (p - o)];
    }
    S[e] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int col = lane % 16, kq = lane / 16;   // operand column (a) and k slot
  for (int tile = wave; tile < NT; tile += (int)blockDim.x / 64) {
    const int row = tile * 16 + col;   // this lane's A row (b,c,d)
    const bool live = row < N3;
    size_t off = 0;
    // Yg's two-body part vanishes unless its class pattern is within one
    // index of (v,v,o,o) or (o,o,v,v): which classes of t its row admits
    bool y_occ = false, y_vir = false;
    if (live) {
      const int b = row / N2, c = row / NA % NA, d = row % NA;
      off = (((size_t)orb[d] * n + orb[c]) * n + orb[b]) * n;
      const int qrs = (b < NO) << 2 | (c < NO) << 1 | (d < NO);   // occupied bits
      auto near = [&](int pat) {   // pat: occupied bits of (t, q, r, s)
        return __builtin_popcount(pat ^ 0x3) <= 1 || __builtin_popcount(pat ^ 0xC) <= 1;
      };
      y_occ = near(8 | qrs);
      y_vir = near(qrs);
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int t0 = 0; t0 < np; t0 += 4 * W) {
      const int t = t0 + W * kq;   // this lane's W consecutive t (all < n or all >= n)
      const bool in = live && t < n;
      dw ah, ay;
#pragma unroll
      for (int w = 0; w < W; ++w) ah[w] = ay[w] = 0.0;
      if (in) {
        ah = *reinterpret_cast<const dw*>(Xh + off + t);
        bool any = false;
#pragma unroll
        for (int w = 0; w < W; ++w) any = any || (t + w < o ? y_occ : y_vir);
        if (any) {   // structural zeros of Yg are not read
          ay = *reinterpret_cast<const dw*>(Xy + off + t);
#pragma unroll
          for (int w = 0; w < W; ++w)
            if (!(t + w < o ? y_occ : y_vir)) ay[w] = 0.0;
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const double sb = col < NA ? S[col * np + t + w] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ah[w], sb, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[w], 0.5 * sb, acc, 0, 0, 0);
      }
    }
    // lane holds D[row kq + 4r][column col]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = tile * 16 + kq + 4 * r;
      if (orow < N3 && col < NA) Z[col * N3 + orow] = acc[r];
    }
  }
  __syncthreads();
  double* slot = heff + heff_off[k] + 1 + N2;
  double* zk = zs ? zs + (size_t)blockIdx.x * (N2 * N2) : nullptr;
  for (int e = threadIdx.x; e < N2 * N2; e += blockDim.x) {
    const int a = e / N3, b = e / N2 % NA, c = e / NA % NA, d = e % NA;
    const double z = Z[a * N3 + (b * NA + c) * NA + d] + Z[b * N3 + (a * NA + d) * NA + c] +
                     Z[c * N3 + (d * NA + a) * NA + b] + Z[d * N3 + (c * NA + b) * NA + a];
    if (zk)
      zk[e] = -z;
    else
      slot[e] -= z;
  }
}

// The occupied-pair ladders of [H_N, sigma] + [Yg, sigma]/2 that have no
// global precomputed form, on the space's two-body block: with X = H_N + Yg/2,
//   M[(p,q)][(r,s)] = sum_{t,u occupied} X(p,q,t,u) t2[t,u,r,s]   (r,s virtual)
// (orbital indices of the space, all t,u), the element (p,q,r,s) gains
//   M[(p,q)][(r,s)]  when r,s are virtual and p,q not both occupied, and
//   M[(r,s)][(p,q)]  when p,q are virtual and r,s not both occupied
// (the second by X(t,u,r,s) = X(r,s,t,u)); the assignment is the same on every
// member of an element's symmetry orbit.  The (t,u) pairs are staged in
// chunks: X rows [NA^2][chunk] and t2 [chunk][NV^2] in LDS; the product runs
// on the matrix cores (v_mfma_f64_16x16x4f64), wavefront w taking rows
// [16w, 16w + 16) of M (NA^2 <= 64 rows, NV^2 <= 16 columns).
// With mpd (the dense form, for large space counts) M is read from
// mpd[tri(p,q)][(r,s)] = sum_{t,u occ} X(p,q,t,u) t2[t,u,r,s] (rows p <= q;
// M(q,p,s,r) = M(p,q,r,s) by the pair symmetry of X and t2) instead.
// With zs the block adds its part to zs[blockIdx.x][NA^4] (writes it when
// zs_init, i.e. when no k_heff_z wrote there first) instead of the slot.
template <int NA>
__global__ __launch_bounds__(256) void k_heff_pp(const double* __restrict__ Xh,
                                                 const double* __restrict__ Xy,
                                                 const double* __restrict__ t2,
                                                 const double* __restrict__ mpd,
                                                 const SpaceDev* __restrict__ spaces,
                                                 const int32_t* __restrict__ idx,
                                                 const int64_t* __restrict__ heff_off, int n,
                                                 int o, double* heff, double* zs, int zs_init) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NO = NA / 2, NV = NA - NO, N2 = NA * NA, NR = NV * NV, NM = N2 * NR;
  constexpr int kChunk = 64, NT = (N2 + 15) / 16;
  static_assert(NT <= 4 && NR <= 16, "one row tile per wavefront, one column tile");
  __shared__ double xs[N2 * kChunk];   // X(p,q,t,u), [pq][tu - c0]
  __shared__ double ts[kChunk * NR];   // t2[t,u,r,s], [tu - c0][rs]
  __shared__ double M[NM];
  __shared__ int orb[NA];
  const int k = idx[blockIdx.x];
  if (threadIdx.x < NA) orb[threadIdx.x] = spaces[k].orb[threadIdx.x];
  __syncthreads();
  const int v = n - o, oo = o * o;
  if (mpd) {
    for (int m = threadIdx.x; m < NM; m += blockDim.x) {
      const int p = orb[m / NR / NA], q = orb[m / NR % NA];
      const int r = orb[NO + m % NR / NV] - o, s = orb[NO + m % NV] - o;
      M[m] = p <= q ? mpd[tri_row(p, q, n) * v * v + (size_t)r * v + s]
                    : mpd[tri_row(q, p, n) * v * v + (size_t)s * v + r];
    }
  } else {
  const float inv_o = 1.0f / (float)o;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int row = wave * 16 + lane % 16, col = lane % 16, kq = lane / 16;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < oo; c0 += kChunk) {
    const int cn = min(kChunk, oo - c0);
    for (int e = threadIdx.x; e < N2 * kChunk; e += blockDim.x) {
      const int pq = e / kChunk, i = e % kChunk, tu = c0 + i;
      if (i >= cn) continue;
      // t = tu / o in single precision: (tu + 1/2) / o is at least 1/(2o)
      // from an integer, far beyond the rounding error for tu < 2^12
      const int t = (int)(((float)tu + 0.5f) * inv_o), u = tu - t * o;
      const size_t x = (((size_t)orb[pq / NA] * n + orb[pq % NA]) * n + t) * n + u;
      // Yg vanishes on (o,o,o,o): not read for p, q both occupied
      const bool y_on = pq / NA >= NO || pq % NA >= NO;
      xs[pq * kChunk + i] = Xh[x] + (y_on ? 0.5 * Xy[x] : 0.0);
    }
    for (int e = threadIdx.x; e < cn * NR; e += blockDim.x) {
      const int tu = c0 + e / NR, rs = e % NR;
      const int r = orb[NO + rs / NV] - o, s = orb[NO + rs % NV] - o;
      ts[e] = t2[((size_t)tu * v + r) * v + s];
    }
    __syncthreads();
    if (wave < NT)
      for (int k0 = 0; k0 < cn; k0 += 4) {
        const int k = k0 + kq;
        const double a = (row < N2 && k < cn) ? xs[row * kChunk + k] : 0.0;
        const double b = (col < NR && k < cn) ? ts[k * NR + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    __syncthreads();
  }
  // lane holds M[row 16w + kq + 4r][column col]
  if (wave < NT)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = wave * 16 + kq + 4 * r;
      if (orow < N2 && col < NR) M[orow * NR + col] = acc[r];
    }
  }
  __syncthreads();
  double* slot = heff + heff_off[k] + 1 + N2;
  double* zk = zs ? zs + (size_t)blockIdx.x * (N2 * N2) : nullptr;
  for (int e = threadIdx.x; e < N2 * N2; e += blockDim.x) {
    const int a = e / (N2 * NA), b = e / N2 % NA, c = e / NA % NA, d = e % NA;
    double x = 0.0;
    if (c >= NO && d >= NO && !(a < NO && b < NO))
      x += M[(a * NA + b) * NR + (c - NO) * NV + (d - NO)];
    if (a >= NO && b >= NO && !(c < NO && d < NO))
      x += M[(c * NA + d) * NR + (a - NO) * NV + (b - NO)];
    if (!zk)
      slot[e] += x;
    else if (zs_init)
      zk[e] = x;
    else
      zk[e] += x;
  }
}

// The one- and zero-body elements of part 2 (- 1/2 [E,sigma]): one
// wavefront per element (the pairs la <= lb, then the scalar), its terms
// split over the 64 lanes and summed; 512 threads per space.
template <int NA>
__global__ __launch_bounds__(512) void k_heff_low(const SpaceDev* __restrict__ spaces,
                                                  const int32_t* __restrict__ idx,
                                                  const int64_t* __restrict__ heff_off,
                                                  const double* __restrict__ tab,
                                                  int64_t tab_stride, int n, int o,
                                                  double* heff) {
  extern __shared__ double tl[];
  const int k = idx[blockIdx.x];
  int s1, s2, s3, s4;
  const int tot = mark_sizes(NA, &s1, &s2, &s3, &s4);
  const double* src = tab + (int64_t)k * tab_stride;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) tl[e] = src[e];
  __syncthreads();
  const MarkTables T{tl, tl + s1, tl + s1 + s2, tl + s1 + s2 + s3, NA};
  const MarkedE<NA> E{T};
  const MarkedSigma<NA> D{T};
  const MarkedShape<NA> shape;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  CommE<MarkedE<NA>, MarkedSigma<NA>, true, MarkedShape<NA>> ce{E, D, shape, n, o};
  ce.ln = lane;
  ce.nl = 64;
  double* slot = heff + heff_off[k];
  constexpr int npairs = NA * (NA + 1) / 2;
  for (int e = wave; e <= npairs; e += blockDim.x / 64) {
    int la = 0, lb = 0;
    if (e < npairs) {   // the e-th pair la <= lb
      int r = e;
      while (r >= NA - la) {
        r -= NA - la;
        ++la;
      }
      lb = la + r;
    }
    const double x = wave_sum(e < npairs ? ce.c1(la, lb) : ce.c0());
    if (lane == 0) {
      if (e < npairs) {
        slot[1 + la * NA + lb] += -0.5 * x;
        if (la != lb) slot[1 + lb * NA + la] += -0.5 * x;
      } else {
        slot[0] += -0.5 * x;
      }
    }
  }
}

// The two-body parts that k_heff_z and k_heff_pp leave in a buffer of their
// own: class c's block i at p + off[c] + i * na^4, its spaces the ones at
// [first[c], first[c + 1]) of the list (p NULL: none).
struct ZSum {
  const double* p;
  long long off[3];
  int first[3];
};

// Rewrite each slot from normal order to CAS form (after adding the ZSum
// part to the two-body block and, when given, the extra terms xtra at the
// slot's offset to every part):
//   Ec = x0 - 2 sum_k x1_kk + sum_kl (2 x2_klkl - x2_kllk)
//   h_pq = x1_pq - sum_k (2 x2_pkqk - x2_pkkq),  g(pq|rs) = x2_prqs
__global__ __launch_bounds__(256) void k_heff_cas(const SpaceDev* __restrict__ spaces,
                                                  const int32_t* __restrict__ idx,
                                                  const int64_t* __restrict__ heff_off,
                                                  ZSum zsum, const double* __restrict__ xtra,
                                                  double* heff) {
  extern __shared__ double sm[];
  const int k = idx[blockIdx.x];
  const SpaceDev sp = spaces[k];
  const int na = sp.na, ne = sp.nocc, n2 = na * na, n4 = n2 * n2;
  double* slot = heff + heff_off[k];
  const double* zk = nullptr;
  if (zsum.p) {
    const int c = ne - 2;   // size class: na = 2 nocc
    zk = zsum.p + zsum.off[c] + (size_t)(blockIdx.x - zsum.first[c]) * n4;
  }
  const double* xk = xtra ? xtra + heff_off[k] : nullptr;
  for (int e = threadIdx.x; e < 1 + n2 + n4; e += blockDim.x)
    sm[e] = (zk && e > n2 ? slot[e] + zk[e - 1 - n2] : slot[e]) + (xk ? xk[e] : 0.0);
  __syncthreads();
  const double* x1 = sm + 1;
  const double* x2 = sm + 1 + n2;
  for (int e = threadIdx.x; e < n4; e += blockDim.x) {
    const int s = e % na, r = e / na % na, q = e / n2 % na, p = e / (n2 * na);
    slot[1 + n2 + e] = x2[((p * na + r) * na + q) * na + s];
  }
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    const int p = e / na, q = e % na;
    double h = x1[e];
    for (int kk = 0; kk < ne; ++kk)
      h -= 2.0 * x2[((p * na + kk) * na + q) * na + kk] - x2[((p * na + kk) * na + kk) * na + q];
    slot[1 + e] = h;
  }
  if (threadIdx.x == 0) {
    double ec = sm[0];
    for (int kk = 0; kk < ne; ++kk) ec -= 2.0 * x1[kk * na + kk];
    for (int kk = 0; kk < ne; ++kk)
      for (int l = 0; l < ne; ++l)
        ec += 2.0 * x2[((kk * na + l) * na + kk) * na + l] - x2[((kk * na + l) * na + l) * na + kk];
    slot[0] = ec;
  }
}

}  // namespace

void launch_pack_x_pairs(const double* Xh, const double* Xy, int n, int o, double* xp,
                         hipStream_t st) {
  k_pack_x_pairs<<<grid_for((size_t)n * (n + 1) / 2 * o * o, kBlock, 65536), kBlock, 0, st>>>(
      Xh, Xy, n, o, xp);
}

// per space: the marked tables, then H_N and Yg restricted to the space
int heff_table_stride(int na_max) {
  int s1, s2, s3, s4;
  const int n2 = na_max * na_max;
  return mark_sizes(na_max, &s1, &s2, &s3, &s4) + 2 * (n2 + n2 * n2);
}

int heff_lds_doubles(int na) {
  int s1, s2, s3, s4;
  const int n2 = na * na;
  const int mark = mark_sizes(na, &s1, &s2, &s3, &s4);
  return std::max(mark, std::max(2 * (n2 + n2 * n2), n2 * n2 + n2 + 1));
}

namespace {
template <class Kern>
void allow_lds(Kern* kern, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
}  // namespace

hipError_t launch_heff(const double* f, const double* V, const double* y1, const double* y2,
                       const double* L, const double* LY, const RingOps& rings, const double* t1,
                       const double* t2, int n,
                       int o, const double* scal, const SpaceDev* spaces, const int64_t* heff_off,
                       const int32_t* task_table, int task_stride, const int* task_slots,
                       const int32_t* cls_idx, const int* cls_off, int K, int na_max,
                       double* tab, double* fs1, const double* zc, const double* mpd, double* heff,
                       hipStream_t st, double* zs, hipStream_t st2, hipEvent_t fork_ev,
                       hipEvent_t join_ev, int phase, const double* xtra) {
  GlobalOps g{f, V, y1, y2, L, LY, t1, t2, n, o, rings.ga_h, rings.g22_h, rings.j1_h,
              rings.j2_h, rings.ga_y, rings.g22_y, rings.j1_y, rings.j2_y,
              rings.zv,   rings.zo,  rings.u_h, rings.s2p, rings.s2q, rings.c1_h, rings.c1_y,
              rings.lo_h, rings.lo_y, rings.pf};
  g.zc = zc;
  g.qf = rings.qf;
  g.fs1 = fs1;
  const int tab_stride = heff_table_stride(na_max);
  // the tables (phase 0) read only prepare's outputs, f and t1
  if (phase != 1) {
    k_fs1<<<(2 * n * n + kBlock - 1) / kBlock, kBlock, 0, st>>>(f, t1, n, o, fs1);
    for (int c = 0; c < 3; ++c) {
      const int count = cls_off[c + 1] - cls_off[c];
      if (count <= 0) continue;
      const int32_t* idx = cls_idx + cls_off[c];
      if (c == 0) k_heff_tab<4><<<count, kBlock, 0, st>>>(g, spaces, idx, tab, tab_stride);
      if (c == 1) k_heff_tab<6><<<count, kBlock, 0, st>>>(g, spaces, idx, tab, tab_stride);
      if (c == 2) k_heff_tab<8><<<count, kBlock, 0, st>>>(g, spaces, idx, tab, tab_stride);
    }
  }
  if (phase == 0) return hipSuccess;
  // k_heff_z and k_heff_pp read only the operators, t1, t2 and mpd: with zs
  // they write there (k_heff_cas adds it), on st2 when given, beside the
  // table and element kernels
  ZSum zsum{nullptr, {0, 0, 0}, {0, 0, 0}};
  const bool use_zs = zs != nullptr, fork = use_zs && st2 != nullptr;
  if (use_zs) {
    long long acc = 0;
    for (int c = 0; c < 3; ++c) {
      const long long na = 2 * (c + 2);
      zsum.off[c] = acc;
      zsum.first[c] = cls_off[c];
      acc += (long long)(cls_off[c + 1] - cls_off[c]) * na * na * na * na;
    }
    zsum.p = zs;
  }
  if (fork) {
    hipError_t e = hipEventRecord(fork_ev, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st2, fork_ev, 0);
    if (e != hipSuccess) return e;
  }
  // per class: the sigma1 x two-body part (per-space form) and the
  // occupied-pair ladders, into zs when given, else into the slots
  auto z_pp = [&](hipStream_t s) {
    for (int c = 0; c < 3; ++c) {
      const int count = cls_off[c + 1] - cls_off[c];
      if (count <= 0) continue;
      const int na = 2 * (c + 2);
      const int32_t* idx = cls_idx + cls_off[c];
      double* zsc = use_zs ? zs + zsum.off[c] : nullptr;
      const int init = zc != nullptr;   // no k_heff_z wrote zs first
      // W = 2 (16-byte row loads) needs even n: rows then start 16-byte
      // aligned and a lane's pair of t never straddles n
      const bool w2 = n % 2 == 0;
      const size_t zlds = (size_t)(na * ((n + 7) & ~7) + na * na * na * na) * sizeof(double);
      if (c == 0) {
        if (!zc && w2) k_heff_z<4, 2><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        if (!zc && !w2) k_heff_z<4, 1><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        k_heff_pp<4><<<count, 256, 0, s>>>(V, y2, t2, mpd, spaces, idx, heff_off, n, o, heff, zsc, init);
      } else if (c == 1) {
        if (!zc && w2) k_heff_z<6, 2><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        if (!zc && !w2) k_heff_z<6, 1><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        k_heff_pp<6><<<count, 256, 0, s>>>(V, y2, t2, mpd, spaces, idx, heff_off, n, o, heff, zsc, init);
      } else {
        if (!zc && w2) k_heff_z<8, 2><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        if (!zc && !w2) k_heff_z<8, 1><<<count, 256, zlds, s>>>(V, y2, t1, spaces, idx, heff_off, n, o, heff, zsc);
        k_heff_pp<8><<<count, 256, 0, s>>>(V, y2, t2, mpd, spaces, idx, heff_off, n, o, heff, zsc, init);
      }
    }
  };
  if (fork) {
    z_pp(st2);
    const hipError_t e = hipEventRecord(join_ev, st2);
    if (e != hipSuccess) return e;
  } else if (use_zs) {
    z_pp(st);
  }
  // parts 0, 1, 2 per size class: its task count and LDS.  The (4,4) class
  // (about 100 KB of staged tables) runs 1024-thread workgroups, so that its
  // tables are staged twice per space instead of five times and four times
  // as many wavefronts share them; the others run 256-thread workgroups.
  // Workgroup x takes a space, y a chunk of tasks, x fastest: the chunks of
  // one space never run together (they update the same output lines).
  for (int PART = 0; PART < 3; ++PART)
    for (int c = 0; c < 3; ++c) {
      const int count = cls_off[c + 1] - cls_off[c];
      if (count <= 0) continue;
      const int na = 2 * (c + 2), n2 = na * na;
      int s1, s2, s3, s4;
      const int mark = mark_sizes(na, &s1, &s2, &s3, &s4);
      const size_t lds = (size_t)(PART == 2 ? mark : 2 * (n2 + n2 * n2)) * sizeof(double);
      const int32_t* idx = cls_idx + cls_off[c];
      // part 2 (two-body elements only) covers the two-body slots
      const int slots = PART == 2 ? task_slots[3 + c] : task_slots[c];
      if (c == 2) {
        const dim3 grid(count, (slots + 1023) / 1024);
        if (PART == 0) {
          allow_lds(&k_heff_part<0, 1024, 0>, lds);
          k_heff_part<0, 1024, 0><<<grid, 1024, lds, st>>>(g, scal, spaces, idx, heff_off, task_table,
                                                        task_stride, tab, tab_stride, heff);
        } else if (PART == 1) {
          allow_lds(&k_heff_part<1, 1024, 0>, lds);
          k_heff_part<1, 1024, 0><<<grid, 1024, lds, st>>>(g, scal, spaces, idx, heff_off, task_table,
                                                        task_stride, tab, tab_stride, heff);
        } else {
          allow_lds(&k_heff_part<2, 1024, 8>, lds);
          k_heff_part<2, 1024, 8><<<grid, 1024, lds, st>>>(g, scal, spaces, idx, heff_off, task_table,
                                                        task_stride, tab, tab_stride, heff);
        }
        continue;
      }
      const dim3 grid(count, (slots + kBlock - 1) / kBlock);
      if (PART == 0)
        k_heff_part<0, 256, 0><<<grid, kBlock, lds, st>>>(g, scal, spaces, idx, heff_off,
                                                          task_table, task_stride, tab, tab_stride,
                                                          heff);
      else if (PART == 1)
        k_heff_part<1, 256, 0><<<grid, kBlock, lds, st>>>(g, scal, spaces, idx, heff_off,
                                                          task_table, task_stride, tab, tab_stride,
                                                          heff);
      else if (c == 0)
        k_heff_part<2, 256, 4><<<grid, kBlock, lds, st>>>(g, scal, spaces, idx, heff_off,
                                                          task_table, task_stride, tab, tab_stride,
                                                          heff);
      else
        k_heff_part<2, 256, 6><<<grid, kBlock, lds, st>>>(g, scal, spaces, idx, heff_off,
                                                          task_table, task_stride, tab, tab_stride,
                                                          heff);
    }
  for (int c = 0; c < 3; ++c) {
    const int count = cls_off[c + 1] - cls_off[c];
    if (count <= 0) continue;
    const int na = 2 * (c + 2);
    int s1, s2, s3, s4;
    const size_t lds = (size_t)mark_sizes(na, &s1, &s2, &s3, &s4) * sizeof(double);
    const int32_t* idx = cls_idx + cls_off[c];
    if (c == 0) {
      k_heff_low<4><<<count, 512, lds, st>>>(spaces, idx, heff_off, tab, tab_stride, n, o, heff);
    } else if (c == 1) {
      k_heff_low<6><<<count, 512, lds, st>>>(spaces, idx, heff_off, tab, tab_stride, n, o, heff);
    } else {
      allow_lds(&k_heff_low<8>, lds);
      k_heff_low<8><<<count, 512, lds, st>>>(spaces, idx, heff_off, tab, tab_stride, n, o, heff);
    }
  }
  if (fork) {
    const hipError_t e = hipStreamWaitEvent(st, join_ev, 0);
    if (e != hipSuccess) return e;
  } else if (!use_zs) {
    z_pp(st);
  }
  const int tasks = na_max * na_max * na_max * na_max + na_max * na_max + 1;
  const size_t lds = (size_t)tasks * sizeof(double);
  k_heff_cas<<<K, kBlock, lds, st>>>(spaces, cls_idx, heff_off, zsum, xtra, heff);
  return hipSuccess;
}

}  // namespace qf
