// Host implementation of Algorithm 1 (coverage-driven active-space sampling)
// and of amplitude ownership ("each excitation belongs to the first space,
// in energy order, that reaches it").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/qflow.h"

namespace {

// partial Fisher-Yates: k of 0..N-1, one uniform per swap; sorted result
bool draw(int N, int k, const double* u, int64_t n_u, int64_t* pos, std::vector<int>& idx,
          int* out) {
  if (*pos + k > n_u) return false;
  idx.resize(N);
  std::iota(idx.begin(), idx.end(), 0);
  for (int m = 0; m < k; ++m) {
    const int j = m + (int)std::floor(u[(*pos)++] * (double)(N - m));
    std::swap(idx[m], idx[j]);
  }
  std::copy(idx.begin(), idx.begin() + k, out);
  std::sort(out, out + k);
  return true;
}

}  // namespace

extern "C" {

int qflow_sample_spaces(int32_t No, int32_t Nv, int32_t no, int32_t nv, const double* eps,
                        const double* u, int64_t n_u, int32_t cap, qflow_space* out,
                        double* delta_eps, int32_t max_out, int32_t* K_out, int64_t* used) {
  if (No < 2 || Nv < 2 || no < 2 || nv < 2 || no > No || nv > Nv || no + nv > 8 || !eps ||
      !u || !out || !delta_eps || !K_out || !used || max_out < 0)
    return QFLOW_E_INVALID_ARG;
  const int64_t npo = (int64_t)No * (No - 1) / 2, npv = (int64_t)Nv * (Nv - 1) / 2;
  auto pair = [](int a, int b, int N) {   // index of (a<b) in the upper triangle
    return (int64_t)a * (2 * N - a - 1) / 2 + (b - a - 1);
  };
  std::vector<uint8_t> remaining(npo * npv, 1);
  int64_t left = npo * npv, pos = 0;
  struct Cand {
    int o[4], v[4];
    double de;
  };
  std::vector<Cand> S;
  std::vector<int> scratch;
  while (left > 0 && (cap <= 0 || (int)S.size() < cap)) {
    Cand c{};
    if (!draw(No, no, u, n_u, &pos, scratch, c.o) || !draw(Nv, nv, u, n_u, &pos, scratch, c.v)) {
      *used = pos;
      return QFLOW_E_INVALID_ARG;   // uniforms exhausted
    }
    bool any = false;
    for (int a = 0; a < no; ++a)
      for (int b = a + 1; b < no; ++b)
        for (int x = 0; x < nv; ++x)
          for (int y = x + 1; y < nv; ++y) {
            const int64_t t = pair(c.o[a], c.o[b], No) * npv + pair(c.v[x], c.v[y], Nv);
            if (remaining[t]) {
              remaining[t] = 0;
              --left;
              any = true;
            }
          }
    if (!any) continue;
    double sv = 0.0, so = 0.0;
    for (int x = 0; x < nv; ++x) sv += eps[No + c.v[x]];
    for (int a = 0; a < no; ++a) so += eps[c.o[a]];
    c.de = sv - so;
    S.push_back(c);
  }
  std::stable_sort(S.begin(), S.end(), [&](const Cand& a, const Cand& b) {
    if (a.de != b.de) return a.de < b.de;
    for (int i = 0; i < no; ++i)
      if (a.o[i] != b.o[i]) return a.o[i] < b.o[i];
    for (int i = 0; i < nv; ++i)
      if (a.v[i] != b.v[i]) return a.v[i] < b.v[i];
    return false;
  });
  if ((int64_t)S.size() > max_out) {
    *used = pos;
    return QFLOW_E_INVALID_ARG;
  }
  for (size_t k = 0; k < S.size(); ++k) {
    qflow_space s{};
    s.n_o = no;
    s.n_v = nv;
    for (int a = 0; a < no; ++a) s.orb[a] = S[k].o[a];
    for (int x = 0; x < nv; ++x) s.orb[no + x] = No + S[k].v[x];
    out[k] = s;
    delta_eps[k] = S[k].de;
  }
  *K_out = (int32_t)S.size();
  *used = pos;
  return QFLOW_OK;
}

int qflow_build_owners(int32_t No, int32_t Nv, int32_t K, const qflow_space* spaces,
                       int32_t* owner1, int32_t* owner2) {
  if (No < 1 || Nv < 1 || K < 0 || (K > 0 && !spaces) || !owner1 || !owner2)
    return QFLOW_E_INVALID_ARG;
  std::fill(owner1, owner1 + (size_t)No * Nv, -1);
  std::fill(owner2, owner2 + (size_t)No * No * Nv * Nv, -1);
  for (int k = 0; k < K; ++k) {
    const qflow_space& s = spaces[k];
    if (s.n_o < 1 || s.n_v < 1 || s.n_o + s.n_v > 8) return QFLOW_E_INVALID_ARG;
    for (int a = 0; a < s.n_o + s.n_v; ++a) {
      const int p = s.orb[a];
      if (a < s.n_o ? (p < 0 || p >= No) : (p < No || p >= No + Nv)) return QFLOW_E_INVALID_ARG;
    }
    for (int i = 0; i < s.n_o; ++i)
      for (int a = 0; a < s.n_v; ++a) {
        int32_t& w = owner1[(size_t)s.orb[i] * Nv + (s.orb[s.n_o + a] - No)];
        if (w < 0) w = k;
      }
    for (int i = 0; i < s.n_o; ++i)
      for (int j = 0; j < s.n_o; ++j)
        for (int a = 0; a < s.n_v; ++a)
          for (int b = 0; b < s.n_v; ++b) {
            const size_t g = (((size_t)s.orb[i] * No + s.orb[j]) * Nv + (s.orb[s.n_o + a] - No)) *
                                 Nv + (s.orb[s.n_o + b] - No);
            if (owner2[g] < 0) owner2[g] = k;
          }
  }
  return QFLOW_OK;
}

}  // extern "C"
