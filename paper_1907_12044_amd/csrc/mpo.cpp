// Frenkel-Holstein MPO (Sec. II.C, eq:holstein; MPO form eq:mpo) built on the
// host from the model parameters.  Finite-state construction with
// complementary operators for the all-to-all exciton coupling: on a bond with
// k electronic sites to its left and n_e - k to its right the hopping terms
// are carried either by 2k channels a+_j, a_j (one per left site j, closed
// by J_jm a_m or J_mj a+_m at a right site m) or, once k > n_e - k, by
// 2(n_e - k) channels sum_j J_jn a+_j and sum_j J_nj a_j (one per right site
// n, closed by a_n or a+_n at n).  The switch happens at one electronic site,
// where each left channel feeds every right channel with weight J.  Inside
// the mode block of electronic site m one more channel carries n_m to the
// modes' g w (b+ + b) terms.  Bond dimension 2 + 2 min(k, n_e - k) + [mode block].
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/tdvp.h"

namespace {

enum ChanType { READY = 0, DONE = 1, CRE = 2, ANN = 3, RCRE = 4, RANN = 5, NUM = 6 };

struct Chan {
  int type, idx;
  bool operator==(const Chan &o) const { return type == o.type && idx == o.idx; }
};

struct Chain {
  int n, n_e;
  const int32_t *kind, *owner, *phys;
};

std::vector<Chan> channels(const Chain &c, int b) {
  std::vector<Chan> ch;
  if (b == 0) { ch.push_back({READY, 0}); return ch; }
  if (b == c.n) { ch.push_back({DONE, 0}); return ch; }
  ch.push_back({READY, 0});
  int k = 0;
  for (int i = 0; i < b; ++i) k += (c.kind[i] == 0);
  const int kr = c.n_e - k;
  if (k > 0 && kr > 0) {
    if (k <= kr) {
      for (int i = 0; i < b; ++i)
        if (c.kind[i] == 0) { ch.push_back({CRE, c.owner[i]}); ch.push_back({ANN, c.owner[i]}); }
    } else {
      for (int i = b; i < c.n; ++i)
        if (c.kind[i] == 0) { ch.push_back({RCRE, c.owner[i]}); ch.push_back({RANN, c.owner[i]}); }
    }
  }
  if (c.kind[b] == 1 && c.owner[b] == c.owner[b - 1]) ch.push_back({NUM, c.owner[b]});
  ch.push_back({DONE, 0});
  return ch;
}

int find(const std::vector<Chan> &v, Chan c) {
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i] == c) return (int)i;
  return -1;
}

typedef std::vector<double> Op;   // d x d complex stored as real (all operators are real)

Op eye(int d) { Op o(d * d, 0.0); for (int i = 0; i < d; ++i) o[i * d + i] = 1.0; return o; }
Op lower(int d) {   // a / b : |k-1><k| sqrt(k)
  Op o(d * d, 0.0);
  for (int k = 1; k < d; ++k) o[(k - 1) * d + k] = std::sqrt((double)k);
  return o;
}
Op raise(int d) {   // a+ / b+ : |k><k-1| sqrt(k)
  Op o(d * d, 0.0);
  for (int k = 1; k < d; ++k) o[k * d + (k - 1)] = std::sqrt((double)k);
  return o;
}
Op number(int d) { Op o(d * d, 0.0); for (int k = 0; k < d; ++k) o[k * d + k] = (double)k; return o; }

}  // namespace

extern "C" tdvp_status tdvp_holstein_mpo(int n, const int32_t *kind, const int32_t *owner,
                                         const int32_t *phys, int n_e, const double *eps,
                                         const double *J, const double *w, const double *g,
                                         int32_t *bond_out, int64_t *total_elems, double *W_out) {
  if (n <= 0 || !kind || !owner || !phys || !bond_out || !total_elems) return TDVP_E_ARG;
  if (n_e < 0) return TDVP_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (kind[i] != 0 && kind[i] != 1) return TDVP_E_ARG;
    if (owner[i] < 0 || owner[i] >= (n_e > 0 ? n_e : 1)) return TDVP_E_ARG;
    if (phys[i] < 1 || (kind[i] == 0 && phys[i] != 2)) return TDVP_E_SHAPE;
    if (kind[i] == 1 && (i == 0 || owner[i - 1] != owner[i])) return TDVP_E_SHAPE;
  }
  Chain c{n, n_e, kind, owner, phys};
  std::vector<std::vector<Chan>> ch(n + 1);
  int64_t total = 0;
  for (int b = 0; b <= n; ++b) {
    ch[b] = channels(c, b);
    bond_out[b] = (int32_t)ch[b].size();
  }
  for (int i = 0; i < n; ++i)
    total += (int64_t)ch[i].size() * phys[i] * phys[i] * ch[i + 1].size();
  *total_elems = total;
  if (!W_out) return TDVP_OK;
  if (!eps || (n_e > 0 && !J) || !w || !g) return TDVP_E_ARG;

  double *out = W_out;
  for (int i = 0; i < n; ++i) {
    const int d = phys[i];
    const std::vector<Chan> &L = ch[i], &R = ch[i + 1];
    const int Wl = (int)L.size(), Wr = (int)R.size();
    const int64_t sz = (int64_t)Wl * d * d * Wr;
    std::memset(out, 0, sizeof(double) * 2 * sz);
    auto put = [&](Chan lc, Chan rc, double coef, const Op &op) {
      const int a = find(L, lc), b = find(R, rc);
      if (a < 0 || b < 0 || coef == 0.0) return;
      for (int so = 0; so < d; ++so)
        for (int si = 0; si < d; ++si) {
          const double v = op[so * d + si];
          if (v == 0.0) continue;
          const int64_t idx = (((int64_t)a * d + so) * d + si) * Wr + b;
          out[2 * idx] += coef * v;
        }
    };
    const Op I = eye(d), lo = lower(d), up = raise(d), nm = number(d);
    const Chan ready{READY, 0}, done{DONE, 0};
    put(ready, ready, 1.0, I);
    put(done, done, 1.0, I);
    if (kind[i] == 0) {
      const int m = owner[i];
      put(ready, done, eps[m], nm);
      put(ready, Chan{NUM, m}, 1.0, nm);
      // open: site m joins the left part
      put(ready, Chan{CRE, m}, 1.0, up);
      put(ready, Chan{ANN, m}, 1.0, lo);
      for (const Chan &rc : R) {
        if (rc.type == RCRE) put(ready, rc, J[m * n_e + rc.idx], up);   // J_mn a+_m
        if (rc.type == RANN) put(ready, rc, J[rc.idx * n_e + m], lo);   // J_nm a_m
      }
      for (const Chan &lc : L) {
        if (lc.type == CRE) {
          const int j = lc.idx;
          put(lc, lc, 1.0, I);                                   // pass through
          put(lc, done, J[j * n_e + m], lo);                      // J_jm a+_j a_m
          for (const Chan &rc : R)
            if (rc.type == RCRE) put(lc, rc, J[j * n_e + rc.idx], I);
        } else if (lc.type == ANN) {
          const int j = lc.idx;
          put(lc, lc, 1.0, I);
          put(lc, done, J[m * n_e + j], up);                      // J_mj a+_m a_j
          for (const Chan &rc : R)
            if (rc.type == RANN) put(lc, rc, J[rc.idx * n_e + j], I);
        } else if (lc.type == RCRE) {
          if (lc.idx == m) put(lc, done, 1.0, lo);
          else put(lc, lc, 1.0, I);
        } else if (lc.type == RANN) {
          if (lc.idx == m) put(lc, done, 1.0, up);
          else put(lc, lc, 1.0, I);
        }
      }
    } else {
      const int m = owner[i];
      put(ready, done, w[i], nm);
      for (const Chan &lc : L)
        if (lc.type == CRE || lc.type == ANN || lc.type == RCRE || lc.type == RANN) put(lc, lc, 1.0, I);
      Op x(d * d);
      for (int q = 0; q < d * d; ++q) x[q] = lo[q] + up[q];
      put(Chan{NUM, m}, done, g[i] * w[i], x);
      put(Chan{NUM, m}, Chan{NUM, m}, 1.0, I);
    }
    out += 2 * sz;
  }
  return TDVP_OK;
}
