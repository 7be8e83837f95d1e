// QR of a tall complex matrix by shifted Cholesky QR in three passes, for
// the gauge shifts of the sweep at larger bond dimension (eq:QR), where one
// work-group's Householder QR runs out of LDS and parallelism.  The method
// is the published shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa,
// Yamamoto, Yanagisawa: "Shifted Cholesky QR for computing the QR
// factorization of ill-conditioned matrices", SIAM J. Sci. Comput. 42
// (2020)), whose shift rule is used unchanged; the kernels are this
// library's own.
//
// Pass p (W_0 = A):  G = W_p^H W_p  (MFMA);  R_p = chol(G [+ s I])  with
// G = R_p^H R_p, diag(R_p) > 0;  W_{p+1} = W_p R_p^{-1}  (GEMM).
// The first pass adds the shift s = 11 (m n + n (n + 1)) u tr(G) (u the
// unit round-off), which keeps the Cholesky factorisation defined up to a
// condition number ~1/u; the next two passes restore orthogonality to
// round-off.  Q = W_3, R = R_3 R_2 R_1: upper triangular with real positive
// diagonal, i.e. the same factorisation (C = L D with diag(D) real >= 0) that
// the Householder paths produce, unique for full-rank input.
//
// Kernels: cq_prep (A through strides / conjugation into W_0), per pass
// cq_gram (upper 16x16 tiles of G, K split over the 16 waves of a
// work-group), cq_chol (one work-group: blocked Cholesky and block-triangular
// inverse on the matrix cores) and cgemm for W R^{-1} and
// the running product of the R factors (the last ones write Q and R through
// the caller's strides).
// One cq_chol call factors n <= 128; up to n = 256 the factorisation is
// blocked 2 x 2 around two calls (see cholqr).
#include <utility>

#include "common.h"
#include "mfma.h"

namespace tdvp {

namespace {

constexpr int CQ_THREADS = 1024;
constexpr int CQ_NMAX = 128;

__global__ __launch_bounds__(256) void cq_prep_kernel(QrArgs p, double2 *W0, int64_t ws) {
  const int64_t inst = blockIdx.y;
  const double2 *A = p.A + inst * p.inst.a;
  W0 += inst * ws;
  const int64_t total = (int64_t)p.m * p.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / p.n, c = e - r * p.n;
    double2 v = A[r * p.a_rs + c * p.a_cs];
    if (p.conjA) v.y = -v.y;
    W0[e] = v;
  }
}

// G[i][j] = sum_k conj(W[k][i]) W[k][j] on the upper 16x16 tiles (tj >= ti);
// the 16 waves of a work-group take interleaved 4-row slices of k, and the
// wave results are added in order through LDS.
__global__ __launch_bounds__(CQ_THREADS) void cq_gram_kernel(const double2 *W, int m, int n,
                                                             double2 *G, int64_t ws) {
  const int64_t inst = blockIdx.y;
  W += inst * ws;
  G += inst * ws;
  const int nt = (n + 15) / 16;
  int t = blockIdx.x, ti = 0;
  while (t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = ti * 16 + (lane & 15), j = tj * 16 + (lane & 15);
  f64x4_t cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  for (int k0 = 4 * wave; k0 < m; k0 += 4 * (CQ_THREADS / 64)) {
    const int k = k0 + (lane >> 4);
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (k < m) {
      if (i < n) a = W[(int64_t)k * n + i];
      if (j < n) b = W[(int64_t)k * n + j];
    }
    // conj(a) * b
    cr = Mf<double>::mfma(a.x, b.x, cr);
    cr = Mf<double>::mfma(a.y, b.y, cr);
    ci = Mf<double>::mfma(a.x, b.y, ci);
    ci = Mf<double>::mfma(-a.y, b.x, ci);
  }
  // waves 8..15 park their results, waves 0..7 add them to their own, then
  // 8 partial tiles are added in order (32 KiB of LDS)
  __shared__ double red[8][2][256];
  if (wave >= 8) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[wave - 8][0][r * 64 + lane] = cr[r];
      red[wave - 8][1][r * 64 + lane] = ci[r];
    }
  }
  __syncthreads();
  if (wave < 8) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[wave][0][r * 64 + lane] += cr[r];
      red[wave][1][r * 64 + lane] += ci[r];
    }
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const int r = threadIdx.x >> 6, ln = threadIdx.x & 63;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < 8; ++w) {
      sr += red[w][0][r * 64 + ln];
      si += red[w][1][r * 64 + ln];
    }
    const int gi = ti * 16 + Mf<double>::row(ln, r), gj = tj * 16 + (ln & 15);
    if (gi < n && gj < n) G[(int64_t)gi * n + gj] = make_double2(sr, si);
  }
}

__device__ __forceinline__ double2 shfl_c(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// 16x16 complex blocks in LDS: element (i, j) at i * 16 + (j ^ i), so that
// sixteen lanes reading a row or a column touch sixteen different banks.
__device__ __forceinline__ int bo(int i, int j) { return (i << 4) | (j ^ i); }

// acc += op(A) B on the matrix cores of one wave, op(A) = A^H when adj, with
// three real products per complex one: P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2.
struct CAcc {
  f64x4_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
  __device__ double re(int r) const { return p1[r] - p2[r]; }
  __device__ double im(int r) const { return p3[r] - p1[r] - p2[r]; }
};
__device__ __forceinline__ void blk_mma(const double2 *A, bool adj, const double2 *B, CAcc &acc) {
  const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const int k = k0 + kk;
    double2 av = adj ? A[bo(k, i)] : A[bo(i, k)];
    if (adj) av.y = -av.y;
    const double2 bv = B[bo(k, i)];
    acc.p1 = Mf<double>::mfma(av.x, bv.x, acc.p1);
    acc.p2 = Mf<double>::mfma(av.y, bv.y, acc.p2);
    acc.p3 = Mf<double>::mfma(av.x + av.y, bv.x + bv.y, acc.p3);
  }
}

// Cross-lane moves of one wave for the 16x16 diagonal block held as lane
// (g, c) = (lane / 16, lane % 16) <- rows g + 4 q of column c.
// value of lane l (l uniform), as a wave-uniform scalar
__device__ __forceinline__ double rd_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// lane (g, c) <- lane (g, K): DPP row_newbcast (every lane is written, so
// no old value is needed)
template <int K> __device__ __forceinline__ double nbc(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_mov_dpp((int)b, 0x150 + K, 0xF, 0xF, true);
  const unsigned hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + K, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int K> __device__ __forceinline__ double2 nbc(double2 v) { return make_double2(nbc<K>(v.x), nbc<K>(v.y)); }
// lane (g, c) <- lane (gk, c): the 32-lane swap pairs rows (0, 1) with
// (2, 3), the 16-lane swap then row 0 with 1 and 2 with 3
__device__ __forceinline__ unsigned grp32(unsigned v, int gk) {
  const auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  const unsigned a = gk < 2 ? s[0] : s[1];
  const auto t = __builtin_amdgcn_permlane16_swap(a, a, false, false);
  return (gk & 1) ? t[1] : t[0];
}
__device__ __forceinline__ double grp(double v, int gk) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = grp32((unsigned)b, gk), hi = grp32((unsigned)(b >> 32), gk);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double2 grp(double2 v, int gk) { return make_double2(grp(v.x, gk), grp(v.y, gk)); }

// Step k of the one-wave factorisation of a 16x16 diagonal block.  Lane
// (g, c) holds column c of rows g + 4 q: d the Hermitian block being
// reduced, r the rows of R found so far.  Pivot p = D[k][k]; row k of R is
// D[k][c] / sqrt(p) (c > k), sqrt(p) (c == k), 0 (c < k); Schur complement
// D[i][c] -= D[i][k] D[k][c] / p.  The update runs unmasked: rows and
// columns <= k of d are never read again.  yk[k] = 1 / R[k][k].  k is a
// template argument so every lane move is an immediate-controlled DPP /
// swap and all registers are indexed statically.
template <int k> __device__ __forceinline__ void chol_step(double2 (&d)[4], double2 (&r)[4], double (&yk)[16],
                                                           int g, int c, double pmin) {
  constexpr int qk = k >> 2, gk = k & 3;
  double p = rd_lane(d[qk].x, 16 * gk + k);
  if (!(p > pmin)) p = pmin;                        // (numerically) singular: floor the pivot
  const double y = rsqrt_nr(p), ip = y * y;
  yk[k] = y;
  const double2 dkc = grp(d[qk], gk);               // D[k][c] in every row group
  {                                                 // row k of R (selects, no branch)
    const bool own = g == gk, above = c > k, diag = c == k;
    const double rx = above ? dkc.x * y : (diag ? p * y : 0.0);
    const double ry = above ? dkc.y * y : 0.0;
    r[qk].x = own ? rx : r[qk].x;
    r[qk].y = own ? ry : r[qk].y;
  }
  const double2 t = make_double2(dkc.x * ip, dkc.y * ip);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (4 * q + 3 > k) {                            // some row g + 4 q is below row k
      const double2 dik = nbc<k>(d[q]);             // D[i][k], i = g + 4 q
      d[q].x = fma(dik.y, t.y, fma(-dik.x, t.x, d[q].x));
      d[q].y = fma(-dik.y, t.x, fma(-dik.x, t.y, d[q].y));
    }
  }
}
// Step k of X = R^{-1} by back substitution on B = I (b holds B, rows
// g + 4 q of column c; r holds R, zero below the diagonal):
// X[k][c] = B[k][c] / R[k][k] goes to x, then B[i][c] -= R[i][k] X[k][c]
// (a no-op for the rows i > k, where R[i][k] = 0).
template <int k> __device__ __forceinline__ void inv_step(double2 (&b)[4], double2 (&x)[4], const double2 (&r)[4],
                                                          const double (&yk)[16], int g) {
  constexpr int qk = k >> 2, gk = k & 3;
  const double2 bk = grp(b[qk], gk);
  const double2 xk = make_double2(bk.x * yk[k], bk.y * yk[k]);
  x[qk].x = g == gk ? xk.x : x[qk].x;
  x[qk].y = g == gk ? xk.y : x[qk].y;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (4 * q < k) {                                // some row g + 4 q is above row k
      const double2 rik = nbc<k>(r[q]);             // R[i][k]
      b[q].x = fma(rik.y, xk.y, fma(-rik.x, xk.x, b[q].x));
      b[q].y = fma(-rik.y, xk.x, fma(-rik.x, xk.y, b[q].y));
    }
  }
}
template <int... ks>
__device__ __forceinline__ void chol_block(double2 (&d)[4], double2 (&r)[4], double (&yk)[16], int g, int c,
                                           double pmin, std::integer_sequence<int, ks...>) {
  (chol_step<ks>(d, r, yk, g, c, pmin), ...);
}
template <int... ks>
__device__ __forceinline__ void inv_block(double2 (&b)[4], double2 (&x)[4], const double2 (&r)[4],
                                          const double (&yk)[16], int g, std::integer_sequence<int, ks...>) {
  (inv_step<15 - ks>(b, x, r, yk, g), ...);         // k = 15 down to 0
}

// One work-group per instance: blocked right-looking Cholesky G = R^H R in
// 16x16 blocks (n padded to a multiple of 16 with an identity block), then
// R^{-1} by block back substitution.  Per block column K: wave 0 factors
// the diagonal block in registers, writes R_KK to the output and keeps
// X_KK = R_KK^{-1} in the block's place; the waves form the block row
// R_KJ = X_KK^H G_KJ and the trailing update G_IJ -= R_KI^H R_KJ on the
// matrix cores.  The upper blocks live in LDS (packed by block row); R and
// R^{-1} are written as full n x n matrices (zeros below the diagonal).
struct CholArgs {
  const double2 *G; double2 *R; double2 *Rinv;
  int n, ld;                       // order of this block; row stride of G, R and Rinv
  const double *diag;              // device: [0] diagonal shift, [1] pivot floor (cq_diag_kernel)
  int shift;                       // add diag[0] to the diagonal
  int64_t ws;                      // instance stride of the work area (elements)
};

constexpr int CQ_NB = CQ_NMAX / 16;   // block rows / columns at most
constexpr int CQ_CHOL_THREADS = 512;  // 8 waves (>= CQ_NB - 1 for the back substitution)
constexpr int CQ_RSTEP = CQ_CHOL_THREADS / CQ_NMAX;   // rows per pass of the row-major copies
constexpr int CQ_U = 8;                                // copies in flight per thread (LDS to global)
constexpr int CQ_UL = CQ_NMAX / CQ_RSTEP;              // global loads in flight per thread: all rows

__device__ __forceinline__ int bidx(int I, int J, int nb) { return I * nb - (I * (I - 1)) / 2 + (J - I); }

__global__ __launch_bounds__(CQ_CHOL_THREADS) void cq_chol_kernel(CholArgs a) {
  extern __shared__ double2 Bk[];   // packed upper blocks
  const int64_t inst = blockIdx.x;
  const double2 *G = a.G + inst * a.ws;
  double2 *Rout = a.R + inst * a.ws;
  double2 *Rinv = a.Rinv + inst * a.ws;
  const int n = a.n, ld = a.ld, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = (n + 15) / 16, np = 16 * nb;
  // row-major copies: thread (i0, j) takes column j, rows i0 + CQ_RSTEP u
  const int cj = tid & (CQ_NMAX - 1), ci0 = tid / CQ_NMAX;
  // load the upper blocks (identity padding beyond n)
  {
    double2 v[CQ_UL];
#pragma unroll
    for (int u = 0; u < CQ_UL; ++u) {
      const int i = ci0 + CQ_RSTEP * u;
      v[u] = make_double2(0.0, 0.0);
      if (i < n && cj < n && (cj >> 4) >= (i >> 4)) v[u] = G[(int64_t)i * ld + cj];
      else if (i == cj) v[u] = make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < CQ_UL; ++u) {
      const int i = ci0 + CQ_RSTEP * u;
      if (i < np && cj < np && (cj >> 4) >= (i >> 4)) Bk[bidx(i >> 4, cj >> 4, nb) * 256 + bo(i & 15, cj & 15)] = v[u];
    }
  }
  __syncthreads();
  const double pmin = a.diag[inst * a.ws * 2 + 1];
  // diagonal shift (first pass)
  if (a.shift && wave == 0) {
    const double shift = a.diag[inst * a.ws * 2];
    for (int i = lane; i < n; i += 64) Bk[bidx(i >> 4, i >> 4, nb) * 256 + bo(i & 15, i & 15)].x += shift;
  }
  __syncthreads();
  for (int K = 0; K < nb; ++K) {
    double2 *D = Bk + bidx(K, K, nb) * 256;     // G_KK, then X_KK
    if (wave == 0) {
      const int c = lane & 15, g = lane >> 4;
      double2 d[4], r[4], b[4], x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {             // the full Hermitian block from its upper half
        const int i = g + 4 * q;
        const double2 v = c >= i ? D[bo(i, c)] : D[bo(c, i)];
        d[q] = c >= i ? v : make_double2(v.x, -v.y);
        r[q] = x[q] = make_double2(0.0, 0.0);
        b[q] = make_double2(i == c ? 1.0 : 0.0, 0.0);
      }
      double yk[16];
      chol_block(d, r, yk, g, c, pmin, std::make_integer_sequence<int, 16>{});
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * K + g + 4 * q, jj = 16 * K + c;
        if (i < n && jj < n) Rout[(int64_t)i * ld + jj] = r[q];
      }
      inv_block(b, x, r, yk, g, std::make_integer_sequence<int, 16>{});
#pragma unroll
      for (int q = 0; q < 4; ++q) D[bo(g + 4 * q, c)] = x[q];
    }
    __syncthreads();
    // block row: R_KJ = X_KK^H G_KJ, one wave per block
    for (int J = K + 1 + wave; J < nb; J += CQ_CHOL_THREADS / 64) {
      double2 *Bj = Bk + bidx(K, J, nb) * 256;
      CAcc acc;
      blk_mma(D, true, Bj, acc);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        Bj[bo(Mf<double>::row(lane, rr), lane & 15)] = make_double2(acc.re(rr), acc.im(rr));
    }
    __syncthreads();
    // trailing update G_IJ -= R_KI^H R_KJ, K < I <= J
    {
      const int nt = nb - K - 1;
      for (int t = wave; t < nt * (nt + 1) / 2; t += CQ_CHOL_THREADS / 64) {
        int I = 0, u = t;
        while (u >= nt - I) { u -= nt - I; ++I; }
        I += K + 1;
        const int J = I + u;
        double2 *Cij = Bk + bidx(I, J, nb) * 256;
        CAcc acc;
        blk_mma(Bk + bidx(K, I, nb) * 256, true, Bk + bidx(K, J, nb) * 256, acc);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          double2 &c = Cij[bo(Mf<double>::row(lane, rr), lane & 15)];
          c.x -= acc.re(rr);
          c.y -= acc.im(rr);
        }
      }
    }
    __syncthreads();
  }
  // R: the blocks above the diagonal blocks (written above) and zeros below
  for (int s0 = 0; s0 < n; s0 += CQ_U * CQ_RSTEP) {
    double2 v[CQ_U];
#pragma unroll
    for (int u = 0; u < CQ_U; ++u) {
      const int i = s0 + ci0 + CQ_RSTEP * u;
      v[u] = make_double2(0.0, 0.0);
      if (i < n && cj < n && (cj >> 4) > (i >> 4)) v[u] = Bk[bidx(i >> 4, cj >> 4, nb) * 256 + bo(i & 15, cj & 15)];
    }
#pragma unroll
    for (int u = 0; u < CQ_U; ++u) {
      const int i = s0 + ci0 + CQ_RSTEP * u;
      if (i < n && cj < n && (cj >> 4) != (i >> 4)) Rout[(int64_t)i * ld + cj] = v[u];
    }
  }
  __syncthreads();
  // R^{-1} by block back substitution, X_IJ = -X_II S_IJ with
  // S_IJ = sum_{K=I+1..J} R_IK X_KJ, right-looking from the bottom: at step
  // K (nb-1 down to 1) every pair I < K <= J adds R_IK X_KJ to S_IJ, then
  // block row K-1, whose sums are complete, is formed in the place of R's
  // row K-1 (read for the last time at this step; the diagonal blocks hold
  // X_II since the factorisation).  The pairs (I, J) are dealt to the waves
  // round-robin in row-major order, each keeping its sums in registers, so
  // the longest chain of block products is ~21 instead of nb (nb + 1) / 2 - 1.
  {
    constexpr int NW = CQ_CHOL_THREADS / 64;
    constexpr int NS = (CQ_NB * (CQ_NB - 1) / 2 + NW - 1) / NW;   // pairs per wave
    const int npairs = nb * (nb - 1) / 2;
    int pi[NS], pj[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      int u = wave + NW * t, I = 0;
      pi[t] = pj[t] = -1;
      if (u < npairs) {
        while (u >= nb - 1 - I) { u -= nb - 1 - I; ++I; }
        pi[t] = I;
        pj[t] = I + 1 + u;
      }
    }
    CAcc sum[NS];
    for (int K = nb - 1; K >= 1; --K) {
#pragma unroll
      for (int t = 0; t < NS; ++t)
        if (pi[t] >= 0 && pi[t] < K && K <= pj[t])
          blk_mma(Bk + bidx(pi[t], K, nb) * 256, false, Bk + bidx(K, pj[t], nb) * 256, sum[t]);
      __syncthreads();   // every R_IK and X_KJ of this step has been read
#pragma unroll
      for (int t = 0; t < NS; ++t)
        if (pi[t] == K - 1) {
          double2 *Xj = Bk + bidx(pi[t], pj[t], nb) * 256;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            Xj[bo(Mf<double>::row(lane, rr), lane & 15)] = make_double2(sum[t].re(rr), sum[t].im(rr));
          __builtin_amdgcn_wave_barrier();
          CAcc acc;
          blk_mma(Bk + bidx(pi[t], pi[t], nb) * 256, false, Xj, acc);
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            Xj[bo(Mf<double>::row(lane, rr), lane & 15)] = make_double2(-acc.re(rr), -acc.im(rr));
        }
      __syncthreads();   // block row K - 1 of X is formed
    }
  }
  for (int s0 = 0; s0 < n; s0 += CQ_U * CQ_RSTEP) {
    double2 v[CQ_U];
#pragma unroll
    for (int u = 0; u < CQ_U; ++u) {
      const int i = s0 + ci0 + CQ_RSTEP * u;
      v[u] = make_double2(0.0, 0.0);
      if (i < n && cj < n && (cj >> 4) >= (i >> 4)) v[u] = Bk[bidx(i >> 4, cj >> 4, nb) * 256 + bo(i & 15, cj & 15)];
    }
#pragma unroll
    for (int u = 0; u < CQ_U; ++u) {
      const int i = s0 + ci0 + CQ_RSTEP * u;
      if (i < n && cj < n) Rinv[(int64_t)i * ld + cj] = v[u];
    }
  }
}

// Per instance (one work-group each), from the diagonal of G: out[0] = the
// first pass's shift s = 11 (m n + n (n + 1)) u tr(G) (0 when !shift), and
// out[1] = the pivot floor 1e-20 max_i (G_ii + s): a Schur-complement pivot
// below it (a numerically singular G, e.g. from an exactly rank-deficient
// input) is replaced by it, which lifts the null directions to moderate
// size so that the next passes orthonormalise them instead of overflowing.
__global__ __launch_bounds__(256) void cq_diag_kernel(const double2 *G, int m, int n, int shift,
                                                      double *out, int64_t ws) {
  __shared__ double part[4], pmax[4];
  const int64_t inst = blockIdx.x;
  G += inst * ws;
  double t = 0.0, mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = G[(int64_t)i * n + i].x;
    t += v;
    mx = fmax(mx, v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    t += __shfl_xor(t, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = t;
    pmax[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tr = part[0] + part[1] + part[2] + part[3];
    const double gmax = fmax(fmax(pmax[0], pmax[1]), fmax(pmax[2], pmax[3]));
    const double s = shift ? 11.0 * ((double)m * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * tr : 0.0;
    out[inst * ws * 2] = s;
    out[inst * ws * 2 + 1] = fmax(1e-20 * (gmax + s), 1e-300);
  }
}

// zero the rows nlo..n-1, columns 0..nlo-1 of two n x n matrices
__global__ __launch_bounds__(256) void cq_zero_lower_kernel(double2 *A, double2 *B, int n, int nlo,
                                                            int64_t ws) {
  const int64_t inst = blockIdx.y;
  A += inst * ws;
  B += inst * ws;
  const int64_t cnt = (int64_t)(n - nlo) * nlo;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    const int64_t i = nlo + e / nlo, j = e % nlo;
    A[i * n + j] = make_double2(0.0, 0.0);
    B[i * n + j] = make_double2(0.0, 0.0);
  }
}

}  // namespace

bool cholqr_ok(int m, int n) { return n >= 1 && n <= 2 * CQ_NMAX && m >= n; }

int64_t cholqr_work_elems(int m, int n) {
  // W_0..W_2, G, R_p, Rinv, two running products, a block temporary, the shift
  return 3 * (int64_t)m * n + 6 * (int64_t)n * n + 16;
}

void cholqr_init() {
  (void)hipFuncSetAttribute((const void *)cq_chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            CQ_NB * (CQ_NB + 1) / 2 * 256 * (int)sizeof(double2));
  (void)hipGetLastError();
}

hipError_t cholqr(const QrArgs &p, hipStream_t s) {
  const int m = p.m, n = p.n, R = p.inst.count;
  if (!cholqr_ok(m, n)) return hipErrorInvalidValue;
  const int64_t mn = (int64_t)m * n, nn = (int64_t)n * n, ws = p.inst.skip;
  double2 *Wb[3] = {p.work, p.work + mn, p.work + 2 * mn};
  double2 *G = p.work + 3 * mn;
  double2 *Rk = G + nn, *Rinv = Rk + nn;
  double2 *Racc[2] = {Rinv + nn, Rinv + 2 * nn};
  double2 *Tm = Rinv + 3 * nn;
  double *diagv = reinterpret_cast<double *>(Tm + nn);   // shift, pivot floor
  {
    int64_t gx = (mn + 255) / 256;
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(cq_prep_kernel, dim3((unsigned)gx, R), dim3(256), 0, s, p, Wb[0], ws);
  }
  const int nt = (n + 15) / 16;
  // one cq_chol call covers at most CQ_NMAX; beyond that the factorisation
  // is blocked 2 x 2 (n1 = CQ_NMAX):
  //   R11 = chol(G11 + s I), R12 = R11^{-H} G12, R22 = chol(G22 + s I - R12^H R12),
  //   R^{-1} = [R11^{-1}, -R11^{-1} R12 R22^{-1}; 0, R22^{-1}]
  const int n1 = n <= CQ_NMAX ? n : CQ_NMAX, n2 = n - n1;
  auto lds_of = [](int k) { const int b = (k + 15) / 16; return (size_t)(b * (b + 1) / 2) * 256 * sizeof(double2); };
  // general product Z (M x N) = op(X) (M x K) Y (K x N) in the work area, row strides given
  auto gemm = [&](const double2 *X, int64_t xr, int64_t xc, int conjX, const double2 *Y, int64_t yr,
                  double2 *Z, int64_t zr, int M_, int N_, int K_, int mode) {
    GemmArgs g{};
    g.A = X; g.B = Y; g.C = Z;
    g.M = M_; g.N = N_; g.K = K_; g.batch = 1;
    g.sam = xr; g.sak = xc; g.sbk = yr; g.sbn = 1; g.scm = zr; g.scn = 1;
    g.conjA = conjX;
    g.mode = mode;
    g.inst.count = R; g.inst.a = ws; g.inst.b = ws; g.inst.c = ws;
    return cgemm(F64, F64, F64, g, s);
  };
  // n x n product X Y (row-major operands in the work area) into Z with
  // strides (zr, zc) and instance stride zs; conj: conjugated result
  auto nn_gemm = [&](const double2 *X, const double2 *Y, double2 *Z, int64_t zr, int64_t zc,
                     int64_t zs, int conj) {
    GemmArgs g{};
    g.A = X; g.B = Y; g.C = Z;
    g.M = n; g.N = n; g.K = n; g.batch = 1;
    g.sam = n; g.sak = 1; g.sbk = n; g.sbn = 1; g.scm = zr; g.scn = zc;
    g.conjA = conj; g.conjB = conj;
    g.inst.count = R; g.inst.a = ws; g.inst.b = ws; g.inst.c = zs;
    return cgemm(F64, F64, F64, g, s);
  };
  for (int pass = 0; pass < 3; ++pass) {
    const bool last = pass == 2;
    hipLaunchKernelGGL(cq_gram_kernel, dim3(nt * (nt + 1) / 2, R), dim3(CQ_THREADS), 0, s, Wb[pass],
                       m, n, G, ws);
    hipLaunchKernelGGL(cq_diag_kernel, dim3(R), dim3(256), 0, s, G, m, n, pass == 0 ? 1 : 0, diagv, ws);
    double2 *Rp = pass == 0 ? Racc[0] : Rk;
    CholArgs ca{};
    ca.G = G; ca.R = Rp; ca.Rinv = Rinv;
    ca.n = n1; ca.ld = n; ca.ws = ws;
    ca.diag = diagv;
    ca.shift = pass == 0;
    hipLaunchKernelGGL(cq_chol_kernel, dim3(R), dim3(CQ_CHOL_THREADS), lds_of(n1), s, ca);
    hipError_t e = hipSuccess;
    if (n2 > 0) {
      // R12 = R11^{-H} G12 (into R), then G22 <- G22 - R12^H R12
      e = gemm(Rinv, 1, n, 1, G + n1, n, Rp + n1, n, n1, n2, n1, 0);
      if (e == hipSuccess) e = gemm(Rp + n1, 1, n, 1, Rp + n1, n, G + (int64_t)n1 * n + n1, n, n2, n2, n1, 1);
      if (e != hipSuccess) return e;
      CholArgs cb = ca;
      cb.G = G + (int64_t)n1 * n + n1;
      cb.R = Rp + (int64_t)n1 * n + n1;
      cb.Rinv = Rinv + (int64_t)n1 * n + n1;
      cb.n = n2;
      hipLaunchKernelGGL(cq_chol_kernel, dim3(R), dim3(CQ_CHOL_THREADS), lds_of(n2), s, cb);
      // upper-right block of R^{-1}: -R11^{-1} (R12 R22^{-1})
      e = gemm(Rp + n1, n, 1, 0, Rinv + (int64_t)n1 * n + n1, n, Tm, n2, n1, n2, n2, 0);
      if (e == hipSuccess) e = gemm(Rinv, n, 1, 0, Tm, n2, Rinv + n1, n, n1, n2, n1, 2);
      if (e != hipSuccess) return e;
      {
        int64_t gx = ((int64_t)n2 * n1 + 255) / 256;
        if (gx > 256) gx = 256;
        hipLaunchKernelGGL(cq_zero_lower_kernel, dim3((unsigned)gx, R), dim3(256), 0, s, Rp, Rinv, n, n1, ws);
      }
    }
    // R = R_3 R_2 R_1, accumulated from the left; the last product goes to
    // the caller's R through its strides
    if (pass == 1) e = nn_gemm(Rk, Racc[0], Racc[1], n, 1, ws, 0);
    if (last) e = nn_gemm(Rk, Racc[1], p.R, p.r_rs, p.r_cs, p.inst.c, p.conjR);
    if (e != hipSuccess) return e;
    // W_{p+1} = W_p Rinv; the last one is Q, written through the caller's
    // strides (conjugated output = product of conjugated operands)
    GemmArgs g{};
    g.A = Wb[pass]; g.B = Rinv;
    g.M = m; g.N = n; g.K = n; g.batch = 1;
    g.sam = n; g.sak = 1; g.sbk = n; g.sbn = 1;
    g.inst.count = R;
    g.inst.a = ws; g.inst.b = ws;
    if (last) {
      g.C = p.Q; g.scm = p.q_rs; g.scn = p.q_cs;
      g.conjA = p.conjQ; g.conjB = p.conjQ;
      g.inst.c = p.inst.b;
    } else {
      g.C = Wb[pass + 1]; g.scm = n; g.scn = 1;
      g.inst.c = ws;
    }
    e = cgemm(F64, F64, F64, g, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace tdvp
