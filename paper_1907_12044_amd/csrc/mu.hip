// Device kernels of TDVP-MU (Sec. II.A.2, "TDVP-MU": eq:tdvp1_C,
// eq:tdvp1_mu_rcano, eq:tdvp1_mu_L, eq:reg2) integrated with the
// variable-mean-field scheme (an embedded Runge-Kutta 5(4) pair):
//
//  * mu_reginv: the regularised inverse P = V Lam~^{-1} U^H of a bond matrix
//    D = U Lam V^H, Lam~ = Lam + sqrt(eps) exp(-Lam / sqrt(eps)) (eq:reg2),
//    from a one-sided Jacobi SVD of D in one work-group (FP64; D up to
//    64 x 64 held in LDS with the accumulated right rotations), the bonds
//    of a chain side by side in one launch;
//  * svd_split: the truncated SVD that splits a two-site tensor (eq:SVD) in
//    the two-site projector-splitting step, with the same Jacobi sweeps;
//  * merge_mpo: two neighbouring MPO sites as one (the two-site operator);
//  * mu_finish: out = -i (X - Y), the projected site derivative of
//    eq:tdvp1_mu_L once Y = A (A^H X) has been formed by the GEMMs;
//  * lincomb: out = x_0 + sum_j a_j x_j over packed state vectors (the
//    Runge-Kutta stages);
//  * rk_err_partials: per-work-group sums of |err_e / (atol + rtol
//    max(|y_e|, |y'_e|))|^2 (the step-size control norm).
#include <algorithm>

#include "common.h"
#include "util.h"

namespace tdvp {

namespace {

constexpr int RI_THREADS = 256;
constexpr int RI_MAXN = 64;
constexpr int RI_SWEEPS = 40;   // most Jacobi sweeps (convergence is quadratic; ~8-12 needed)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {   // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// One-sided Jacobi on the m x n matrix held column-major in B (LDS,
// B[c * m + r], np = n rounded up to even, column n a zero column when n
// is odd): the columns of B J are made orthogonal by plane rotations J
// applied to column pairs (p, q) in a round-robin order (np/2 disjoint
// pairs per round, np - 1 rounds per sweep, all pairs of a round at once);
// V (np x np, column-major, identity on entry) accumulates J.  At
// convergence B = U Lam with Lam_j = |b_j|, and the matrix is U Lam V^H.
// A pair is rotated when |b_p^H b_q| > m u sqrt(|b_p|^2 |b_q|^2) (u the unit
// round-off) and both |b_p|^2, |b_q|^2 exceed `small` (columns at the
// rounding level of a rank-deficient matrix are left alone: rotating them
// against each other only shrinks them into the subnormal range); the
// sweeps stop when no pair of a sweep was rotated (at most RI_SWEEPS).
// Every thread of the work-group calls it.
__device__ void jacobi_columns(double2 *B, double2 *V, int m, int np, int *rotated, double small) {
  const int tid = threadIdx.x;
  // Each pair is handled by a group of G threads (G = 256 / (np/2), a power
  // of two dividing 64, at least 8) that split the rows.
  const int npairs = np / 2;
  int G = RI_THREADS / npairs;
  G = G >= 64 ? 64 : (G >= 32 ? 32 : (G >= 16 ? 16 : 8));
  const int grp = tid / G, gl = tid % G;
  const double tol = (double)m * 1.1102230246251565e-16;
  for (int sweep = 0; sweep < RI_SWEEPS; ++sweep) {
    if (tid == 0) *rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      if (grp < npairs) {
        // round-robin (circle) pairing: position 0 fixed, the others rotate
        int a = grp, b = np - 1 - grp;
        auto slot = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + round) % (np - 1); };
        int p = slot(a), q = slot(b);
        if (p > q) { const int t = p; p = q; q = t; }
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
        for (int r = gl; r < m; r += G) {
          const double2 x = B[p * m + r], y = B[q * m + r];
          al += x.x * x.x + x.y * x.y;
          be += y.x * y.x + y.y * y.y;
          const double2 g = cconjmul(x, y);
          gr += g.x;
          gi += g.y;
        }
        for (int o = G / 2; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, G);
          be += __shfl_xor(be, o, G);
          gr += __shfl_xor(gr, o, G);
          gi += __shfl_xor(gi, o, G);
        }
        const double gabs = sqrt(gr * gr + gi * gi);
        if (al > small && be > small && gabs > tol * sqrt(al * be) && gabs > 0.0) {
          // rotation of the real symmetric [[al, |g|], [|g|, be]] after the
          // phase e^{-i phi} (g = |g| e^{i phi}) is taken into column q
          const double zeta = (be - al) / (2.0 * gabs);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          const double2 ph = make_double2(gr / gabs, -gi / gabs);      // e^{-i phi}
          for (int r = gl; r < m; r += G) {
            const double2 x = B[p * m + r], y = cmul(ph, B[q * m + r]);
            B[p * m + r] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            B[q * m + r] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          for (int r = gl; r < np; r += G) {
            const double2 x = V[p * np + r], y = cmul(ph, V[q * np + r]);
            V[p * np + r] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            V[q * np + r] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          if (gl == 0) *rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = *rotated;
    __syncthreads();
    if (!any) break;
  }
}

// Loads the row-major m x n matrix X into B (column-major, np columns, the
// padding column zero) and sets V to the identity.
__device__ void jacobi_load(const double2 *X, int m, int n, int np, double2 *B, double2 *V) {
  for (int e = threadIdx.x; e < np * m; e += RI_THREADS) {
    const int c = e / m, r = e % m;
    B[e] = c < n ? X[(int64_t)r * n + c] : make_double2(0.0, 0.0);
  }
  for (int e = threadIdx.x; e < np * np; e += RI_THREADS) {
    const int c = e / np, r = e % np;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
}

// Regularised inverse of each n x n bond matrix D of the batch (one
// work-group per matrix, blockIdx.x):
//   P = V Lam~^{-1} U^H = sum_j v_j b_j^H / (Lam_j Lam~_j).
__global__ __launch_bounds__(RI_THREADS) void mu_reginv_kernel(RegInvBatch bt) {
  const double2 *D = bt.D[blockIdx.x];
  double2 *P = bt.P[blockIdx.x];
  const int n = bt.n[blockIdx.x];
  const double eps = bt.eps;
  __shared__ double2 B[RI_MAXN * RI_MAXN];
  __shared__ double2 V[RI_MAXN * RI_MAXN];
  __shared__ double lam[RI_MAXN];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int np = (n + 1) & ~1;               // even column count (one zero column if n is odd)
  jacobi_load(D, n, n, np, B, V);
  jacobi_columns(B, V, n, np, &rotated, 0.0);
  for (int j = tid; j < n; j += RI_THREADS) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += B[j * n + r].x * B[j * n + r].x + B[j * n + r].y * B[j * n + r].y;
    lam[j] = sqrt(s);
  }
  __syncthreads();
  const double se = sqrt(eps);
  // P[k][l] = sum_j V[k][j] conj(B[l][j]) / (lam_j lam~_j)
  for (int e = tid; e < n * n; e += RI_THREADS) {
    const int k = e / n, l = e % n;
    double pr = 0.0, pi = 0.0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[j];
      if (!(lj > 0.0)) continue;
      const double w = 1.0 / (lj * (lj + se * exp(-lj / se)));
      const double2 v = V[j * np + k], b = B[j * n + l];
      // v conj(b)
      pr += w * (v.x * b.x + v.y * b.y);
      pi += w * (v.y * b.x - v.x * b.y);
    }
    P[(int64_t)k * n + l] = make_double2(pr, pi);
  }
}

// Truncated SVD split of a two-site tensor (eq:SVD): X (m x n row-major,
// m, n <= 64) = U Lam V^H, the `keep` largest singular values kept (in
// descending order).  mode 0: A = U (m x keep), Bo = Lam V^H (keep x n);
// mode 1: A = U Lam, Bo = V^H.  The sum of the squares of the singular
// values dropped is added to *discarded (may be null).  The Jacobi sweeps
// run on the columns of a tall matrix: X itself when m >= n, else X^H
// (whose columns' rotations then give U, and its orthogonalised columns
// Lam V^H's rows); a wide matrix's surplus columns would only shrink to
// rounding noise.  Columns below u^2 |X|_F^2 are taken as zero.
__global__ __launch_bounds__(RI_THREADS) void svd_split_kernel(const double2 *X, int m, int n, int keep,
                                                               int mode, double2 *A, double2 *Bo,
                                                               double *discarded) {
  __shared__ double2 B[RI_MAXN * RI_MAXN];
  __shared__ double2 V[RI_MAXN * RI_MAXN];
  __shared__ double lam[RI_MAXN];
  __shared__ double part[RI_THREADS];
  __shared__ int ord[RI_MAXN];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const bool tr = n > m;
  const int rows = tr ? n : m, cols = tr ? m : n;   // rows >= cols
  const int np = (cols + 1) & ~1;
  double f2 = 0.0;
  for (int e = tid; e < np * rows; e += RI_THREADS) {
    const int c = e / rows, r = e % rows;
    double2 v = make_double2(0.0, 0.0);
    if (c < cols) {
      const double2 x = tr ? X[(int64_t)c * n + r] : X[(int64_t)r * n + c];
      v = tr ? make_double2(x.x, -x.y) : x;
    }
    B[e] = v;
    f2 += v.x * v.x + v.y * v.y;
  }
  for (int e = tid; e < np * np; e += RI_THREADS) {
    const int c = e / np, r = e % np;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  part[tid] = f2;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < RI_THREADS; ++k) t += part[k];
    part[0] = t;
  }
  __syncthreads();
  const double u = 1.1102230246251565e-16;
  jacobi_columns(B, V, rows, np, &rotated, u * u * part[0]);
  for (int j = tid; j < cols; j += RI_THREADS) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r)
      s += B[j * rows + r].x * B[j * rows + r].x + B[j * rows + r].y * B[j * rows + r].y;
    lam[j] = sqrt(s);
  }
  __syncthreads();
  if (tid == 0) {
    // column order by descending singular value (insertion sort, <= 64
    // columns; ties keep the lower column first)
    for (int j = 0; j < cols; ++j) {
      int k = j;
      while (k > 0 && lam[ord[k - 1]] < lam[j]) {
        ord[k] = ord[k - 1];
        --k;
      }
      ord[k] = j;
    }
    if (discarded) {
      double dw = 0.0;
      for (int j = keep; j < cols; ++j) dw += lam[ord[j]] * lam[ord[j]];
      *discarded += dw;
    }
  }
  __syncthreads();
  // U column j: b_c / lam_c (X tall) or v_c (X wide); V^H row j: conj(v_c)
  // (tall) or conj(b_c) / lam_c (wide), with c = ord[j]
  for (int e = tid; e < m * keep; e += RI_THREADS) {
    const int r = e / keep, j = e % keep;
    const int c = ord[j];
    const double lc = lam[c], inv = lc > 0.0 ? 1.0 / lc : 0.0;
    double2 uv;
    if (!tr) {
      const double2 b = B[c * rows + r];
      uv = make_double2(b.x * inv, b.y * inv);
    } else {
      uv = V[c * np + r];
    }
    const double sc = mode == 0 ? 1.0 : lc;
    A[e] = make_double2(sc * uv.x, sc * uv.y);
  }
  for (int e = tid; e < keep * n; e += RI_THREADS) {
    const int j = e / n, col = e % n;
    const int c = ord[j];
    const double lc = lam[c], inv = lc > 0.0 ? 1.0 / lc : 0.0;
    double2 vh;   // row j of V^H
    if (!tr) {
      const double2 v = V[c * np + col];
      vh = make_double2(v.x, -v.y);
    } else {
      const double2 b = B[c * rows + col];
      vh = make_double2(b.x * inv, -b.y * inv);
    }
    const double sc = mode == 0 ? lc : 1.0;
    Bo[e] = make_double2(sc * vh.x, sc * vh.y);
  }
}

// Two neighbouring MPO sites as one: W[w][(s1 s2)][(t1 t2)][v] =
// sum_u W1[w][s1][t1][u] W2[u][s2][t2][v] (all row-major c128).
__global__ __launch_bounds__(256) void merge_mpo_kernel(const double2 *W1, const double2 *W2, int wl, int d1,
                                                        int wm, int d2, int wr, double2 *W) {
  const int64_t D = (int64_t)d1 * d2;
  const int64_t total = (int64_t)wl * D * D * wr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(e % wr);
    const int64_t t = (e / wr) % D, s = (e / (wr * D)) % D;
    const int w = (int)(e / (wr * D * D));
    const int s1 = (int)(s / d2), s2 = (int)(s % d2), t1 = (int)(t / d2), t2 = (int)(t % d2);
    double re = 0.0, im = 0.0;
    for (int u = 0; u < wm; ++u) {
      const double2 a = W1[(((int64_t)w * d1 + s1) * d1 + t1) * wm + u];
      const double2 b = W2[(((int64_t)u * d2 + s2) * d2 + t2) * wr + v];
      re += a.x * b.x - a.y * b.y;
      im += a.x * b.y + a.y * b.x;
    }
    W[e] = make_double2(re, im);
  }
}

constexpr int LB = 256;

// out = -i (X - Y)  (Y == null: out = -i X)
__global__ __launch_bounds__(LB) void mu_finish_kernel(const double2 *X, const double2 *Y, double2 *out,
                                                       int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * LB + threadIdx.x; e < n; e += (int64_t)gridDim.x * LB) {
    const double2 x = X[e], y = Y ? Y[e] : make_double2(0.0, 0.0);
    out[e] = make_double2(x.y - y.y, -(x.x - y.x));
  }
}

__global__ __launch_bounds__(LB) void lincomb_kernel(LinComb lc, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * LB + threadIdx.x; e < n; e += (int64_t)gridDim.x * LB) {
    double2 v = lc.x0 ? lc.x0[e] : make_double2(0.0, 0.0);
    for (int j = 0; j < lc.m; ++j) {
      const double2 w = lc.x[j][e];
      v.x += lc.a[j] * w.x;
      v.y += lc.a[j] * w.y;
    }
    lc.out[e] = v;
  }
}

__global__ __launch_bounds__(LB) void rk_err_kernel(const double2 *err, const double2 *y, const double2 *ynew,
                                                    int64_t n, double rtol, double atol, double *part) {
  __shared__ double sh[LB / 64];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * LB + threadIdx.x; e < n; e += (int64_t)gridDim.x * LB) {
    const double a = sqrt(y[e].x * y[e].x + y[e].y * y[e].y);
    const double b = sqrt(ynew[e].x * ynew[e].x + ynew[e].y * ynew[e].y);
    const double sc = atol + rtol * fmax(a, b);
    const double er = err[e].x / sc, ei = err[e].y / sc;
    s += er * er + ei * ei;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < LB / 64; ++w) t += sh[w];
    part[blockIdx.x] = t;
  }
}

int vec_grid(int64_t n) {
  int64_t g = (n + LB - 1) / LB;
  if (g > RK_PARTS) g = RK_PARTS;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

hipError_t mu_reginv(const RegInvBatch &b, hipStream_t s) {
  if (b.count < 1 || b.count > REGINV_BATCH) return hipErrorInvalidValue;
  for (int k = 0; k < b.count; ++k)
    if (b.n[k] < 1 || b.n[k] > RI_MAXN || !b.D[k] || !b.P[k]) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mu_reginv_kernel, dim3(b.count), dim3(RI_THREADS), 0, s, b);
  return hipGetLastError();
}

hipError_t svd_split(const double2 *X, int m, int n, int keep, int mode, double2 *A, double2 *B,
                     double *discarded, hipStream_t s) {
  if (m < 1 || n < 1 || m > RI_MAXN || n > RI_MAXN || keep < 1 || keep > n || keep > m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(svd_split_kernel, dim3(1), dim3(RI_THREADS), 0, s, X, m, n, keep, mode, A, B, discarded);
  return hipGetLastError();
}

hipError_t merge_mpo(const double2 *W1, const double2 *W2, int wl, int d1, int wm, int d2, int wr, double2 *W,
                     hipStream_t s) {
  const int64_t total = (int64_t)wl * d1 * d2 * d1 * d2 * wr;
  if (total < 1) return hipErrorInvalidValue;
  const int64_t g = std::min<int64_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(merge_mpo_kernel, dim3((unsigned)g), dim3(256), 0, s, W1, W2, wl, d1, wm, d2, wr, W);
  return hipGetLastError();
}

hipError_t mu_finish(const double2 *X, const double2 *Y, double2 *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(mu_finish_kernel, dim3(vec_grid(n)), dim3(LB), 0, s, X, Y, out, n);
  return hipGetLastError();
}

hipError_t lincomb(const LinComb &lc, int64_t n, hipStream_t s) {
  if (lc.m < 0 || lc.m > LINCOMB_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lincomb_kernel, dim3(vec_grid(n)), dim3(LB), 0, s, lc, n);
  return hipGetLastError();
}

int rk_err_partials(const double2 *err, const double2 *y, const double2 *ynew, int64_t n, double rtol,
                    double atol, double *part, hipStream_t s) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(rk_err_kernel, dim3(g), dim3(LB), 0, s, err, y, ynew, n, rtol, atol, part);
  return hipGetLastError() == hipSuccess ? g : -1;
}

}  // namespace tdvp
