// Device kernels of TDVP-MU (Sec. II.A.2, "TDVP-MU": eq:tdvp1_C,
// eq:tdvp1_mu_rcano, eq:tdvp1_mu_L, eq:reg2) integrated with the
// variable-mean-field scheme (an embedded Runge-Kutta 5(4) pair):
//
//  * mu_reginv: the regularised inverse P = V Lam~^{-1} U^H of a bond matrix
//    D = U Lam V^H, Lam~ = Lam + sqrt(eps) exp(-Lam / sqrt(eps)) (eq:reg2),
//    from a one-sided Jacobi SVD of D in one work-group (FP64; D up to
//    64 x 64 held in LDS with the accumulated right rotations), the bonds
//    of a chain side by side in one launch;
//  * mu_finish: out = -i (X - Y), the projected site derivative of
//    eq:tdvp1_mu_L once Y = A (A^H X) has been formed by the GEMMs;
//  * lincomb: out = x_0 + sum_j a_j x_j over packed state vectors (the
//    Runge-Kutta stages);
//  * rk_err_partials: per-work-group sums of |err_e / (atol + rtol
//    max(|y_e|, |y'_e|))|^2 (the step-size control norm).
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

// One-sided Jacobi SVD of the n x n matrix D (row-major, n <= 64): the
// columns of B = D J are made orthogonal by plane rotations J applied to
// column pairs (p, q) in a round-robin order (n/2 disjoint pairs per round,
// n - 1 rounds per sweep, all pairs of a round at once); V accumulates J.
// At convergence B = U Lam with Lam_j = |b_j|, so
//   P = V Lam~^{-1} U^H = sum_j v_j b_j^H / (Lam_j Lam~_j).
// A pair is rotated when |b_p^H b_q| > n u sqrt(|b_p|^2 |b_q|^2) (u the unit
// round-off); the sweeps stop when no pair of a sweep was rotated (at most
// RI_SWEEPS).
// Odd n is padded with one zero column (never rotated: its norm is 0).
// One work-group per matrix of the batch (blockIdx.x).
__global__ __launch_bounds__(RI_THREADS) void mu_reginv_kernel(RegInvBatch bt) {
  const double2 *D = bt.D[blockIdx.x];
  double2 *P = bt.P[blockIdx.x];
  const int n = bt.n[blockIdx.x];
  const double eps = bt.eps;
  __shared__ double2 B[RI_MAXN * RI_MAXN];   // column-major: B[c * n + r]
  __shared__ double2 V[RI_MAXN * RI_MAXN];
  __shared__ double lam[RI_MAXN];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int np = (n + 1) & ~1;               // even column count (one zero column if n is odd)
  for (int e = tid; e < np * n; e += RI_THREADS) {
    const int c = e / n, r = e % n;
    B[e] = c < n ? D[(int64_t)r * n + c] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < np * np; e += RI_THREADS) {
    const int c = e / np, r = e % np;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Each pair is handled by a group of G threads (G = 256 / (np/2), a power
  // of two dividing 64, at least 8) that split the rows.
  const int npairs = np / 2;
  int G = RI_THREADS / npairs;
  G = G >= 64 ? 64 : (G >= 32 ? 32 : (G >= 16 ? 16 : 8));
  const int grp = tid / G, gl = tid % G;
  const double tol = (double)n * 1.1102230246251565e-16;
  for (int sweep = 0; sweep < RI_SWEEPS; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      if (grp < npairs) {
        // round-robin (circle) pairing: position 0 fixed, the others rotate
        int a = grp, b = np - 1 - grp;
        auto slot = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + round) % (np - 1); };
        int p = slot(a), q = slot(b);
        if (p > q) { const int t = p; p = q; q = t; }
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
        for (int r = gl; r < n; r += G) {
          const double2 x = B[p * n + r], y = B[q * n + r];
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
        if (gabs > tol * sqrt(al * be) && gabs > 0.0) {
          // rotation of the real symmetric [[al, |g|], [|g|, be]] after the
          // phase e^{-i phi} (g = |g| e^{i phi}) is taken into column q
          const double zeta = (be - al) / (2.0 * gabs);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          const double2 ph = make_double2(gr / gabs, -gi / gabs);      // e^{-i phi}
          for (int r = gl; r < n; r += G) {
            const double2 x = B[p * n + r], y = cmul(ph, B[q * n + r]);
            B[p * n + r] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            B[q * n + r] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          for (int r = gl; r < np; r += G) {
            const double2 x = V[p * np + r], y = cmul(ph, V[q * np + r]);
            V[p * np + r] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
            V[q * np + r] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
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
