// Lanczos propagator y = exp(z H) x for the local equations eq:tdvp2_C and
// eq:tdvp2_D (Sec. II.A.2): Krylov basis, three-term recurrence with full
// classical Gram-Schmidt re-orthogonalisation, small exponential of the
// tridiagonal projected matrix T -- all in FP64 on the device.
//
// Basis vectors are stored unnormalised: v_j = scale_j u_j.  Step j is
//   w   = H u_j                                (operator kernels, P partial sums)
//   c_i = scale_i scale_j <u_i, w>,  i <= j    (lz_dots writes partial dots)
//   u_{j+1} = scale_j w - sum_i c_i scale_i u_i (lz_update reduces the dots
//   alpha_j = Re c_j                             and writes partial norms)
//   beta_j = |u_{j+1}|, scale_{j+1} = 1/beta_j  (reduced by lz_dots of step j+1)
// so no separate normalisation pass is needed.  Grid-wide sums are never
// finished inside the kernel that produces them: each kernel writes one
// partial per work-group, and every work-group of the NEXT kernel adds those
// partials in work-group order (kernel boundaries order the memory; no
// atomics or fences).  The breakdown test for step j-1 is therefore taken at
// the start of lz_dots(j); a stopped solve makes every later kernel return
// at once, so one fixed launch sequence serves every Krylov length.
#include <type_traits>

#include "common.h"

namespace tdvp {

namespace {

template <typename T> __device__ __forceinline__ T *shift_bytes(T *p, int64_t bytes) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<typename std::remove_const<T>::type *>(p)) + bytes);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of v over a 256-thread block, result valid in every thread.
__device__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

// exp(z T) e_1 for the k x k real symmetric tridiagonal T(alpha, beta),
// computed by one wave64 (lane i holds component i): T is shifted by the
// mean of its diagonal (the shift returns as the scalar factor
// exp(z shift)); the interval is cut into s pieces with
// theta = |z| |T'| / s <= 2 (Gershgorin bound on |T'|), and on each piece
// the Taylor series of exp is summed to m terms, m the smallest with
// theta^(m+1) / (m+1)! <= 1e-17 (a bound on the truncation error of a
// piece relative to the unit-norm vector it acts on).
// Writes k complex coefficients to (outr, outi).
__device__ void exp_tridiag_e1_wave(const double *alpha, const double *beta, int k, double zr,
                                    double zi, double *outr, double *outi) {
  const int lane = threadIdx.x & 63;
  const bool act = lane < k;
  double a = act ? alpha[lane] : 0.0;
  const double bu = (lane + 1 < k) ? beta[lane] : 0.0;       // T[lane][lane+1]
  const double shift = wave_sum(a) / (double)k;
  a = act ? a - shift : 0.0;
  const double bd = __shfl_up(bu, 1, 64);                    // T[lane][lane-1]
  const double bdl = (lane > 0 && act) ? bd : 0.0;
  const double gersh = wave_max(fabs(a) + fabs(bu) + fabs(bdl));
  const double zabs = sqrt(zr * zr + zi * zi);
  const double pieces = ceil(zabs * gersh / 2.0);
  // a non-finite T (from a non-finite input) gives one piece: the result is
  // non-finite but the loop stays bounded
  int ns = (pieces >= 1.0 && pieces <= 65536.0) ? (int)pieces : (pieces > 65536.0 ? 65536 : 1);
  const double hr = zr / ns, hi = zi / ns;
  const double theta = zabs * gersh / ns;
  int mterms = 1;
  {
    double term = theta;   // theta^m / m!
    while (mterms < 40 && term * theta / (mterms + 1) > 1e-17) {
      term *= theta / (mterms + 1);
      ++mterms;
    }
    mterms += 1;
  }
  double vr = (lane == 0) ? 1.0 : 0.0, vi = 0.0;
  for (int s = 0; s < ns; ++s) {
    double tr = vr, ti = vi, sr = vr, si = vi;
    for (int t = 1; t <= mterms; ++t) {
      const double tmr = __shfl_up(tr, 1, 64), tmi = __shfl_up(ti, 1, 64);
      const double tpr = __shfl_down(tr, 1, 64), tpi = __shfl_down(ti, 1, 64);
      double xr = a * tr + bdl * tmr + bu * tpr;
      double xi = a * ti + bdl * tmi + bu * tpi;
      if (!act) { xr = 0.0; xi = 0.0; }
      const double inv = 1.0 / (double)t;
      tr = (hr * xr - hi * xi) * inv;
      ti = (hr * xi + hi * xr) * inv;
      sr += tr;
      si += ti;
    }
    vr = sr;
    vi = si;
  }
  // multiply by exp(z shift)
  const double er = exp(zr * shift);
  double sn, cs;
  sincos(zi * shift, &sn, &cs);
  const double pr = er * cs, pi = er * sn;
  if (act) {
    outr[lane] = vr * pr - vi * pi;
    outi[lane] = vr * pi + vi * pr;
  }
}

__global__ __launch_bounds__(LZ_BLOCK) void lz_start_kernel(LzState *st, LzPartials *pp,
                                                            const double2 *x, double2 *u0,
                                                            int64_t n, double zr, double zi,
                                                            double tol, int keff, LzInst in) {
  const int64_t wo = (int64_t)blockIdx.y * in.wss;
  st = shift_bytes(st, wo);
  pp = shift_bytes(pp, wo);
  u0 = shift_bytes(u0, wo);
  x += (int64_t)blockIdx.y * in.xs;
  __shared__ double sh[8];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = x[e];
    u0[e] = v;
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    pp->nrm[blockIdx.x] = s;
    if (blockIdx.x == 0) {
      st->stop = 0;
      st->k = 0;
      st->keff = keff;
      st->z_re = zr;
      st->z_im = zi;
      st->tol = tol;
    }
  }
}

// Start of step j: close step j-1 (beta_{j-1}, breakdown and tolerance
// tests, scale_j), then w = sum_p ypart[p] -> U[j+1] with per-block partial
// dots <u_i, w> (i <= j) and |w|^2.
template <typename TY, int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_dots_kernel(LzState *st, LzPartials *pp,
                                                           const TY *ypart, int P,
                                                           int64_t pstride, double2 *U,
                                                           int64_t ldu, int j, int64_t n,
                                                           LzInst in) {
  {
    const int64_t wo = (int64_t)blockIdx.y * in.wss;
    st = shift_bytes(st, wo);
    pp = shift_bytes(pp, wo);
    ypart = shift_bytes(ypart, wo);
    U = shift_bytes(U, wo);
  }
  if (st->stop) return;
  __shared__ int stop_s;
  __shared__ double coefr[KMAX], coefi[KMAX];
  const int G = gridDim.x;
  __shared__ double nrm_s;
  if (threadIdx.x < 64) {   // fixed-order tree sum of the previous kernel's partial norms
    double t = 0.0;
    for (int b = threadIdx.x; b < G; b += 64) t += pp->nrm[b];
    t = wave_sum(t);
    if (threadIdx.x == 0) nrm_s = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = nrm_s;
    const double nv = sqrt(t);
    int stop = 0;
    if (j == 0) {
      if (!(nv > 0.0) || !isfinite(nv)) stop = 1;
      if (blockIdx.x == 0) {
        st->xnorm = nv;
        st->scale[0] = stop ? 0.0 : 1.0 / nv;
      }
    } else {
      if (!(nv > 1e-12 * st->aw[j - 1]) || !isfinite(nv) || j >= st->keff) stop = 1;
      if (!stop && blockIdx.x == 0) {
        st->beta[j - 1] = nv;
        st->scale[j] = 1.0 / nv;
      }
    }
    stop_s = stop;
  }
  __syncthreads();
  if (!stop_s && j > 0 && st->tol > 0.0) {
    // a-posteriori estimate |z beta_{j-1} [exp(z T_j) e_1]_{j-1}| (every block alike)
    const double bj = sqrt(nrm_s);
    if (threadIdx.x < 64) {
      // T_j needs beta_0 .. beta_{j-2}, all written by earlier kernels
      exp_tridiag_e1_wave(st->alpha, st->beta, j, st->z_re, st->z_im, coefr, coefi);
      if (threadIdx.x == 0) {
        const double zabs = sqrt(st->z_re * st->z_re + st->z_im * st->z_im);
        const double c = sqrt(coefr[j - 1] * coefr[j - 1] + coefi[j - 1] * coefi[j - 1]);
        if (zabs * bj * c < st->tol) stop_s = 1;
      }
    }
    __syncthreads();
  }
  if (stop_s) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->k = j;
      st->stop = 1;
    }
    return;
  }
  // Chunks of 256 elements.  Phase 1: w for the chunk (one element per
  // thread) into LDS and U[j+1].  Phase 2: thread (g, t), g = tid / 32,
  // t = tid % 32, accumulates <u_i, w> over the chunk for i = g, g+8, g+16,
  // g+24: 32 independent loads per thread per chunk.
  constexpr int NQ = (JB + 7) / 8;
  __shared__ double2 wl[LZ_BLOCK];
  __shared__ double w2s[LZ_BLOCK / 64];
  const int g8 = threadIdx.x >> 5, t32 = threadIdx.x & 31;
  double ar[NQ], ai[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
  double w2 = 0.0;
  double2 *wdst = U + (int64_t)(j + 1) * ldu;
  for (int64_t c0 = (int64_t)blockIdx.x * LZ_BLOCK; c0 < n; c0 += (int64_t)G * LZ_BLOCK) {
    const int64_t e = c0 + threadIdx.x;
    double wr = 0.0, wi = 0.0;
    if (e < n) {
#pragma unroll 4
      for (int p = 0; p < P; ++p) {
        const TY v = ypart[(int64_t)p * pstride + e];
        wr += (double)v.x;
        wi += (double)v.y;
      }
      wdst[e] = make_double2(wr, wi);
      w2 += wr * wr + wi * wi;
    }
    wl[threadIdx.x] = make_double2(wr, wi);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = g8 + 8 * q;
      if (i <= j) {
        const double2 *ui = U + (int64_t)i * ldu + c0;
#pragma unroll
        for (int t = 0; t < LZ_BLOCK / 32; ++t) {
          const int el = t32 + 32 * t;
          if (c0 + el < n) {
            const double2 u = ui[el];
            const double2 w = wl[el];
            ar[q] += u.x * w.x + u.y * w.y;
            ai[q] += u.x * w.y - u.y * w.x;
          }
        }
      }
    }
    __syncthreads();
  }
  // reduce over the 32 threads of each group (half a wave), fixed tree
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      ar[q] += __shfl_xor(ar[q], o, 32);
      ai[q] += __shfl_xor(ai[q], o, 32);
    }
    const int i = g8 + 8 * q;
    if (t32 == 0 && i <= j) {
      pp->dre[blockIdx.x][i] = ar[q];
      pp->dim[blockIdx.x][i] = ai[q];
    }
  }
  w2 = wave_sum(w2);
  if ((threadIdx.x & 63) == 0) w2s[threadIdx.x >> 6] = w2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < LZ_BLOCK / 64; ++w) a += w2s[w];
    pp->w2[blockIdx.x] = a;
  }
}

// u_{j+1} = scale_j w - sum_{i<=j} c_i scale_i u_i ; per-block |u_{j+1}|^2.
template <int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_update_kernel(LzState *st, LzPartials *pp,
                                                             double2 *U, int64_t ldu, int j,
                                                             int64_t n, LzInst in) {
  {
    const int64_t wo = (int64_t)blockIdx.y * in.wss;
    st = shift_bytes(st, wo);
    pp = shift_bytes(pp, wo);
    U = shift_bytes(U, wo);
  }
  if (st->stop) return;
  __shared__ double sh[8];
  __shared__ double cr[JB], ci[JB];
  const int G = gridDim.x;
  const double sj = st->scale[j];
  if (threadIdx.x <= j) {
    const int i = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int blk = 0; blk < G; ++blk) { a += pp->dre[blk][i]; b += pp->dim[blk][i]; }
    const double si = st->scale[i];
    const double sc = si * sj;
    cr[i] = a * sc * si;      // c_i scale_i
    ci[i] = b * sc * si;
    if (i == j && blockIdx.x == 0) st->alpha[j] = a * sc;
  }
  if (threadIdx.x == 32 && blockIdx.x == 0) {
    double t = 0.0;
    for (int blk = 0; blk < G; ++blk) t += pp->w2[blk];
    st->aw[j] = sqrt(t) * sj;
  }
  __syncthreads();
  double2 *w = U + (int64_t)(j + 1) * ldu;
  double s2 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double2 wv = w[e];
    double xr = sj * wv.x, xi = sj * wv.y;
#pragma unroll 8
    for (int i = 0; i <= j; ++i) {
      const double2 u = U[(int64_t)i * ldu + e];
      xr -= cr[i] * u.x - ci[i] * u.y;
      xi -= cr[i] * u.y + ci[i] * u.x;
    }
    w[e] = make_double2(xr, xi);
    s2 += xr * xr + xi * xi;
  }
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) pp->nrm[blockIdx.x] = s2;
}

// y = |x| sum_i [exp(z T_k) e_1]_i v_i with k = the final basis size (keff
// unless the solve stopped early).  Every block evaluates the small
// exponential redundantly (wave 0), then combines its slice of the basis.
__global__ __launch_bounds__(LZ_BLOCK) void lz_finish_kernel(LzState *st, const double2 *U,
                                                             int64_t ldu, int64_t n, int keff,
                                                             double2 *y, int32_t *k_used,
                                                             LzInst in) {
  {
    const int64_t wo = (int64_t)blockIdx.y * in.wss;
    st = shift_bytes(st, wo);
    U = shift_bytes(U, wo);
    y += (int64_t)blockIdx.y * in.ys;
    if (k_used) k_used += blockIdx.y;
  }
  __shared__ double cr[KMAX], ci[KMAX];
  const int k = st->stop ? st->k : keff;
  const double xn = st->xnorm;
  const bool zero = !(xn > 0.0) || k <= 0;
  if (!zero && threadIdx.x < 64)
    exp_tridiag_e1_wave(st->alpha, st->beta, k, st->z_re, st->z_im, cr, ci);
  __syncthreads();
  if (!zero && threadIdx.x < k) {
    const double sc = xn * st->scale[threadIdx.x];
    cr[threadIdx.x] *= sc;
    ci[threadIdx.x] *= sc;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double yr = 0.0, yi = 0.0;
    if (!zero) {
      for (int i = 0; i < k; ++i) {
        const double2 u = U[(int64_t)i * ldu + e];
        yr += cr[i] * u.x - ci[i] * u.y;
        yi += cr[i] * u.y + ci[i] * u.x;
      }
    }
    y[e] = make_double2(yr, yi);
  }
  if (k_used && blockIdx.x == 0 && threadIdx.x == 0) *k_used = zero ? 0 : k;
}

// Work-groups for an n-element vector pass: one element per thread, at most
// LZ_GRID groups (so the partial sums stay short).
int grid_for(int64_t n) {
  int64_t g = (n + LZ_BLOCK - 1) / LZ_BLOCK;
  if (g > LZ_GRID) g = LZ_GRID;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t lz_start(LzState *st, LzPartials *pp, const double2 *x, double2 *u0, int64_t n,
                    double zr, double zi, double tol, int keff, const LzInst &in, hipStream_t s) {
  hipLaunchKernelGGL(lz_start_kernel, dim3(grid_for(n), in.count), dim3(LZ_BLOCK), 0, s, st, pp, x,
                     u0, n, zr, zi, tol, keff, in);
  return hipGetLastError();
}

hipError_t lz_dots(LzState *st, LzPartials *pp, DType ty, const void *ypart, int P, int64_t pstride,
                   double2 *U, int64_t ldu, int j, int64_t n, const LzInst &in, hipStream_t s) {
  const dim3 g(grid_for(n), in.count), b(LZ_BLOCK);
#define LZ_DOTS(T, JB)                                                                         \
  hipLaunchKernelGGL((lz_dots_kernel<T, JB>), g, b, 0, s, st, pp, (const T *)ypart, P, pstride, \
                     U, ldu, j, n, in)
  if (ty == F64) {
    if (j < 4) LZ_DOTS(double2, 4);
    else if (j < 8) LZ_DOTS(double2, 8);
    else if (j < 16) LZ_DOTS(double2, 16);
    else LZ_DOTS(double2, 32);
  } else {
    if (j < 4) LZ_DOTS(float2, 4);
    else if (j < 8) LZ_DOTS(float2, 8);
    else if (j < 16) LZ_DOTS(float2, 16);
    else LZ_DOTS(float2, 32);
  }
#undef LZ_DOTS
  return hipGetLastError();
}

hipError_t lz_update(LzState *st, LzPartials *pp, double2 *U, int64_t ldu, int j, int64_t n,
                     const LzInst &in, hipStream_t s) {
  const dim3 g(grid_for(n), in.count), b(LZ_BLOCK);
  if (j < 4) hipLaunchKernelGGL((lz_update_kernel<4>), g, b, 0, s, st, pp, U, ldu, j, n, in);
  else if (j < 8) hipLaunchKernelGGL((lz_update_kernel<8>), g, b, 0, s, st, pp, U, ldu, j, n, in);
  else if (j < 16) hipLaunchKernelGGL((lz_update_kernel<16>), g, b, 0, s, st, pp, U, ldu, j, n, in);
  else hipLaunchKernelGGL((lz_update_kernel<32>), g, b, 0, s, st, pp, U, ldu, j, n, in);
  return hipGetLastError();
}

hipError_t lz_finish(LzState *st, const double2 *U, int64_t ldu, int64_t n, int keff, double2 *y,
                     int32_t *k_used, const LzInst &in, hipStream_t s) {
  hipLaunchKernelGGL(lz_finish_kernel, dim3(grid_for(n), in.count), dim3(LZ_BLOCK), 0, s, st, U,
                     ldu, n, keff, y, k_used, in);
  return hipGetLastError();
}

}  // namespace tdvp
