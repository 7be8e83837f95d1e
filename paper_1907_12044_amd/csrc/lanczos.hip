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
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "mfma.h"

namespace tdvp {

namespace {

template <typename T> __device__ __forceinline__ T *shift_bytes(T *p, int64_t bytes) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<typename std::remove_const<T>::type *>(p)) + bytes);
}

// largest power of two <= x (x >= 1)
constexpr int pow2_floor(int x) {
  int p = 1;
  while (2 * p <= x) p *= 2;
  return p;
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

// Neighbour exchange across the whole wave through DPP wave shifts (no LDS
// round trip): shr1 gives lane i the value of lane i-1 (lane 0: 0), shl1
// the value of lane i+1 (lane 63: 0).
__device__ __forceinline__ double wave_shr1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_shl1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// value of v in lane l (l uniform across the wave)
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
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
  const double inv_lane = 1.0 / (double)(lane + 1);   // 1/t for term t = lane + 1
  double vr = (lane == 0) ? 1.0 : 0.0, vi = 0.0;
  for (int s = 0; s < ns; ++s) {
    double tr = vr, ti = vi, sr = vr, si = vi;
    for (int t = 1; t <= mterms; ++t) {
      const double tmr = wave_shr1(tr), tmi = wave_shr1(ti);
      const double tpr = wave_shl1(tr), tpi = wave_shl1(ti);
      double xr = a * tr + bdl * tmr + bu * tpr;
      double xi = a * ti + bdl * tmi + bu * tpi;
      if (!act) { xr = 0.0; xi = 0.0; }
      const double inv = lane_value(inv_lane, t - 1);
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

// Start of Lanczos step j, run by every work-group of the kernel that opens
// the step: add the Gprev partial norms of the previous kernel (fixed
// tree), then close step j-1: beta_{j-1} and scale_j, the breakdown test
// beta_{j-1} <= 1e-12 |H v_{j-1}|, the basis-size limit and, with tol > 0,
// the a-posteriori estimate |z beta_{j-1} [exp(z T_j) e_1]_{j-1}| < tol.
// |H v_{j-1}| is st->aw[j-1] (Gw == 0) or comes from the Gw partials
// pp->w2 of |H u_{j-1}|^2.  Work-group 0 records the scalars.  Returns true
// (in every thread) if the basis is final; the caller then returns.
// The loads of close_step, issued by wave 0 (Gprev, Gw <= LZ_GRID) so that a
// kernel can request them together with its other inputs.
constexpr int SP_Q = LZ_GRID / 64;   // partials per lane of wave 0
struct StepPre {
  double nr[SP_Q], w2[SP_Q];
  double aw, sprev, tol;
  int keff;
};
__device__ __forceinline__ void close_step_load(const LzState *st, const LzPartials *pp, int Gprev,
                                                int j, int Gw, StepPre &p,
                                                const double *nrm = nullptr) {
  if (!nrm) nrm = pp->nrm;
#pragma unroll
  for (int q = 0; q < SP_Q; ++q) p.nr[q] = p.w2[q] = 0.0;
  p.aw = p.sprev = p.tol = 0.0;
  p.keff = 0;
  if (threadIdx.x < 64) {
#pragma unroll
    for (int q = 0; q < SP_Q; ++q) {
      const int b = threadIdx.x + 64 * q;
      if (b < Gprev) p.nr[q] = nrm[b];
      if (j > 0 && b < Gw) p.w2[q] = pp->w2[b];
    }
    if (threadIdx.x == 0) {
      p.tol = st->tol;
      if (j > 0) {
        p.keff = st->keff;
        if (Gw > 0) p.sprev = st->scale[j - 1];
        else p.aw = st->aw[j - 1];
      }
    }
  }
}

__device__ bool close_step_finish(LzState *st, const StepPre &p, int j, int Gw, int bx,
                                  double *scale_out = nullptr) {
  __shared__ int stop_s;
  __shared__ double nrm_s, aw_s, tol_s;
  __shared__ double coefr[KMAX], coefi[KMAX];
  if (threadIdx.x < 64) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < SP_Q; ++q) {
      a += p.nr[q];
      b += p.w2[q];
    }
    double t = wave_sum(a);
    double t2 = wave_sum(b);
    if (threadIdx.x == 0) {
      nrm_s = t;
      aw_s = Gw > 0 ? sqrt(t2) * p.sprev : p.aw;
      tol_s = p.tol;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double nv = sqrt(nrm_s);
    int stop = 0;
    // a non-finite norm (from a non-finite input or operator) stops the
    // solve and raises the sticky flag that tdvp_observe reports
    const bool bad = !isfinite(nv) || !isfinite(aw_s);
    if (bad && bx == 0) *st->nonfinite = 1;
    if (j == 0) {
      if (!(nv > 0.0) || bad) stop = 1;
      if (bx == 0) {
        st->xnorm = nv;
        st->scale[0] = stop ? 0.0 : 1.0 / nv;
      }
    } else {
      if (!(nv > 1e-12 * aw_s) || bad || j >= p.keff) stop = 1;
      if (!stop && bx == 0) {
        st->beta[j - 1] = nv;
        st->scale[j] = 1.0 / nv;
      }
    }
    if (scale_out) *scale_out = stop ? 0.0 : 1.0 / nv;   // (shared; read after the barrier below)
    stop_s = stop;
  }
  __syncthreads();
  if (!stop_s && j > 0 && tol_s > 0.0) {
    const double bj = sqrt(nrm_s);
    if (threadIdx.x < 64) {
      // T_j needs beta_0 .. beta_{j-2}, all written by earlier kernels
      exp_tridiag_e1_wave(st->alpha, st->beta, j, st->z_re, st->z_im, coefr, coefi);
      if (threadIdx.x == 0) {
        const double zabs = sqrt(st->z_re * st->z_re + st->z_im * st->z_im);
        const double c = sqrt(coefr[j - 1] * coefr[j - 1] + coefi[j - 1] * coefi[j - 1]);
        if (zabs * bj * c < tol_s) stop_s = 1;
      }
    }
    __syncthreads();
  }
  const bool stop = stop_s != 0;
  if (stop && bx == 0 && threadIdx.x == 0) {
    st->k = j;
    st->stop = 1;
  }
  return stop;
}


constexpr int LU_E = 64;
// Work-groups per instance of lz_start, lz_update and lz_finish (the first
// two write one norm partial each): LU_E elements per work-group and pass,
// at most LZ_GRID, and for a batch of `count` instances no more than give
// ~1024 work-groups in all (a batch fills the chip with fewer work-groups
// per instance, and each runs more passes with the next pass's loads in
// flight).  One instance: min(n / LU_E, LZ_GRID).
__host__ __device__ inline int upd_grid(int64_t n, int count) {
  int64_t g = (n + LU_E - 1) / LU_E;
  if (g > LZ_GRID) g = LZ_GRID;
  const int c = count > 1 ? count : 1;
  const int64_t want = (1024 + c - 1) / c;
  if (g > want) g = want < 16 ? 16 : want;
  if (g < 1) g = 1;
  return (int)g;
}

__device__ __forceinline__ void lz_start_body(LzState *st, LzPartials *pp, const double2 *x,
                                              double2 *u0, int64_t n, double zr, double zi,
                                              double tol, int keff, int trows, int *nonfinite,
                                              LzInst in, const BlockXYZ &blk) {
  const int64_t wo = (int64_t)blk.y * in.wss;
  st = shift_bytes(st, wo);
  pp = shift_bytes(pp, wo);
  u0 = shift_bytes(u0, wo);
  x += (int64_t)blk.y * in.xs;
  __shared__ double sh[8];
  double s = 0.0;
  const int64_t tcols = trows > 0 ? n / trows : 0;
  for (int64_t e = (int64_t)blk.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)blk.gx * blockDim.x) {
    // column-major basis: u0[c * trows + r] = x[r * tcols + c]
    const double2 v = trows > 0 ? x[(e % trows) * tcols + e / trows] : x[e];
    u0[e] = v;
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    pp->nrm[blk.x] = s;
    if (blk.x == 0) {
      st->stop = 0;
      st->k = 0;
      st->keff = keff;
      st->z_re = zr;
      st->z_im = zi;
      st->tol = tol;
      st->nonfinite = nonfinite;
    }
  }
}

__global__ __launch_bounds__(LZ_BLOCK) void lz_start_kernel(LzState *st, LzPartials *pp,
                                                            const double2 *x, double2 *u0,
                                                            int64_t n, double zr, double zi,
                                                            double tol, int keff, int trows,
                                                            int *nonfinite, LzInst in) {
  lz_start_body(st, pp, x, u0, n, zr, zi, tol, keff, trows, nonfinite, in, native_block());
}
__global__ __launch_bounds__(LZ_BLOCK) void lz_start_grouped_kernel(Grp<LzStartArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  const LzStartArgs &a = g.a[k];
  lz_start_body(a.st, a.pp, a.x, a.u0, a.n, a.zr, a.zi, a.tol, a.keff, a.trows, a.nonfinite, a.in, b);
}

// Start of step j: close step j-1 (beta_{j-1}, breakdown and tolerance
// tests, scale_j), then w = sum_p ypart[p] -> U[j+1] with per-block partial
// dots <u_i, w> (i <= j) and |w|^2.
// The element layout is lz_update's: a work-group takes LU_E elements per
// pass, wave q projects onto u_i for i = q, q + 4, ..., and every wave forms
// w for the pass from the P parts itself (the four waves read the same
// parts; the repeats hit the cache), so no pass needs a barrier; wave 0
// stores w and adds |w|^2.  The loads of the next pass are issued before
// the arithmetic of this one.
template <typename TY, int JB>
__device__ __forceinline__ void lz_dots_body(LzState *st, LzPartials *pp, const TY *ypart, int P,
                                             int64_t pstride, double2 *U, int64_t ldu, int j,
                                             int64_t n, LzInst in, const BlockXYZ &blk) {
  {
    const int64_t wo = (int64_t)blk.y * in.wss;
    st = shift_bytes(st, wo);
    pp = shift_bytes(pp, wo);
    ypart = shift_bytes(ypart, wo);
    U = shift_bytes(U, wo);
  }
  // the stop flag is loaded with the other inputs and tested before any write
  const int stopped = st->stop;
  StepPre pre;
  close_step_load(st, pp, upd_grid(n, in.count), j, 0, pre);
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  constexpr int NI = (JB + 3) / 4;        // basis vectors per wave
  constexpr int PR = 4;                   // parts of w held in registers (more: loaded after)
  double2 *wdst = U + (int64_t)(j + 1) * ldu;
  const int64_t b0 = (int64_t)blk.x * LU_E, bstride = (int64_t)blk.gx * LU_E;
  double2 uv[NI];
  TY yv[PR];
  auto load = [&](int64_t e) {
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int i = q + 4 * t;
      uv[t] = (i <= j && e < n) ? U[(int64_t)i * ldu + e] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int p = 0; p < PR; ++p) {
      yv[p].x = 0;
      yv[p].y = 0;
      if (p < P && e < n) yv[p] = ypart[(int64_t)p * pstride + e];
    }
  };
  load(b0 + lane);
  if (stopped || close_step_finish(st, pre, j, 0, blk.x)) return;   // (synchronises the work-group)
  double ar[NI], ai[NI];
#pragma unroll
  for (int t = 0; t < NI; ++t) { ar[t] = 0.0; ai[t] = 0.0; }
  double w2 = 0.0;
  for (int64_t base = b0; base < n; base += bstride) {
    const int64_t e = base + lane;
    double2 ucur[NI];
    TY ycur[PR];
#pragma unroll
    for (int t = 0; t < NI; ++t) ucur[t] = uv[t];
#pragma unroll
    for (int p = 0; p < PR; ++p) ycur[p] = yv[p];
    if (base + bstride < n) load(base + bstride + lane);
    double wr = 0.0, wi = 0.0;
    if (e < n) {
#pragma unroll
      for (int p = 0; p < PR; ++p) {
        wr += (double)ycur[p].x;
        wi += (double)ycur[p].y;
      }
      for (int p = PR; p < P; ++p) {
        const TY v = ypart[(int64_t)p * pstride + e];
        wr += (double)v.x;
        wi += (double)v.y;
      }
      if (q == 0) {
        wdst[e] = make_double2(wr, wi);
        w2 += wr * wr + wi * wi;
      }
    }
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      if (q + 4 * t <= j) {
        ar[t] += ucur[t].x * wr + ucur[t].y * wi;
        ai[t] += ucur[t].x * wi - ucur[t].y * wr;
      }
    }
  }
  // wave sums (fixed tree) -> one partial per work-group and basis vector
#pragma unroll
  for (int t = 0; t < NI; ++t) {
    const int i = q + 4 * t;
    const double a = wave_sum(ar[t]), b = wave_sum(ai[t]);
    if (lane == 0 && i <= j) pp->dot[i][blk.x] = make_double2(a, b);
  }
  if (q == 0) {
    w2 = wave_sum(w2);
    if (lane == 0) pp->w2[blk.x] = w2;
  }
}

template <typename TY, int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_dots_kernel(LzState *st, LzPartials *pp,
                                                           const TY *ypart, int P,
                                                           int64_t pstride, double2 *U,
                                                           int64_t ldu, int j, int64_t n,
                                                           LzInst in) {
  lz_dots_body<TY, JB>(st, pp, ypart, P, pstride, U, ldu, j, n, in, native_block());
}
template <typename TY, int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_dots_grouped_kernel(Grp<LzDotsArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  const LzDotsArgs &a = g.a[k];
  lz_dots_body<TY, JB>(a.st, a.pp, (const TY *)a.ypart, a.P, a.pstride, a.U, a.ldu, a.j, a.n, a.in, b);
}

// u_{j+1} = scale_j w - sum_{i<=j} c_i scale_i u_i ; per-block |u_{j+1}|^2.
// w is U[j+1] (written by lz_dots), or on the fused path the sum of the P
// partial vectors Yp[p] (then the per-block |w|^2 partials are written too).
// A work-group takes LU_E elements per pass; wave q adds the basis vectors
// i = q, q + 4, ... and the partial vectors p = q, q + 4, ..., and wave 0
// combines the four wave sums in order.  A thread's loads for its first
// pass are issued before the reduction of the dot partials, so the two
// latencies overlap.
template <int JB>
__device__ __forceinline__ void lz_update_body(LzState *st, LzPartials *pp, double2 *U, int64_t ldu,
                                               int j, int64_t n, int Gd, const double2 *Yp, int P,
                                               LzInst in, const BlockXYZ &blk, int close = 0) {
  {
    const int64_t wo = (int64_t)blk.y * in.wss;
    st = shift_bytes(st, wo);
    pp = shift_bytes(pp, wo);
    U = shift_bytes(U, wo);
    if (Yp) Yp = shift_bytes(Yp, wo);
  }
  // the stop flag was written by the previous kernel: its load is issued
  // together with this kernel's other loads (all of them read memory that
  // exists whether or not the solve has stopped) and tested before any write
  const int stopped = st->stop;
  __shared__ double sh[8];
  __shared__ double cr[JB], ci[JB];
  __shared__ double2 pw[4][LU_E], ps[4][LU_E];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  double2 *w = U + (int64_t)(j + 1) * ldu;
  const int64_t b0 = (int64_t)blk.x * LU_E, bstride = (int64_t)blk.gx * LU_E;
  constexpr int NI = (JB + 3) / 4;         // basis vectors per wave
  constexpr int NP = (HS_PMAX + 3) / 4;    // partial vectors per wave
  double2 uv[NI], yv[NP];
#define LZ_UPDATE_LOAD(e)                                                                  \
  do {                                                                                     \
    _Pragma("unroll") for (int t = 0; t < NP; ++t) {                                       \
      const int p = q + 4 * t;                                                             \
      yv[t] = make_double2(0.0, 0.0);                                                      \
      if ((e) < n) {                                                                       \
        if (Yp) {                                                                          \
          if (p < P) yv[t] = Yp[(int64_t)p * n + (e)];                                     \
        } else if (p == 0) {                                                               \
          yv[t] = w[e];                                                                    \
        }                                                                                  \
      }                                                                                    \
    }                                                                                      \
    _Pragma("unroll") for (int t = 0; t < NI; ++t) {                                       \
      const int i = q + 4 * t;                                                             \
      uv[t] = (i <= j && (e) < n) ? U[(int64_t)i * ldu + (e)] : make_double2(0.0, 0.0);   \
    }                                                                                      \
  } while (0)
  if (b0 < n) LZ_UPDATE_LOAD(b0 + lane);
  if (Gd < 0) Gd = pp->ndot;
  double sj;
  if (close) {
    // close step j - 1 here (the projections came from a GEMM epilogue)
    __shared__ double sj_s;
    StepPre pre;
    close_step_load(st, pp, upd_grid(n, in.count), j, 0, pre, ((j - 1) & 1) ? pp->nrm : pp->nrm_odd);
    if (stopped || close_step_finish(st, pre, j, 0, blk.x, &sj_s)) return;   // (synchronises)
    sj = sj_s;
  } else {
    sj = st->scale[j];
  }
  // Reduce the Gd dot partials of the previous kernel: LPI lanes per basis
  // index i (256 / JB rounded down to a power of two; lane l adds partials
  // l, l + LPI, ...), then a fixed tree over the LPI lanes.
  {
    constexpr int LPI = pow2_floor(LZ_BLOCK / JB);
    static_assert(LPI * JB <= LZ_BLOCK && LPI <= 64, "lanes per basis index");
    const int i = threadIdx.x / LPI, l8 = threadIdx.x % LPI;
    double a = 0.0, b = 0.0;
    if (i <= j) {
      const double2 *dp = pp->dot[i];
#pragma unroll 8
      for (int blk = l8; blk < Gd; blk += LPI) {
        const double2 v = dp[blk];
        a += v.x;
        b += v.y;
      }
    }
#pragma unroll
    for (int o = LPI / 2; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, LPI);
      b += __shfl_xor(b, o, LPI);
    }
    if (stopped) return;   // (the same value in every thread)
    if (l8 == 0 && i <= j) {
      // scale_j: this kernel's own close (WG 0 writes it to st concurrently)
      const double si = i == j ? sj : st->scale[i];
      const double sc = si * sj;
      cr[i] = a * sc * si;      // c_i scale_i
      ci[i] = b * sc * si;
      if (i == j && blk.x == 0) st->alpha[j] = a * sc;
    }
    if (!Yp && blk.x == 0 && threadIdx.x >= 192) {   // last wave: |H v_j|
      double t = 0.0;
      for (int blk = threadIdx.x - 192; blk < Gd; blk += 64) t += pp->w2[blk];
      t = wave_sum(t);
      if (threadIdx.x == 192) st->aw[j] = sqrt(t) * sj;
    }
  }
  __syncthreads();
  double s2 = 0.0, sw = 0.0;
  for (int64_t base = b0; base < n; base += bstride) {
    const int64_t e = base + lane;
    // this pass's inputs, then the next pass's loads (issued before the arithmetic)
    double2 ucur[NI], ycur[NP];
#pragma unroll
    for (int t = 0; t < NI; ++t) ucur[t] = uv[t];
#pragma unroll
    for (int t = 0; t < NP; ++t) ycur[t] = yv[t];
    if (base + bstride < n) LZ_UPDATE_LOAD(base + bstride + lane);
    double2 acc = ycur[0];
#pragma unroll
    for (int t = 1; t < NP; ++t) {
      acc.x += ycur[t].x;
      acc.y += ycur[t].y;
    }
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int i = q + 4 * t;
      if (i <= j) {
        sr += cr[i] * ucur[t].x - ci[i] * ucur[t].y;
        si += cr[i] * ucur[t].y + ci[i] * ucur[t].x;
      }
    }
    pw[q][lane] = acc;
    ps[q][lane] = make_double2(sr, si);
    __syncthreads();
    if (q == 0 && e < n) {
      double2 wv = pw[0][lane], sv = ps[0][lane];
#pragma unroll
      for (int t = 1; t < 4; ++t) {
        wv.x += pw[t][lane].x;
        wv.y += pw[t][lane].y;
        sv.x += ps[t][lane].x;
        sv.y += ps[t][lane].y;
      }
      const double xr = sj * wv.x - sv.x, xi = sj * wv.y - sv.y;
      w[e] = make_double2(xr, xi);
      s2 += xr * xr + xi * xi;
      sw += wv.x * wv.x + wv.y * wv.y;
    }
    __syncthreads();
  }
#undef LZ_UPDATE_LOAD
  s2 = block_sum(s2, sh);
  if (Yp) sw = block_sum(sw, sh + 4);
  if (threadIdx.x == 0) {
    if (close) (j & 1 ? pp->nrm : pp->nrm_odd)[blk.x] = s2;
    else pp->nrm[blk.x] = s2;
    if (Yp) pp->w2[blk.x] = sw;
  }
}

template <int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_update_kernel(LzState *st, LzPartials *pp,
                                                             double2 *U, int64_t ldu, int j,
                                                             int64_t n, int Gd,
                                                             const double2 *Yp, int P,
                                                             LzInst in, int close) {
  lz_update_body<JB>(st, pp, U, ldu, j, n, Gd, Yp, P, in, native_block(), close);
}
template <int JB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_update_grouped_kernel(Grp<LzUpdateArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  const LzUpdateArgs &a = g.a[k];
  lz_update_body<JB>(a.st, a.pp, a.U, a.ldu, a.j, a.n, a.Gd, a.Yp, a.P, a.in, b, a.close);
}

// y = |x| sum_i [exp(z T_k) e_1]_i v_i with k = the final basis size (keff
// unless the solve stopped early).  Every work-group evaluates the small
// exponential redundantly (wave 0) and combines LU_E elements per pass:
// wave q adds the basis vectors i = q, q + 4, ..., whose loads are issued
// before the exponential, and wave 0 adds the four wave sums in order.
template <int KB>
__device__ __forceinline__ void lz_finish_body(LzState *st, const double2 *U, int64_t ldu, int64_t n,
                                               int keff, double2 *y, int32_t *k_used, int trows,
                                               LzInst in, const BlockXYZ &blk) {
  {
    const int64_t wo = (int64_t)blk.y * in.wss;
    st = shift_bytes(st, wo);
    U = shift_bytes(U, wo);
    y += (int64_t)blk.y * in.ys;
    if (k_used) k_used += blk.y;
  }
  __shared__ double cr[KMAX], ci[KMAX];
  __shared__ double2 ps[4][LU_E];
  constexpr int NI = (KB + 3) / 4;         // basis vectors per wave
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blk.x * LU_E, bstride = (int64_t)blk.gx * LU_E;
  double2 uv[NI];
#define LZ_FINISH_LOAD(e)                                                                  \
  do {                                                                                     \
    _Pragma("unroll") for (int t = 0; t < NI; ++t) {                                       \
      const int i = q + 4 * t;                                                             \
      uv[t] = (i < keff && (e) < n) ? U[(int64_t)i * ldu + (e)] : make_double2(0.0, 0.0);  \
    }                                                                                      \
  } while (0)
  if (b0 < n) LZ_FINISH_LOAD(b0 + lane);
  const int k = st->stop ? st->k : keff;
  const double xn = st->xnorm;
  // a zero input gives y = 0; a non-finite one gives y = NaN (never a
  // finite-looking result)
  const bool nanout = !isfinite(xn);
  const bool zero = !(xn > 0.0) || k <= 0 || nanout;
  if (!zero && threadIdx.x < 64)
    exp_tridiag_e1_wave(st->alpha, st->beta, k, st->z_re, st->z_im, cr, ci);
  __syncthreads();
  if (!zero && threadIdx.x < k) {
    const double sc = xn * st->scale[threadIdx.x];
    cr[threadIdx.x] *= sc;
    ci[threadIdx.x] *= sc;
  }
  __syncthreads();
  for (int64_t base = b0; base < n; base += bstride) {
    const int64_t e = base + lane;
    double2 ucur[NI];
#pragma unroll
    for (int t = 0; t < NI; ++t) ucur[t] = uv[t];
    if (base + bstride < n) LZ_FINISH_LOAD(base + bstride + lane);
    double yr = nanout ? __builtin_nan("") : 0.0, yi = yr;
    if (!zero) {
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        const int i = q + 4 * t;
        if (i < k) {
          yr += cr[i] * ucur[t].x - ci[i] * ucur[t].y;
          yi += cr[i] * ucur[t].y + ci[i] * ucur[t].x;
        }
      }
    }
    ps[q][lane] = make_double2(yr, yi);
    __syncthreads();
    if (q == 0 && e < n) {
      double2 v = ps[0][lane];
#pragma unroll
      for (int t = 1; t < 4; ++t) {
        v.x += ps[t][lane].x;
        v.y += ps[t][lane].y;
      }
      if (trows > 0) {
        const int64_t tcols = n / trows;
        y[(e % trows) * tcols + e / trows] = v;
      } else {
        y[e] = v;
      }
    }
    __syncthreads();
  }
#undef LZ_FINISH_LOAD
  if (k_used && blk.x == 0 && threadIdx.x == 0) *k_used = zero ? 0 : k;
}

template <int KB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_finish_kernel(LzState *st, const double2 *U,
                                                             int64_t ldu, int64_t n, int keff,
                                                             double2 *y, int32_t *k_used,
                                                             int trows, LzInst in) {
  lz_finish_body<KB>(st, U, ldu, n, keff, y, k_used, trows, in, native_block());
}
template <int KB>
__global__ __launch_bounds__(LZ_BLOCK) void lz_finish_grouped_kernel(Grp<LzFinishArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  const LzFinishArgs &a = g.a[k];
  lz_finish_body<KB>(a.st, a.U, a.ldu, a.n, a.keff, a.y, a.k_used, a.trows, a.in, b);
}

// ---------------------------------------------------------------------------
// Fused Lanczos step: H[i] u_j (all three contraction stages) plus the
// projections <u_i, H u_j> in ONE launch.  Work-group (p, r') forms the part
// of output column r' of y[l', s', r'] that comes from the bra-side indices
// l in [l0, l0 + nl), l0 = p nl:
//   T1[(l, s)][wr] = sum_r u[(l, s)][r] R[r'][wr][r]        (MFMA, N = Wr <= 16)
//   T2[(wl, l)][s'] = sum_{nonzero W} W[wl][s'][s][wr] T1[(l, s)][wr]   (LDS)
//   y_p[l'][s']    = sum_{(wl, l)} L[l'][wl][l] T2[(wl, l)][s']  (MFMA)
// writes y_p to Yp[p] and the dots <u_i, y_p> to partial slot p Mr + r';
// lz_update adds the P parts (H u_j = sum_p y_p, dots likewise).  Splitting
// the sum over l spreads one column over P work-groups, so a small bond
// still fills the chip.  On this path the basis vectors are stored
// column-major (index r' Ml d + (l', s')), so a column is contiguous;
// lz_start and lz_finish convert from and to the row-major site tensor.
// With row == NULL the operator is the bond operator of eq:tdvp2_D (d = 1,
// T2 = T1^T).  The nonzeros of W come as a CSR table over rows (wl, s').

constexpr int HS_WAVES = 8;            // waves per work-group of the fused step
constexpr int HS_NZ = 512;             // W nonzeros staged in LDS (more: read from global)
constexpr int HS_RV = 4;               // R-slice elements per thread: Mr <= 128
constexpr int HS_XV = 4;               // staged x-slice elements per thread
constexpr int HS_LV = 8;               // staged L-slice elements per thread

// Complex C (Mrows x 16) = A (Mrows x K) B (K x 16) on the MFMA units of one
// work-group (three real products per complex one): 16-row tiles; when there are fewer tiles than waves the K
// range of a tile is split over several waves and the parts are added in
// order through `red` (HS_WAVES x 2 x 256 values).  A comes from
// loadA(row, k, re, im) (row < Mrows, k < K); B from LDS planes [K4][16]
// whose rows K..K4-1 are zero.  store(row, col, re, im) receives every
// result with row < Mrows.
template <typename T, typename LoadA, typename Store>
__device__ __forceinline__ void hs_mm16(int Mrows, int K, const T *b_re, const T *b_im, T *red,
                                        LoadA loadA, Store store) {
  using AccT = typename Mf<T>::acc;
  constexpr int NT = HS_WAVES * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int RT = (Mrows + 15) / 16, K4 = (K + 3) & ~3;
  const int TPR = min(RT, HS_WAVES), parts = HS_WAVES / TPR;
  const int kchunk = ((K4 / 4 + parts - 1) / parts) * 4;
  for (int rt0 = 0; rt0 < RT; rt0 += TPR) {
    AccT p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};   // Ar Br, Ai Bi, (Ar+Ai)(Br+Bi)
    const int rt = rt0 + wave % TPR, pt = wave / TPR;
    if (rt < RT && pt < parts) {
      const int kb = pt * kchunk, ke = min(K4, kb + kchunk);
      const int row = rt * 16 + (lane & 15);
#pragma unroll 8
      for (int k0 = kb; k0 < ke; k0 += 4) {
        const int k = k0 + (lane >> 4);
        T ar = 0, ai = 0;
        if (row < Mrows && k < K) loadA(row, k, ar, ai);
        const T br = b_re[k * 16 + (lane & 15)], bi = b_im[k * 16 + (lane & 15)];
        p1 = Mf<T>::mfma(ar, br, p1);
        p2 = Mf<T>::mfma(ai, bi, p2);
        p3 = Mf<T>::mfma(ar + ai, br + bi, p3);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[(wave * 2 + 0) * 256 + r * 64 + lane] = p1[r] - p2[r];
      red[(wave * 2 + 1) * 256 + r * 64 + lane] = p3[r] - p1[r] - p2[r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < min(RT - rt0, TPR) * 256; e += NT) {
      const int tt = e >> 8, rem = e & 255, r = rem >> 6, ln = rem & 63;
      T sr = 0, si = 0;
      for (int p = 0; p < parts; ++p) {
        const int w = p * TPR + tt;
        sr += red[(w * 2 + 0) * 256 + r * 64 + ln];
        si += red[(w * 2 + 1) * 256 + r * 64 + ln];
      }
      const int orow = (rt0 + tt) * 16 + Mf<T>::row(ln, r);
      if (orow < Mrows) store(orow, ln & 15, sr, si);
    }
    __syncthreads();
  }
}

// Stage 2 over the (K3 x d) block of T2: T2[(wl, ll)][s'] from T1 and the
// nonzero table: row pointers rp, columns cl, coefficients (cr, ci) staged
// in LDS, or the c128 table gc in global memory (GL).
template <typename T, bool GL, typename PI>
__device__ __forceinline__ void hs_stage2(T *t2_re, T *t2_im, const T *t1_re, const T *t1_im,
                                          int K3, int nl, int d, int cap, PI rp, PI cl,
                                          const T *cr, const T *ci, const double2 *gc) {
  for (int e = threadIdx.x; e < K3 * d; e += HS_WAVES * 64) {
    const int k = e / d, sp = e - k * d;
    const int wl = k / nl, ll = k - wl * nl;
    const int rw = wl * d + sp, q1 = rp[rw + 1];
    const T *tr_ = t1_re + ll * cap, *ti_ = t1_im + ll * cap;
    T re = 0, im = 0;
    for (int q = rp[rw]; q < q1; ++q) {
      const int cc = cl[q];
      T wre, wim;
      if (GL) {
        const double2 w = gc[q];
        wre = (T)w.x;
        wim = (T)w.y;
      } else {
        wre = cr[q];
        wim = ci[q];
      }
      const T tr = tr_[cc], ti = ti_[cc];
      re += wre * tr - wim * ti;
      im += wre * ti + wim * tr;
    }
    t2_re[k * 16 + sp] = re;
    t2_im[k * 16 + sp] = im;
  }
}

// LDS layout of the fused step (elements of T unless noted); `stg` adds
// the staged x and L slices.
struct HsLayout {
  int Mr4, MP, MP16, K3, K34, Ml16, T1P;
  int rr, t1, t2, red, xs, ls, ycol_b, nz_b, total_b;   // offsets (T elements; _b: bytes)
  __host__ __device__ HsLayout(int Ml, int d, int Mr, int Wl, int Wr, int nl, bool stg, int tb) {
    Mr4 = (Mr + 3) & ~3;
    MP = nl * d;
    MP16 = (MP + 15) & ~15;
    K3 = Wl * nl;
    K34 = (K3 + 3) & ~3;
    Ml16 = (Ml + 15) & ~15;
    T1P = (MP * Wr + 3) & ~3;
    rr = 0;
    t1 = rr + 2 * Mr4 * 16;
    t2 = t1 + 2 * T1P;
    red = t2 + 2 * K34 * 16;
    xs = red + HS_WAVES * 2 * 256;
    ls = xs + (stg ? 2 * Mr4 * MP16 : 0);
    const int tend = ls + (stg ? 2 * K34 * Ml16 : 0);
    ycol_b = tend * tb;
    nz_b = ycol_b + Ml * d * 16;
    total_b = nz_b + HS_NZ * (2 * tb + 4) + (Wl * d + 1) * 4;
  }
};

template <typename T, int JB, bool STG>
__device__ __forceinline__ void heff_small_body(const HeffSmallArgs &a, const BlockXYZ &blk) {
  using VE = typename Mf<T>::c2;
  constexpr int NT = HS_WAVES * 64;
  extern __shared__ char smem[];
  const int Ml = a.Ml, d = a.d, Mr = a.Mr, Wl = a.Wl, Wr = a.Wr;
  const int rp = blk.x % Mr, part = blk.x / Mr;   // output column r', part p
  const int inst = blk.y;
  LzState *st = shift_bytes(a.st, (int64_t)inst * a.wss);
  LzPartials *pp = shift_bytes(a.pp, (int64_t)inst * a.wss);
  double2 *U = shift_bytes(a.U, (int64_t)inst * a.wss);
  double2 *Yp = shift_bytes(a.Yp, (int64_t)inst * a.wss);
  const VE *L = reinterpret_cast<const VE *>(a.L) + (int64_t)inst * a.sL;
  const VE *R = reinterpret_cast<const VE *>(a.R) + (int64_t)inst * a.sR;
  const int j = a.j;
  const int l0 = part * a.nl, nl = min(a.nl, Ml - l0);
  const int ML1 = Ml * d;                  // rows of y
  // this part's shapes (a ragged last part is smaller than the layout's)
  const int MP = nl * d;                   // rows of T1: x rows l0 d .. (l0 + nl) d
  const int K3 = Wl * nl;                  // inner dimension of stage 3
  const int K34 = (K3 + 3) & ~3;
  const HsLayout lay(Ml, d, Mr, Wl, Wr, a.nl, STG, (int)sizeof(T));
  T *base = reinterpret_cast<T *>(smem);
  T *rr_re = base + lay.rr, *rr_im = rr_re + lay.Mr4 * 16;          // stage 1 B [Mr4][16]
  T *t1_re = base + lay.t1, *t1_im = t1_re + lay.T1P;                // [MP][Wr]
  T *t2_re = base + lay.t2, *t2_im = t2_re + lay.K34 * 16;           // [K34][16]
  T *red = base + lay.red;                                           // [HS_WAVES][2][256]
  T *xs_re = base + lay.xs, *xs_im = xs_re + lay.Mr4 * lay.MP16;     // staged x [Mr][MP16]
  T *ls_re = base + lay.ls, *ls_im = ls_re + lay.K34 * lay.Ml16;     // staged L [K34][Ml16]
  double2 *ycol = reinterpret_cast<double2 *>(smem + lay.ycol_b);   // [ML1]
  T *nz_re = reinterpret_cast<T *>(smem + lay.nz_b);                 // staged W table
  T *nz_im = nz_re + HS_NZ;
  int *nz_col = reinterpret_cast<int *>(nz_im + HS_NZ);
  int *nz_row = nz_col + HS_NZ;

  const double2 *x = U + (int64_t)j * a.n + (int64_t)l0 * d;   // u_j, column-major
  const int rows = Wl * d;
  const int *g_row = a.row ? shift_bytes(a.row, (int64_t)inst * a.wss) : nullptr;
  const int *g_col = a.row ? shift_bytes(a.col, (int64_t)inst * a.wss) : nullptr;
  const double2 *g_coef = a.row ? shift_bytes(a.coef, (int64_t)inst * a.wss) : nullptr;
  const int tid = threadIdx.x;
  // One round of global loads: every input of the step is requested before
  // any of them is used (the step state, the close_step partials, the R
  // slice, the W table, the x and L slices of the staged variant and the
  // basis columns of the projections).
  const int stopped = st->stop;
  StepPre pre;
  close_step_load(st, pp, a.Gprev, j, j > 0 ? a.Gw : 0, pre);
  VE rv[HS_RV];
#pragma unroll
  for (int q = 0; q < HS_RV; ++q) {
    const int e = tid + NT * q, k = e >> 4, c = e & 15;
    rv[q].x = 0;
    rv[q].y = 0;
    if (e < lay.Mr4 * 16 && k < Mr && c < Wr) rv[q] = R[((int64_t)rp * Wr + c) * Mr + k];
  }
  const int tcap = min(HS_NZ, rows * d * Wr);
  int nnz = 0, trow = 0, tcol = 0;
  double2 tco = make_double2(0.0, 0.0);
  if (g_row) {
    nnz = g_row[rows];
    if (tid <= rows) trow = g_row[tid];
    if (tid < tcap) {
      tcol = g_col[tid];
      tco = g_coef[tid];
    }
  }
  double2 xv[HS_XV];
  VE lv[HS_LV];
  if (STG) {
#pragma unroll
    for (int q = 0; q < HS_XV; ++q) {
      const int e = tid + NT * q, k = e / lay.MP16, row = e - k * lay.MP16;
      xv[q] = make_double2(0.0, 0.0);
      if (e < lay.Mr4 * lay.MP16 && k < Mr && row < MP) xv[q] = x[(int64_t)k * ML1 + row];
    }
#pragma unroll
    for (int q = 0; q < HS_LV; ++q) {
      const int e = tid + NT * q, row = e / K34, k = e - row * K34;   // k fastest: runs of L
      lv[q].x = 0;
      lv[q].y = 0;
      if (e < K34 * lay.Ml16 && k < K3 && row < Ml) {
        const int wl = k / nl, ll = k - wl * nl;
        lv[q] = L[(int64_t)row * Wl * Ml + wl * Ml + l0 + ll];
      }
    }
  }
  constexpr int NG = NT / 32;              // thread groups of 32 for the projections
  constexpr int NQ = (JB + NG - 1) / NG;
  constexpr int UE = 8;                    // basis elements per (group, q) held in registers
  const int g = tid >> 5, t32 = tid & 31;
  double2 ur[NQ][UE];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = g + NG * q;
    const double2 *ui = U + (int64_t)i * a.n + (int64_t)rp * ML1;
#pragma unroll
    for (int t = 0; t < UE; ++t) {
      const int el = t32 + 32 * t;
      ur[q][t] = (i <= j && el < ML1) ? ui[el] : make_double2(0.0, 0.0);
    }
  }
  // stores to LDS
#pragma unroll
  for (int q = 0; q < HS_RV; ++q) {
    const int e = tid + NT * q;
    if (e < lay.Mr4 * 16) {
      rr_re[e] = rv[q].x;
      rr_im[e] = rv[q].y;
    }
  }
  if (g_row) {
    if (tid <= rows) nz_row[tid] = trow;
    if (tid < tcap) {
      nz_re[tid] = (T)tco.x;
      nz_im[tid] = (T)tco.y;
      nz_col[tid] = tcol;
    }
  }
  if (STG) {
#pragma unroll
    for (int q = 0; q < HS_XV; ++q) {
      const int e = tid + NT * q;
      if (e < lay.Mr4 * lay.MP16) {
        xs_re[e] = (T)xv[q].x;
        xs_im[e] = (T)xv[q].y;
      }
    }
#pragma unroll
    for (int q = 0; q < HS_LV; ++q) {
      const int e = tid + NT * q, row = e / K34, k = e - row * K34;
      if (e < K34 * lay.Ml16) {
        ls_re[k * lay.Ml16 + row] = lv[q].x;
        ls_im[k * lay.Ml16 + row] = lv[q].y;
      }
    }
  }
  for (int e = K3 * 16 + tid; e < K34 * 16; e += NT) {   // zero padding rows of T2
    t2_re[e] = 0;
    t2_im[e] = 0;
  }
  if (stopped) return;
  if (close_step_finish(st, pre, j, j > 0 ? a.Gw : 0, blk.x)) return;   // (synchronises the work-group)

  // stage 1: T1 (MP x Wr) = X[l0 d .., :] (MP x Mr) Rr (Mr x Wr)
  auto st1 = [&](int row, int col, T re, T im) {
    if (col < Wr) {
      t1_re[row * Wr + col] = re;
      t1_im[row * Wr + col] = im;
    }
  };
  if (STG) {
    hs_mm16<T>(MP, Mr, rr_re, rr_im, red,
               [&](int row, int k, T &re, T &im) {
                 re = xs_re[k * lay.MP16 + row];
                 im = xs_im[k * lay.MP16 + row];
               }, st1);
  } else {
    hs_mm16<T>(MP, Mr, rr_re, rr_im, red,
               [&](int row, int k, T &re, T &im) {
                 const double2 v = x[(int64_t)k * ML1 + row];
                 re = (T)v.x;
                 im = (T)v.y;
               }, st1);
  }
  // stage 2: T2[(wl, ll)][s'] for s' < d (padding columns only feed
  // discarded outputs); hs_mm16 ended with a barrier
  if (!g_row) {                            // bond operator: T2[(w, ll)][0] = T1[ll][w]
    for (int k = threadIdx.x; k < K3; k += NT) {
      const int w = k / nl, ll = k - w * nl;
      t2_re[k * 16] = t1_re[ll * Wr + w];
      t2_im[k * 16] = t1_im[ll * Wr + w];
    }
  } else if (nnz <= HS_NZ) {
    hs_stage2<T, false>(t2_re, t2_im, t1_re, t1_im, K3, nl, d, d * Wr, (const int *)nz_row,
                        (const int *)nz_col, nz_re, nz_im, nullptr);
  } else {
    hs_stage2<T, true>(t2_re, t2_im, t1_re, t1_im, K3, nl, d, d * Wr, g_row, g_col, nullptr,
                       nullptr, g_coef);
  }
  __syncthreads();
  // stage 3: y_p (Ml x d) = L[:, :, l0 ..] (Ml x K3) T2 (K3 x d)
  auto st3 = [&](int row, int col, T re, T im) {
    if (col < d) ycol[row * d + col] = make_double2((double)re, (double)im);
  };
  if (STG) {
    hs_mm16<T>(Ml, K3, t2_re, t2_im, red,
               [&](int row, int k, T &re, T &im) {
                 re = ls_re[k * lay.Ml16 + row];
                 im = ls_im[k * lay.Ml16 + row];
               }, st3);
  } else {
    const int64_t lrow = (int64_t)Wl * Ml;
    hs_mm16<T>(Ml, K3, t2_re, t2_im, red,
               [&](int row, int k, T &re, T &im) {
                 const int wl = k / nl, ll = k - wl * nl;
                 const VE v = L[(int64_t)row * lrow + wl * Ml + l0 + ll];
                 re = v.x;
                 im = v.y;
               }, st3);
  }
  // y_p -> Yp[p] (column r'); <u_i, y_p> partials: group g takes i = g, g + NG, ...
  double2 *wdst = Yp + (int64_t)part * a.n + (int64_t)rp * ML1;
  for (int e = threadIdx.x; e < ML1; e += NT) wdst[e] = ycol[e];
  const int slot = blk.x;
  double dr[NQ], di[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    dr[q] = 0.0;
    di[q] = 0.0;
    const int i = g + NG * q;
    if (i <= j) {
#pragma unroll
      for (int t = 0; t < UE; ++t) {
        const int el = t32 + 32 * t;
        if (el < ML1) {
          const double2 u = ur[q][t];
          const double2 y = ycol[el];
          dr[q] += u.x * y.x + u.y * y.y;
          di[q] += u.x * y.y - u.y * y.x;
        }
      }
      const double2 *ui = U + (int64_t)i * a.n + (int64_t)rp * ML1;
#pragma unroll 8
      for (int el = t32 + 32 * UE; el < ML1; el += 32) {
        const double2 u = ui[el];
        const double2 y = ycol[el];
        dr[q] += u.x * y.x + u.y * y.y;
        di[q] += u.x * y.y - u.y * y.x;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      dr[q] += __shfl_xor(dr[q], o, 32);
      di[q] += __shfl_xor(di[q], o, 32);
    }
    const int i = g + NG * q;
    if (t32 == 0 && i <= j) pp->dot[i][slot] = make_double2(dr[q], di[q]);
  }
}

template <typename T, int JB, bool STG>
__global__ __launch_bounds__(HS_WAVES * 64) void heff_small_kernel(HeffSmallArgs a) {
  heff_small_body<T, JB, STG>(a, native_block());
}
template <typename T, int JB, bool STG>
__global__ __launch_bounds__(HS_WAVES * 64) void heff_small_grouped_kernel(Grp<HeffSmallArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  heff_small_body<T, JB, STG>(g.a[k], b);
}

// CSR table of an MPO site tensor W[wl][s'][s][wr] over rows (wl, s'): one
// work-group per instance.  Every thread loads its candidates (index
// e = t + 1024 q) at once; a work-group scan over the nonzero flags, chunk
// by chunk in index order, gives each nonzero its position.
constexpr int WT_THREADS = 1024;
__device__ __forceinline__ void wtable_body(const double2 *W, int rows, int cap, int64_t sW, int *rowp,
                                            int *col, double2 *coef, int64_t wss, const BlockXYZ &blk) {
  constexpr int QN = WT_MAX / WT_THREADS;
  const int inst = blk.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  W += (int64_t)inst * sW;
  rowp = shift_bytes(rowp, (int64_t)inst * wss);
  col = shift_bytes(col, (int64_t)inst * wss);
  coef = shift_bytes(coef, (int64_t)inst * wss);
  const int total = rows * cap;
  double2 v[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int e = t + WT_THREADS * q;
    v[q] = e < total ? W[e] : make_double2(0.0, 0.0);
  }
  __shared__ int wcount[WT_THREADS / 64];
  __shared__ int base_s;
  if (t == 0) base_s = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int e = t + WT_THREADS * q;
    if (WT_THREADS * q >= total) break;
    const bool nz = e < total && (v[q].x != 0.0 || v[q].y != 0.0);
    const unsigned long long m = __ballot(nz);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wave] = __popcll(m);
    __syncthreads();
    int off = base_s;
    for (int w = 0; w < wave; ++w) off += wcount[w];
    const int pos = off + below;
    if (nz) {
      col[pos] = e % cap;
      coef[pos] = v[q];
    }
    // rowp[r] = nonzeros before index r cap
    if (e < total && e % cap == 0) rowp[e / cap] = pos;
    __syncthreads();
    if (t == 0) {
      int s = base_s;
      for (int w = 0; w < WT_THREADS / 64; ++w) s += wcount[w];
      base_s = s;
    }
    __syncthreads();
  }
  if (t == 0) rowp[rows] = base_s;
}

__global__ __launch_bounds__(WT_THREADS) void wtable_kernel(const double2 *W, int rows, int cap,
                                                            int64_t sW, int *rowp, int *col,
                                                            double2 *coef, int64_t wss) {
  wtable_body(W, rows, cap, sW, rowp, col, coef, wss, native_block());
}
__global__ __launch_bounds__(WT_THREADS) void wtable_grouped_kernel(Grp<WtableArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  const WtableArgs &a = g.a[k];
  wtable_body(a.W, a.rows, a.cap, a.sW, a.rowp, a.col, a.coef, a.wss, b);
}

// Work-groups of lz_dots per instance: the grid of lz_update (every lz_update
// work-group adds all of lz_dots' partials, so a batch, which takes fewer
// work-groups per instance, also writes fewer of them).
int dots_grid(int64_t n, int count) { return upd_grid(n, count); }

}  // namespace

hipError_t lz_start(LzState *st, LzPartials *pp, const double2 *x, double2 *u0, int64_t n,
                    double zr, double zi, double tol, int keff, int trows, int *nonfinite,
                    const LzInst &in, hipStream_t s) {
  hipLaunchKernelGGL(lz_start_kernel, dim3(upd_grid(n, in.count), in.count), dim3(LZ_BLOCK), 0, s, st, pp, x,
                     u0, n, zr, zi, tol, keff, trows, nonfinite, in);
  return hipGetLastError();
}

hipError_t lz_dots(LzState *st, LzPartials *pp, DType ty, const void *ypart, int P, int64_t pstride,
                   double2 *U, int64_t ldu, int j, int64_t n, const LzInst &in, hipStream_t s) {
  const dim3 g(dots_grid(n, in.count), in.count), b(LZ_BLOCK);
#define LZ_DOTS(T, JB)                                                                         \
  hipLaunchKernelGGL((lz_dots_kernel<T, JB>), g, b, 0, s, st, pp, (const T *)ypart, P, pstride, \
                     U, ldu, j, n, in)
  if (ty == F64) {
    if (j < 4) LZ_DOTS(double2, 4);
    else if (j < 8) LZ_DOTS(double2, 8);
    else if (j < 16) LZ_DOTS(double2, 16);
    else if (j < 24) LZ_DOTS(double2, 24);
    else LZ_DOTS(double2, 32);
  } else {
    if (j < 4) LZ_DOTS(float2, 4);
    else if (j < 8) LZ_DOTS(float2, 8);
    else if (j < 16) LZ_DOTS(float2, 16);
    else if (j < 24) LZ_DOTS(float2, 24);
    else LZ_DOTS(float2, 32);
  }
#undef LZ_DOTS
  return hipGetLastError();
}

hipError_t lz_update(LzState *st, LzPartials *pp, double2 *U, int64_t ldu, int j, int64_t n, int Gd,
                     const double2 *Yp, int P, const LzInst &in, hipStream_t s, int close) {
  const dim3 g(upd_grid(n, in.count), in.count), b(LZ_BLOCK);
  if (Gd == 0) Gd = dots_grid(n, in.count);
  if (Yp && (P < 1 || P > HS_PMAX)) return hipErrorInvalidValue;
#define LZ_UPD(JB) \
  hipLaunchKernelGGL((lz_update_kernel<JB>), g, b, 0, s, st, pp, U, ldu, j, n, Gd, Yp, P, in, close)
  if (j < 4) LZ_UPD(4);
  else if (j < 8) LZ_UPD(8);
  else if (j < 16) LZ_UPD(16);
  else if (j < 24) LZ_UPD(24);
  else LZ_UPD(32);
#undef LZ_UPD
  return hipGetLastError();
}

int lz_grid(int64_t n, int count) { return upd_grid(n, count); }

size_t heff_small_lds(const HeffSmallArgs &a, int tm_bytes) {
  return HsLayout(a.Ml, a.d, a.Mr, a.Wl, a.Wr, a.nl, a.staged != 0, tm_bytes).total_b;
}

bool heff_small_fits(const HeffSmallArgs &a, int tm_bytes) {
  if (a.staged) {
    const HsLayout l(a.Ml, a.d, a.Mr, a.Wl, a.Wr, a.nl, true, tm_bytes);
    if (l.Mr4 * l.MP16 > HS_XV * HS_WAVES * 64 || l.K34 * l.Ml16 > HS_LV * HS_WAVES * 64)
      return false;
  }
  return a.Mr >= 1 && a.Mr <= 128 && a.Ml >= 1 && a.Wr <= 16 && a.d <= 16 && a.Wl * a.d <= 256 &&
         (int64_t)a.Wl * a.d * a.d * a.Wr <= WT_MAX && a.nl >= 1 && a.P >= 1 &&
         a.P <= HS_PMAX && (int64_t)a.P * a.nl >= a.Ml && (int64_t)(a.P - 1) * a.nl < a.Ml &&
         (int64_t)a.P * a.Mr <= LZ_PARTS && heff_small_lds(a, tm_bytes) <= HEFF_SMALL_LDS;
}

hipError_t heff_small(DType t, const HeffSmallArgs &a, int count, hipStream_t s) {
  static const bool attr = [] {   // once per process (thread-safe static)
#define HS_ATTR(T, JB, S)                                                               \
  (void)hipFuncSetAttribute((const void *)heff_small_kernel<T, JB, S>,                  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, HEFF_SMALL_LDS)
#define HS_ATTR2(T, S) HS_ATTR(T, 4, S); HS_ATTR(T, 8, S); HS_ATTR(T, 16, S); HS_ATTR(T, 32, S)
    HS_ATTR2(double, false); HS_ATTR2(double, true); HS_ATTR2(float, false); HS_ATTR2(float, true);
#undef HS_ATTR2
#undef HS_ATTR
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  const dim3 g(a.Mr * a.P, count), b(HS_WAVES * 64);
  const size_t lds = heff_small_lds(a, t == F64 ? 8 : 4);
#define HS(T, JB, S) hipLaunchKernelGGL((heff_small_kernel<T, JB, S>), g, b, lds, s, a)
#define HS_J(T, S)                 \
  do {                             \
    if (a.j < 4) HS(T, 4, S);      \
    else if (a.j < 8) HS(T, 8, S); \
    else if (a.j < 16) HS(T, 16, S); \
    else HS(T, 32, S);             \
  } while (0)
  if (t == F64) {
    if (a.staged) HS_J(double, true);
    else HS_J(double, false);
  } else {
    if (a.staged) HS_J(float, true);
    else HS_J(float, false);
  }
#undef HS_J
#undef HS
  return hipGetLastError();
}

hipError_t wtable(const double2 *W, int Wl, int d, int Wr, int64_t sW, int *rowp, int *col,
                  double2 *coef, int64_t wss, int count, hipStream_t s) {
  if (Wl * d > 256 || (int64_t)Wl * d * d * Wr > WT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wtable_kernel, dim3(count), dim3(WT_THREADS), 0, s, W, Wl * d, d * Wr, sW,
                     rowp, col, coef, wss);
  return hipGetLastError();
}

hipError_t lz_start_grouped(const LzStartArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<LzStartArgs> g;
  for (int k = 0; k < ng; ++k) g.add(a[k], upd_grid(a[k].n, a[k].in.count), a[k].in.count, 1);
  if (g.ng == 0) return hipSuccess;
  hipLaunchKernelGGL(lz_start_grouped_kernel, dim3(g.blocks()), dim3(LZ_BLOCK), 0, s, g);
  return hipGetLastError();
}

hipError_t lz_dots_grouped(DType ty, const LzDotsArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<LzDotsArgs> g;
  for (int k = 0; k < ng; ++k) {
    if (a[k].j != a[0].j) return hipErrorInvalidValue;
    g.add(a[k], dots_grid(a[k].n, a[k].in.count), a[k].in.count, 1);
  }
  if (g.ng == 0) return hipSuccess;
  const int j = a[0].j;
  const dim3 gr(g.blocks()), b(LZ_BLOCK);
#define LZ_DOTS_G(T, JB) hipLaunchKernelGGL((lz_dots_grouped_kernel<T, JB>), gr, b, 0, s, g)
  if (ty == F64) {
    if (j < 4) LZ_DOTS_G(double2, 4);
    else if (j < 8) LZ_DOTS_G(double2, 8);
    else if (j < 16) LZ_DOTS_G(double2, 16);
    else if (j < 24) LZ_DOTS_G(double2, 24);
    else LZ_DOTS_G(double2, 32);
  } else {
    if (j < 4) LZ_DOTS_G(float2, 4);
    else if (j < 8) LZ_DOTS_G(float2, 8);
    else if (j < 16) LZ_DOTS_G(float2, 16);
    else if (j < 24) LZ_DOTS_G(float2, 24);
    else LZ_DOTS_G(float2, 32);
  }
#undef LZ_DOTS_G
  return hipGetLastError();
}

hipError_t lz_update_grouped(const LzUpdateArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<LzUpdateArgs> g;
  for (int k = 0; k < ng; ++k) {
    LzUpdateArgs ak = a[k];
    if (ak.j != a[0].j) return hipErrorInvalidValue;
    if (ak.Gd == 0) ak.Gd = dots_grid(ak.n, ak.in.count);
    if (ak.Yp && (ak.P < 1 || ak.P > HS_PMAX)) return hipErrorInvalidValue;
    g.add(ak, upd_grid(ak.n, ak.in.count), ak.in.count, 1);
  }
  if (g.ng == 0) return hipSuccess;
  const int j = a[0].j;
  const dim3 gr(g.blocks()), b(LZ_BLOCK);
#define LZ_UPD_G(JB) hipLaunchKernelGGL((lz_update_grouped_kernel<JB>), gr, b, 0, s, g)
  if (j < 4) LZ_UPD_G(4);
  else if (j < 8) LZ_UPD_G(8);
  else if (j < 16) LZ_UPD_G(16);
  else if (j < 24) LZ_UPD_G(24);
  else LZ_UPD_G(32);
#undef LZ_UPD_G
  return hipGetLastError();
}

hipError_t lz_finish_grouped(const LzFinishArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<LzFinishArgs> g;
  int kb = 0;
  for (int k = 0; k < ng; ++k) {
    if (a[k].keff > KMAX) return hipErrorInvalidValue;
    kb = std::max(kb, a[k].keff);
    g.add(a[k], upd_grid(a[k].n, a[k].in.count), a[k].in.count, 1);
  }
  if (g.ng == 0) return hipSuccess;
  const dim3 gr(g.blocks()), b(LZ_BLOCK);
#define LZ_FIN_G(KB) hipLaunchKernelGGL((lz_finish_grouped_kernel<KB>), gr, b, 0, s, g)
  if (kb <= 4) LZ_FIN_G(4);
  else if (kb <= 8) LZ_FIN_G(8);
  else if (kb <= 16) LZ_FIN_G(16);
  else LZ_FIN_G(32);
#undef LZ_FIN_G
  return hipGetLastError();
}

hipError_t heff_small_grouped(DType t, const HeffSmallArgs *a, const int *count, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  static const bool attr = [] {   // once per process (thread-safe static)
#define HSG_ATTR(T, JB, S)                                                              \
  (void)hipFuncSetAttribute((const void *)heff_small_grouped_kernel<T, JB, S>,          \
                            hipFuncAttributeMaxDynamicSharedMemorySize, HEFF_SMALL_LDS)
#define HSG_ATTR2(T, S) HSG_ATTR(T, 4, S); HSG_ATTR(T, 8, S); HSG_ATTR(T, 16, S); HSG_ATTR(T, 32, S)
    HSG_ATTR2(double, false); HSG_ATTR2(double, true); HSG_ATTR2(float, false); HSG_ATTR2(float, true);
#undef HSG_ATTR2
#undef HSG_ATTR
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  Grp<HeffSmallArgs> g;
  size_t lds = 0;
  const int tb = t == F64 ? 8 : 4;
  for (int k = 0; k < ng; ++k) {
    if (a[k].j != a[0].j || a[k].staged != a[0].staged) return hipErrorInvalidValue;
    lds = std::max(lds, heff_small_lds(a[k], tb));
    g.add(a[k], a[k].Mr * a[k].P, count[k], 1);
  }
  if (g.ng == 0) return hipSuccess;
  if (lds > HEFF_SMALL_LDS) return hipErrorInvalidValue;
  const dim3 gr(g.blocks()), b(HS_WAVES * 64);
  const int j = a[0].j;
#define HSG(T, JB, S) hipLaunchKernelGGL((heff_small_grouped_kernel<T, JB, S>), gr, b, lds, s, g)
#define HSG_J(T, S)                  \
  do {                               \
    if (j < 4) HSG(T, 4, S);         \
    else if (j < 8) HSG(T, 8, S);    \
    else if (j < 16) HSG(T, 16, S);  \
    else HSG(T, 32, S);              \
  } while (0)
  if (t == F64) {
    if (a[0].staged) HSG_J(double, true);
    else HSG_J(double, false);
  } else {
    if (a[0].staged) HSG_J(float, true);
    else HSG_J(float, false);
  }
#undef HSG_J
#undef HSG
  return hipGetLastError();
}

hipError_t wtable_grouped(const WtableArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<WtableArgs> g;
  for (int k = 0; k < ng; ++k) {
    if (a[k].rows > 256 || (int64_t)a[k].rows * a[k].cap > WT_MAX) return hipErrorInvalidValue;
    g.add(a[k], a[k].count, 1, 1);
  }
  if (g.ng == 0) return hipSuccess;
  hipLaunchKernelGGL(wtable_grouped_kernel, dim3(g.blocks()), dim3(WT_THREADS), 0, s, g);
  return hipGetLastError();
}

hipError_t lz_finish(LzState *st, const double2 *U, int64_t ldu, int64_t n, int keff, double2 *y,
                     int32_t *k_used, int trows, const LzInst &in, hipStream_t s) {
  if (keff > KMAX) return hipErrorInvalidValue;
  const dim3 g(upd_grid(n, in.count), in.count), b(LZ_BLOCK);
#define LZ_FIN(KB) \
  hipLaunchKernelGGL((lz_finish_kernel<KB>), g, b, 0, s, st, U, ldu, n, keff, y, k_used, trows, in)
  if (keff <= 4) LZ_FIN(4);
  else if (keff <= 8) LZ_FIN(8);
  else if (keff <= 16) LZ_FIN(16);
  else LZ_FIN(32);
#undef LZ_FIN
  return hipGetLastError();
}

}  // namespace tdvp
