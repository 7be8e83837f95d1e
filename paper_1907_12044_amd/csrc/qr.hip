// FP64 Householder QR of a tall complex matrix for the gauge shifts of the
// PS sweep (eq:QR; the right-to-left sweep uses the QR of C^H, i.e. an RQ).
//
// One work-group of 16 wave64 factors the matrix held column-major in LDS
// when it fits (m n <= QR_LDS_ELEMS): for column j the reflector
// H_j = I - tau v v^H with v = x - alpha e_1 and alpha = -exp(i arg x_0) |x|
// (no cancellation in v_0) is built from the sub-diagonal norm and applied
// to the trailing columns, 32 columns at a time with 32 threads per column
// (partial dots reduced through LDS).  R is written out, then the thin Q is
// formed in the same storage by applying the reflectors backwards to
// [I; 0] (column j is replaced by H_j e_j once it is no longer needed), and
// the phases of alpha_j are moved into Q so that diag(R) is real and
// non-negative.  Inputs and outputs go through element strides with
// optional conjugation, so the same kernel serves C = L D (left-to-right)
// and C^H = Q R, C = R^H Q^H (right-to-left).  The matrix never leaves the
// device.
#include "common.h"

namespace tdvp {

namespace {

constexpr int QR_THREADS = 1024;
constexpr int QR_LDS_ELEMS = 8704;          // 136 KiB of complex doubles (+ 23 KiB static)

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fallback for matrices that fit neither one work-group's LDS nor the
// panel path (m > 2560): the same steps on the matrix in the workspace.
__global__ __launch_bounds__(QR_THREADS) void qr_kernel(QrArgs p) {
  {   // instance blockIdx.x
    const int64_t r = blockIdx.x;
    p.A += r * p.inst.a;
    p.Q += r * p.inst.b;
    p.R += r * p.inst.c;
    p.work += r * p.inst.skip;
  }
  const int m = p.m, n = p.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = QR_THREADS / 64;
  double2 *Aw = p.work;     // m x n column-major
  __shared__ double red[NW];
  __shared__ double tau_s[256];
  __shared__ double2 alpha_s[256];
  __shared__ double tail_s;     // sum |A[r][j]|^2 over r > j for the next column

  for (int64_t e = tid; e < (int64_t)m * n; e += QR_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    double2 v = p.A[(int64_t)r * p.a_rs + (int64_t)c * p.a_cs];
    if (p.conjA) v.y = -v.y;
    Aw[e] = v;
  }
  __syncthreads();

  {
    double s = 0.0;
    for (int r = 1 + tid; r < m; r += QR_THREADS) s += Aw[r].x * Aw[r].x + Aw[r].y * Aw[r].y;
    s = wsum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += red[w];
      tail_s = t;
    }
    __syncthreads();
  }

  for (int j = 0; j < n; ++j) {
    double2 *col = Aw + (int64_t)j * m;
    if (tid == 0) {
      const double tail = tail_s;
      const double2 x0 = col[j];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nx = sqrt(tail + ax0 * ax0);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
      const double2 v0 = make_double2(x0.x - al.x, x0.y - al.y);
      const double vn2 = tail + (v0.x * v0.x + v0.y * v0.y);
      tau_s[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      alpha_s[j] = al;
      col[j] = v0;
    }
    __syncthreads();
    const double tau = tau_s[j];
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += NW) {
        double2 *cc = Aw + (int64_t)c * m;
        double dr = 0.0, di = 0.0;   // tau v^H a_c
        for (int r = j + lane; r < m; r += 64) {
          const double2 v = col[r], a = cc[r];
          dr += v.x * a.x + v.y * a.y;
          di += v.x * a.y - v.y * a.x;
        }
        dr = wsum(dr) * tau;
        di = wsum(di) * tau;
        double s2 = 0.0;     // norm below the diagonal of column j+1, for step j+1
        for (int r = j + lane; r < m; r += 64) {
          const double2 v = col[r];
          double2 a = cc[r];
          a.x -= v.x * dr - v.y * di;
          a.y -= v.x * di + v.y * dr;
          cc[r] = a;
          if (r > j + 1) s2 += a.x * a.x + a.y * a.y;
        }
        if (c == j + 1) {
          s2 = wsum(s2);
          if (lane == 0) tail_s = s2;
        }
      }
    } else if (j + 1 < n && wave == 0) {
      const double2 *cc = Aw + (int64_t)(j + 1) * m;
      double s2 = 0.0;
      for (int r = j + 2 + lane; r < m; r += 64) s2 += cc[r].x * cc[r].x + cc[r].y * cc[r].y;
      s2 = wsum(s2);
      if (lane == 0) tail_s = s2;
    }
    __syncthreads();
  }

  // R (rows scaled by conj(phase_r) so the diagonal is |alpha_r|)
  for (int64_t e = tid; e < (int64_t)n * n; e += QR_THREADS) {
    const int r = (int)(e % n), c = (int)(e / n);
    double2 o = make_double2(0.0, 0.0);
    const double2 al = alpha_s[r];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    if (r == c) {
      o = make_double2(aa, 0.0);
    } else if (c > r) {
      const double2 ph = aa > 0.0 ? make_double2(al.x / aa, -al.y / aa) : make_double2(1.0, 0.0);
      const double2 a = Aw[(int64_t)c * m + r];
      o = make_double2(a.x * ph.x - a.y * ph.y, a.x * ph.y + a.y * ph.x);
    }
    if (p.conjR) o.y = -o.y;
    p.R[(int64_t)r * p.r_rs + (int64_t)c * p.r_cs] = o;
  }
  __syncthreads();

  // thin Q in place: after step j, columns j..n-1 hold H_j ... H_{n-1} [I; 0]
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    double2 *v = Aw + (int64_t)j * m;    // v_j in rows j..m-1
    // row j of the accumulated columns c > j is zero (it held R[j][c])
    for (int c = j + 1 + tid; c < n; c += QR_THREADS) Aw[(int64_t)c * m + j] = make_double2(0.0, 0.0);
    __syncthreads();
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += NW) {
        double2 *qc = Aw + (int64_t)c * m;
        double dr = 0.0, di = 0.0;
        for (int r = j + lane; r < m; r += 64) {
          const double2 vv = v[r], a = qc[r];
          dr += vv.x * a.x + vv.y * a.y;
          di += vv.x * a.y - vv.y * a.x;
        }
        dr = wsum(dr) * tau;
        di = wsum(di) * tau;
        for (int r = j + lane; r < m; r += 64) {
          const double2 vv = v[r];
          double2 a = qc[r];
          a.x -= vv.x * dr - vv.y * di;
          a.y -= vv.x * di + vv.y * dr;
          qc[r] = a;
        }
      }
    }
    __syncthreads();
    // column j <- H_j e_j = e_j - tau v conj(v_j)
    const double2 v0 = v[j];
    __syncthreads();
    for (int r = tid; r < m; r += QR_THREADS) {
      double2 o;
      if (r < j) {
        o = make_double2(0.0, 0.0);
      } else {
        const double2 vv = v[r];
        // tau * vv * conj(v0)
        o = make_double2(-tau * (vv.x * v0.x + vv.y * v0.y), -tau * (vv.y * v0.x - vv.x * v0.y));
        if (r == j) o.x += 1.0;
      }
      v[r] = o;
    }
    __syncthreads();
  }

  for (int64_t e = tid; e < (int64_t)m * n; e += QR_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    const double2 al = alpha_s[c];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
    const double2 q = Aw[e];
    double2 o = make_double2(q.x * ph.x - q.y * ph.y, q.x * ph.y + q.y * ph.x);
    if (p.conjQ) o.y = -o.y;
    p.Q[(int64_t)r * p.q_rs + (int64_t)c * p.q_cs] = o;
  }
}

// ---------------------------------------------------------------------------
// Register path for n <= 32 columns and m <= 32 RQ rows (m <= 256 with RQ = 8):
// the shapes of the sweep's gauge shifts at small bond dimension.  Column c
// lives in the registers of half-wave c (thread c * 32 + g holds rows
// g + 32 q), so the trailing update of a step needs no LDS traffic for the
// matrix: the reflector v_j goes to LDS once (column j of V, kept for the
// formation of Q), and each column reduces its dot with v_j inside its
// half-wave (DPP / swizzle butterflies, identical result in every lane).
// One barrier per step.  Q is then formed column by column without
// barriers (column c needs H_c .. H_0 only).  Same reflectors, R and Q
// phases as the other paths.
constexpr int QRR_ELEMS = 8192;          // V in LDS: at most 256 x 32, 128 KiB

template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swz_xor16(double v) {   // lane ^ 16 within 32 lanes
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return __hiloint2double(hi, lo);
}
// Sum over the 32 lanes of a half-wave; every lane gets the same bits
// (each level adds a lane and its partner, and addition commutes).
__device__ __forceinline__ double hw_sum(double v) {
  v += dpp_d<0xB1>(v);     // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);     // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);    // row_half_mirror
  v += dpp_d<0x140>(v);    // row_mirror
  v += swz_xor16(v);
  return v;
}
// value of v in lane l of this half-wave (l uniform)
__device__ __forceinline__ double hw_lane(double v, int l) {
  const int base = threadIdx.x & 32;
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), base + l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), base + l);
  return __hiloint2double(hi, lo);
}

template <int RQ>
__global__ __launch_bounds__(QR_THREADS) void qr_reg_kernel(QrArgs p) {
  extern __shared__ double2 V[];         // m x n column-major: reflector j in column j
  {
    const int64_t r = blockIdx.x;
    p.A += r * p.inst.a;
    p.Q += r * p.inst.b;
    p.R += r * p.inst.c;
  }
  const int m = p.m, n = p.n;
  const int c = threadIdx.x >> 5, g = threadIdx.x & 31;
  __shared__ double tau_s[32];
  __shared__ double2 alpha_s[32];
  double2 a[RQ];
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const int r = g + 32 * q;
    a[q] = make_double2(0.0, 0.0);
    if (c < n && r < m) {
      a[q] = p.A[(int64_t)r * p.a_rs + (int64_t)c * p.a_cs];
      if (p.conjA) a[q].y = -a[q].y;
    }
  }
  for (int j = 0; j < n; ++j) {
    if (c == j) {
      // reflector of column j from its sub-diagonal norm and head x0
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = g + 32 * q;
        if (r > j && r < m) t += a[q].x * a[q].x + a[q].y * a[q].y;
      }
      const double tail = hw_sum(t);
      const int gj = j & 31, qj = j >> 5;
      double2 x0 = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < RQ; ++q)
        if (q == qj) x0 = make_double2(hw_lane(a[q].x, gj), hw_lane(a[q].y, gj));
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nx = sqrt(tail + ax0 * ax0);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
      const double2 v0 = make_double2(x0.x - al.x, x0.y - al.y);
      const double vn2 = tail + (v0.x * v0.x + v0.y * v0.y);
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = g + 32 * q;
        if (r == j) a[q] = v0;
        if (r >= j && r < m) V[(int64_t)j * m + r] = a[q];
      }
      if (g == 0) {
        tau_s[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        alpha_s[j] = al;
      }
    }
    __syncthreads();
    if (c > j && c < n) {
      const double tau = tau_s[j];
      if (tau != 0.0) {
        const double2 *v = V + (int64_t)j * m;
        double2 vr[RQ];
        double dr = 0.0, di = 0.0;     // v^H a_c
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
          const int r = g + 32 * q;
          vr[q] = (r >= j && r < m) ? v[r] : make_double2(0.0, 0.0);
          dr += vr[q].x * a[q].x + vr[q].y * a[q].y;
          di += vr[q].x * a[q].y - vr[q].y * a[q].x;
        }
        const double sr = hw_sum(dr) * tau, si = hw_sum(di) * tau;
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
          a[q].x -= vr[q].x * sr - vr[q].y * si;
          a[q].y -= vr[q].x * si + vr[q].y * sr;
        }
      }
    }
  }
  __syncthreads();
  // R: column c holds R[r][c] in rows r < c; diagonal |alpha_c|; rows scaled by conj(phase_r)
  if (c < n) {
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int r = g + 32 * q;
      if (r < n) {
        double2 o = make_double2(0.0, 0.0);
        const double2 al = alpha_s[r];
        const double aa = sqrt(al.x * al.x + al.y * al.y);
        if (r == c) {
          o = make_double2(aa, 0.0);
        } else if (r < c) {
          const double2 ph = aa > 0.0 ? make_double2(al.x / aa, -al.y / aa) : make_double2(1.0, 0.0);
          o = make_double2(a[q].x * ph.x - a[q].y * ph.y, a[q].x * ph.y + a[q].y * ph.x);
        }
        if (p.conjR) o.y = -o.y;
        p.R[(int64_t)r * p.r_rs + (int64_t)c * p.r_cs] = o;
      }
    }
  }
  // thin Q: column c = H_0 ... H_c e_c (H_j e_c = e_c for j > c)
  if (c < n) {
#pragma unroll
    for (int q = 0; q < RQ; ++q) a[q] = make_double2(g + 32 * q == c ? 1.0 : 0.0, 0.0);
    for (int j = c; j >= 0; --j) {
      const double tau = tau_s[j];
      if (tau == 0.0) continue;
      const double2 *v = V + (int64_t)j * m;
      double2 vr[RQ];
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = g + 32 * q;
        vr[q] = (r >= j && r < m) ? v[r] : make_double2(0.0, 0.0);
        dr += vr[q].x * a[q].x + vr[q].y * a[q].y;
        di += vr[q].x * a[q].y - vr[q].y * a[q].x;
      }
      const double sr = hw_sum(dr) * tau, si = hw_sum(di) * tau;
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        a[q].x -= vr[q].x * sr - vr[q].y * si;
        a[q].y -= vr[q].x * si + vr[q].y * sr;
      }
    }
    const double2 al = alpha_s[c];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int r = g + 32 * q;
      if (r < m) {
        double2 o = make_double2(a[q].x * ph.x - a[q].y * ph.y, a[q].x * ph.y + a[q].y * ph.x);
        if (p.conjQ) o.y = -o.y;
        p.Q[(int64_t)r * p.q_rs + (int64_t)c * p.q_cs] = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// LDS path, tuned for the tall-skinny shapes of the sweep (m n <= 9216).
// Same arithmetic as qr_kernel (same reflectors, same R and Q), but the
// trailing-column work of a step is spread over the whole work-group:
// thread (c, g), c = tid / 32 and g = tid % 32, takes rows j + g + 32 q of
// trailing column c of a batch of 32 columns.  Its partial dot goes to LDS;
// after one barrier every thread adds the 32 partials of its column in
// order (LDS broadcast reads), so a step needs three barriers and no wave
// reductions.  The sub-diagonal norm of the next column comes from the
// same pass.
constexpr int QB_COLS = 32;              // columns per batch (threads / 32)

__global__ __launch_bounds__(QR_THREADS) void qr_lds_kernel(QrArgs p) {
  extern __shared__ double2 Aw[];        // m x n column-major
  {
    const int64_t r = blockIdx.x;
    p.A += r * p.inst.a;
    p.Q += r * p.inst.b;
    p.R += r * p.inst.c;
  }
  const int m = p.m, n = p.n;
  const int tid = threadIdx.x;
  const int cl = tid >> 5, g = tid & 31;
  __shared__ double2 part[QB_COLS][33];  // partial dots, padded rows
  __shared__ double tpart[32];           // partial sub-diagonal norms of the next column
  __shared__ double tau_s[256];
  __shared__ double2 alpha_s[256];

  // load (all loads of a thread issued together)
  constexpr int QN = (QR_LDS_ELEMS + QR_THREADS - 1) / QR_THREADS;
  {
    double2 v[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int e = tid + QR_THREADS * q;
      if (e < m * n) {
        const int r = e % m, c = e / m;
        v[q] = p.A[(int64_t)r * p.a_rs + (int64_t)c * p.a_cs];
      }
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int e = tid + QR_THREADS * q;
      if (e < m * n) {
        if (p.conjA) v[q].y = -v[q].y;
        Aw[e] = v[q];
      }
    }
  }
  __syncthreads();
  // sub-diagonal norm of column 0
  if (cl == 0) {
    double s = 0.0;
    for (int r = 1 + g; r < m; r += 32) s += Aw[r].x * Aw[r].x + Aw[r].y * Aw[r].y;
    tpart[g] = s;
  }
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    double2 *col = Aw + (int64_t)j * m;
    if (tid == 0) {
      double tail = 0.0;
      for (int t = 0; t < 32; ++t) tail += tpart[t];
      const double2 x0 = col[j];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nx = sqrt(tail + ax0 * ax0);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
      const double2 v0 = make_double2(x0.x - al.x, x0.y - al.y);
      const double vn2 = tail + (v0.x * v0.x + v0.y * v0.y);
      tau_s[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      alpha_s[j] = al;
      col[j] = v0;
    }
    __syncthreads();
    const double tau = tau_s[j];
    for (int cb = j + 1; cb < n; cb += QB_COLS) {
      const int c = cb + cl;
      double2 *cc = Aw + (int64_t)c * m;
      double dr = 0.0, di = 0.0;   // v^H a_c over this thread's rows
      if (c < n && tau != 0.0) {
        for (int r = j + g; r < m; r += 32) {
          const double2 v = col[r], a = cc[r];
          dr += v.x * a.x + v.y * a.y;
          di += v.x * a.y - v.y * a.x;
        }
      }
      part[cl][g] = make_double2(dr, di);
      __syncthreads();
      double ts = 0.0;
      if (c < n) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < 32; ++t) {
          const double2 pv = part[cl][t];
          sr += pv.x;
          si += pv.y;
        }
        sr *= tau;
        si *= tau;
        for (int r = j + g; r < m; r += 32) {
          double2 a = cc[r];
          if (tau != 0.0) {
            const double2 v = col[r];
            a.x -= v.x * sr - v.y * si;
            a.y -= v.x * si + v.y * sr;
            cc[r] = a;
          }
          if (r > j + 1) ts += a.x * a.x + a.y * a.y;
        }
      }
      if (c == j + 1) tpart[g] = ts;
      __syncthreads();
    }
  }

  // R (rows scaled by conj(phase_r) so the diagonal is |alpha_r|)
  for (int e = tid; e < n * n; e += QR_THREADS) {
    const int r = e % n, c = e / n;
    double2 o = make_double2(0.0, 0.0);
    const double2 al = alpha_s[r];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    if (r == c) {
      o = make_double2(aa, 0.0);
    } else if (c > r) {
      const double2 ph = aa > 0.0 ? make_double2(al.x / aa, -al.y / aa) : make_double2(1.0, 0.0);
      const double2 a = Aw[(int64_t)c * m + r];
      o = make_double2(a.x * ph.x - a.y * ph.y, a.x * ph.y + a.y * ph.x);
    }
    if (p.conjR) o.y = -o.y;
    p.R[(int64_t)r * p.r_rs + (int64_t)c * p.r_cs] = o;
  }
  __syncthreads();

  // thin Q in place: after step j, columns j..n-1 hold H_j ... H_{n-1} [I; 0]
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    double2 *v = Aw + (int64_t)j * m;    // v_j in rows j..m-1
    // row j of the accumulated columns c > j is zero (it held R[j][c])
    for (int c = j + 1 + tid; c < n; c += QR_THREADS) Aw[(int64_t)c * m + j] = make_double2(0.0, 0.0);
    __syncthreads();
    if (tau != 0.0) {
      for (int cb = j + 1; cb < n; cb += QB_COLS) {
        const int c = cb + cl;
        double2 *qc = Aw + (int64_t)c * m;
        double dr = 0.0, di = 0.0;
        if (c < n) {
          for (int r = j + g; r < m; r += 32) {
            const double2 vv = v[r], a = qc[r];
            dr += vv.x * a.x + vv.y * a.y;
            di += vv.x * a.y - vv.y * a.x;
          }
        }
        part[cl][g] = make_double2(dr, di);
        __syncthreads();
        if (c < n) {
          double sr = 0.0, si = 0.0;
          for (int t = 0; t < 32; ++t) {
            const double2 pv = part[cl][t];
            sr += pv.x;
            si += pv.y;
          }
          sr *= tau;
          si *= tau;
          for (int r = j + g; r < m; r += 32) {
            const double2 vv = v[r];
            double2 a = qc[r];
            a.x -= vv.x * sr - vv.y * si;
            a.y -= vv.x * si + vv.y * sr;
            qc[r] = a;
          }
        }
        __syncthreads();
      }
    }
    // column j <- H_j e_j = e_j - tau v conj(v_j)
    const double2 v0 = v[j];
    __syncthreads();
    for (int r = tid; r < m; r += QR_THREADS) {
      double2 o;
      if (r < j) {
        o = make_double2(0.0, 0.0);
      } else {
        const double2 vv = v[r];
        o = make_double2(-tau * (vv.x * v0.x + vv.y * v0.y), -tau * (vv.y * v0.x - vv.x * v0.y));
        if (r == j) o.x += 1.0;
      }
      v[r] = o;
    }
    __syncthreads();
  }

  for (int e = tid; e < m * n; e += QR_THREADS) {
    const int r = e % m, c = e / m;
    const double2 al = alpha_s[c];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
    const double2 q = Aw[e];
    double2 o = make_double2(q.x * ph.x - q.y * ph.y, q.x * ph.y + q.y * ph.x);
    if (p.conjQ) o.y = -o.y;
    p.Q[(int64_t)r * p.q_rs + (int64_t)c * p.q_cs] = o;
  }
}

// ---------------------------------------------------------------------------
// Multi-work-group path for matrices too large for one work-group's LDS.
// The matrix is copied column-major into the workspace and factored in
// panels of nb columns.  Each panel kernel: every work-group loads the panel
// into its LDS and factors it (all work-groups take identical steps, so
// they hold identical reflectors; work-group 0 writes them back), then
// applies the panel's reflectors to its own share of the trailing columns,
// one column per wave held in registers.  A last kernel forms Q (each wave
// one column, starting from e_c, reflector panels streamed through LDS from
// the last to the first) and writes R, with the phases that make diag(R)
// real and non-negative.

constexpr int PB_THREADS = 256;
constexpr int RPL = 40;                     // rows per lane held in registers: m <= 2560
constexpr int PANEL_LDS_ELEMS = 8960;       // 140 KiB of complex doubles

struct PanelArgs {
  double2 *Aw;        // m x n column-major (leading dimension m), trailing columns updated in place
  double2 *Vst;       // m x n column-major: factored panel columns (R above, reflectors below)
  double *tau;        // [n]
  double2 *alpha;     // [n]
  int m, n, c0, nb;
  int64_t ws;         // instance stride of the work area (complex elements), instance = blockIdx.y
};

__device__ __forceinline__ double bsum256(double v, double *sh) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(PB_THREADS) void qr_panel_kernel(PanelArgs a) {
  extern __shared__ double2 P[];
  {
    const int64_t o = (int64_t)blockIdx.y * a.ws;
    a.Aw += o;
    a.Vst += o;
    a.alpha += o;
    a.tau = reinterpret_cast<double *>(reinterpret_cast<double2 *>(a.tau) + o);
  }
  __shared__ double sh[4];
  __shared__ double tau_p[8];
  __shared__ double2 al_p[8];
  const int m = a.m, n = a.n, c0 = a.c0, nb = a.nb;
  const int mp = m - c0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < mp * nb; e += PB_THREADS) {
    const int r = e % mp, c = e / mp;
    P[e] = a.Aw[(int64_t)(c0 + c) * m + c0 + r];
  }
  __syncthreads();
  // factor the panel in LDS (row r of the panel = row c0 + r of the matrix)
  for (int j = 0; j < nb; ++j) {
    double2 *col = P + (int64_t)j * mp;
    double s = 0.0;
    for (int r = j + 1 + tid; r < mp; r += PB_THREADS) s += col[r].x * col[r].x + col[r].y * col[r].y;
    const double tail = bsum256(s, sh);
    if (tid == 0) {
      const double2 x0 = col[j];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nx = sqrt(tail + ax0 * ax0);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
      const double2 v0 = make_double2(x0.x - al.x, x0.y - al.y);
      const double vn2 = tail + (v0.x * v0.x + v0.y * v0.y);
      tau_p[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      al_p[j] = al;
      col[j] = v0;
    }
    __syncthreads();
    const double tau = tau_p[j];
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < nb; c += PB_THREADS / 64) {
        double2 *cc = P + (int64_t)c * mp;
        double dr = 0.0, di = 0.0;
        for (int r = j + lane; r < mp; r += 64) {
          const double2 v = col[r], x = cc[r];
          dr += v.x * x.x + v.y * x.y;
          di += v.x * x.y - v.y * x.x;
        }
        dr = wsum(dr) * tau;
        di = wsum(di) * tau;
        for (int r = j + lane; r < mp; r += 64) {
          const double2 v = col[r];
          double2 x = cc[r];
          x.x -= v.x * dr - v.y * di;
          x.y -= v.x * di + v.y * dr;
          cc[r] = x;
        }
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    // factored panel -> Vst (a separate array: other work-groups may still be
    // reading the panel from Aw); rows above the panel are final already
    for (int e = tid; e < mp * nb; e += PB_THREADS) {
      const int r = e % mp, c = e / mp;
      a.Vst[(int64_t)(c0 + c) * m + c0 + r] = P[e];
    }
    for (int e = tid; e < c0 * nb; e += PB_THREADS) {
      const int r = e % c0, c = e / c0;
      a.Vst[(int64_t)(c0 + c) * m + r] = a.Aw[(int64_t)(c0 + c) * m + r];
    }
    if (tid < nb) {
      a.tau[c0 + tid] = tau_p[tid];
      a.alpha[c0 + tid] = al_p[tid];
    }
  }
  // trailing columns: one per wave, rows c0..m-1 in registers
  const int gw = blockIdx.x * (PB_THREADS / 64) + wave;
  const int nw = gridDim.x * (PB_THREADS / 64);
  for (int c = c0 + nb + gw; c < n; c += nw) {
    double2 *cg = a.Aw + (int64_t)c * m + c0;
    double2 x[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      x[q] = r < mp ? cg[r] : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < nb; ++j) {
      const double tau = tau_p[j];
      if (tau == 0.0) continue;
      const double2 *v = P + (int64_t)j * mp;
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r >= j && r < mp) {
          const double2 vv = v[r];
          dr += vv.x * x[q].x + vv.y * x[q].y;
          di += vv.x * x[q].y - vv.y * x[q].x;
        }
      }
      dr = wsum(dr) * tau;
      di = wsum(di) * tau;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r >= j && r < mp) {
          const double2 vv = v[r];
          x[q].x -= vv.x * dr - vv.y * di;
          x[q].y -= vv.x * di + vv.y * dr;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (r < mp) cg[r] = x[q];
    }
  }
}

struct FormArgs {
  const double2 *Aw;   // the factored matrix (Vst of the panel kernels)
  const double *tau;
  const double2 *alpha;
  int m, n, nb;
  double2 *Q; int64_t q_rs, q_cs; int conjQ;
  double2 *R; int64_t r_rs, r_cs; int conjR;
  int64_t ws, qs, rs;  // instance strides (work, Q, R), instance = blockIdx.y
};

// Q column c = H_0 ... H_c e_c (one wave per column), and R column c.
__global__ __launch_bounds__(PB_THREADS) void qr_form_kernel(FormArgs a) {
  extern __shared__ double2 V[];
  {
    const int64_t r = blockIdx.y;
    a.Aw += r * a.ws;
    a.alpha += r * a.ws;
    a.tau = reinterpret_cast<const double *>(reinterpret_cast<const double2 *>(a.tau) + r * a.ws);
    a.Q += r * a.qs;
    a.R += r * a.rs;
  }
  const int m = a.m, n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = blockIdx.x * (PB_THREADS / 64) + wave;
  const bool active = c < n;
  double2 x[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = lane + 64 * q;
    x[q] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  // the reflectors that touch column c are H_0..H_c; panels from the one holding c down to 0
  int cmax = blockIdx.x * (PB_THREADS / 64) + (PB_THREADS / 64) - 1;
  if (cmax > n - 1) cmax = n - 1;
  for (int c0 = (cmax / a.nb) * a.nb; c0 >= 0; c0 -= a.nb) {
    const int nbp = (c0 + a.nb <= n) ? a.nb : n - c0;
    const int mp = m - c0;
    __syncthreads();
    for (int e = tid; e < mp * nbp; e += PB_THREADS) {
      const int r = e % mp, cc = e / mp;
      V[e] = a.Aw[(int64_t)(c0 + cc) * m + c0 + r];
    }
    __syncthreads();
    if (!active) continue;
    for (int jj = nbp - 1; jj >= 0; --jj) {
      const int j = c0 + jj;
      if (j > c) continue;
      const double tau = a.tau[j];
      if (tau == 0.0) continue;
      const double2 *v = V + (int64_t)jj * mp;   // v_j row r (matrix row c0 + r), valid for r >= jj
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;          // matrix row
        if (r >= j && r < m) {
          const double2 vv = v[r - c0];
          dr += vv.x * x[q].x + vv.y * x[q].y;
          di += vv.x * x[q].y - vv.y * x[q].x;
        }
      }
      dr = wsum(dr) * tau;
      di = wsum(di) * tau;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r >= j && r < m) {
          const double2 vv = v[r - c0];
          x[q].x -= vv.x * dr - vv.y * di;
          x[q].y -= vv.x * di + vv.y * dr;
        }
      }
    }
  }
  if (!active) return;
  const double2 al = a.alpha[c];
  const double aa = sqrt(al.x * al.x + al.y * al.y);
  const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = lane + 64 * q;
    if (r < m) {
      double2 o = make_double2(x[q].x * ph.x - x[q].y * ph.y, x[q].x * ph.y + x[q].y * ph.x);
      if (a.conjQ) o.y = -o.y;
      a.Q[(int64_t)r * a.q_rs + (int64_t)c * a.q_cs] = o;
    }
  }
  for (int r = lane; r < n; r += 64) {
    double2 o = make_double2(0.0, 0.0);
    if (r == c) {
      o = make_double2(aa, 0.0);
    } else if (r < c) {
      const double2 ar = a.alpha[r];
      const double ra = sqrt(ar.x * ar.x + ar.y * ar.y);
      const double2 pr = ra > 0.0 ? make_double2(ar.x / ra, -ar.y / ra) : make_double2(1.0, 0.0);
      const double2 v = a.Aw[(int64_t)c * m + r];
      o = make_double2(v.x * pr.x - v.y * pr.y, v.x * pr.y + v.y * pr.x);
    }
    if (a.conjR) o.y = -o.y;
    a.R[(int64_t)r * a.r_rs + (int64_t)c * a.r_cs] = o;
  }
}

__global__ void qr_load_kernel(QrArgs p) {
  p.A += (int64_t)blockIdx.y * p.inst.a;
  p.work += (int64_t)blockIdx.y * p.inst.skip;
  const int64_t tot = (int64_t)p.m * p.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % p.m), c = (int)(e / p.m);
    double2 v = p.A[(int64_t)r * p.a_rs + (int64_t)c * p.a_cs];
    if (p.conjA) v.y = -v.y;
    p.work[e] = v;
  }
}

bool lds_ok = false;
bool panel_ok = false;
bool reg_ok = false;

}  // namespace

void qr_init() {
  reg_ok = hipFuncSetAttribute((const void *)qr_reg_kernel<8>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               QRR_ELEMS * (int)sizeof(double2)) == hipSuccess;
  lds_ok = hipFuncSetAttribute((const void *)qr_lds_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               QR_LDS_ELEMS * (int)sizeof(double2)) == hipSuccess;
  panel_ok = hipFuncSetAttribute((const void *)qr_panel_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 PANEL_LDS_ELEMS * (int)sizeof(double2)) == hipSuccess &&
             hipFuncSetAttribute((const void *)qr_form_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 PANEL_LDS_ELEMS * (int)sizeof(double2)) == hipSuccess;
  (void)hipGetLastError();
}


hipError_t qr(const QrArgs &a, hipStream_t s) {
  if (a.n > 256 || a.m < a.n || a.n <= 0) return hipErrorInvalidValue;
  const int64_t elems = (int64_t)a.m * a.n;
  const int R = a.inst.count;
  if (R <= 0) return hipSuccess;
  if (reg_ok && a.n <= 32 && a.m <= 256) {
    hipLaunchKernelGGL(qr_reg_kernel<8>, dim3(R), dim3(QR_THREADS), (size_t)elems * sizeof(double2),
                       s, a);
    return hipGetLastError();
  }
  if (lds_ok && elems <= QR_LDS_ELEMS) {
    hipLaunchKernelGGL(qr_lds_kernel, dim3(R), dim3(QR_THREADS), elems * sizeof(double2), s, a);
    return hipGetLastError();
  }
  if (cholqr_ok(a.m, a.n)) return cholqr(a, s);
  int nb = PANEL_LDS_ELEMS / a.m;
  if (nb > 8) nb = 8;
  if (!panel_ok || a.m > 64 * RPL || nb < 1) {
    hipLaunchKernelGGL(qr_kernel, dim3(R), dim3(QR_THREADS), 0, s, a);
    return hipGetLastError();
  }
  // workspace: Aw (m n) | Vst (m n) | alpha (n) | tau (n doubles)
  double2 *Aw = a.work;
  double2 *Vst = a.work + elems;
  double2 *alpha = a.work + 2 * elems;
  double *tau = reinterpret_cast<double *>(a.work + 2 * elems + a.n);
  {
    int64_t g = (elems + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(qr_load_kernel, dim3((int)g, R), dim3(256), 0, s, a);
  }
  for (int c0 = 0; c0 < a.n; c0 += nb) {
    const int nbp = (c0 + nb <= a.n) ? nb : a.n - c0;
    const int trailing = a.n - c0 - nbp;
    int groups = (trailing + (PB_THREADS / 64) - 1) / (PB_THREADS / 64);
    if (groups < 1) groups = 1;
    PanelArgs pa{Aw, Vst, tau, alpha, a.m, a.n, c0, nbp, a.inst.skip};
    hipLaunchKernelGGL(qr_panel_kernel, dim3(groups, R), dim3(PB_THREADS),
                       (size_t)(a.m - c0) * nbp * sizeof(double2), s, pa);
  }
  FormArgs fa{Vst, tau, alpha, a.m, a.n, nb, a.Q, a.q_rs, a.q_cs, a.conjQ, a.R, a.r_rs, a.r_cs, a.conjR,
              a.inst.skip, a.inst.b, a.inst.c};
  const int groups = (a.n + (PB_THREADS / 64) - 1) / (PB_THREADS / 64);
  hipLaunchKernelGGL(qr_form_kernel, dim3(groups, R), dim3(PB_THREADS),
                     (size_t)a.m * nb * sizeof(double2), s, fa);
  return hipGetLastError();
}

}  // namespace tdvp
