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
// device.  Matrices too large for one work-group's LDS take the shifted
// Cholesky QR (cholqr.hip), which returns the same factorisation.
#include "common.h"

namespace tdvp {

namespace {

constexpr int QR_THREADS = 1024;
constexpr int QR_LDS_ELEMS = 8704;          // 136 KiB of complex doubles (+ 23 KiB static)

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
// LDS path, tuned for the tall-skinny shapes of the sweep (m n <= 8704).
// Same reflectors, R and Q as the register path; the trailing-column work
// of a step is spread over the whole work-group:
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

bool lds_ok = false;
bool reg_ok = false;

}  // namespace

void qr_init() {
  reg_ok = hipFuncSetAttribute((const void *)qr_reg_kernel<8>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               QRR_ELEMS * (int)sizeof(double2)) == hipSuccess;
  lds_ok = hipFuncSetAttribute((const void *)qr_lds_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               QR_LDS_ELEMS * (int)sizeof(double2)) == hipSuccess;
  (void)hipGetLastError();
  cholqr_init();
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
  // every other shape (n <= 256, m >= n): shifted Cholesky QR
  return cholqr(a, s);
}

}  // namespace tdvp
