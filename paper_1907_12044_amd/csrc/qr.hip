// FP64 Householder QR of a tall complex matrix for the gauge shifts of the
// PS sweep (eq:QR; the right-to-left sweep uses the QR of C^H, i.e. an RQ).
//
// One work-group of 16 wave64 factors the matrix held column-major in LDS
// when it fits (m n <= QR_LDS_ELEMS), else in the workspace: for column j
// the reflector H_j = I - tau v v^H with v = x - alpha e_1 and
// alpha = -exp(i arg x_0) |x| (no cancellation in v_0) is built by a block
// reduction and applied to the trailing columns, one column per wave (dot
// by wave reduction, then an axpy).  R is written out, then the thin Q is
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
constexpr int QR_LDS_ELEMS = 9216;          // 144 KiB of complex doubles

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool IN_LDS>
__global__ __launch_bounds__(QR_THREADS) void qr_kernel(QrArgs p) {
  extern __shared__ double2 lds_mat[];
  const int m = p.m, n = p.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = QR_THREADS / 64;
  double2 *Aw = IN_LDS ? lds_mat : p.work;     // m x n column-major
  __shared__ double red[NW];
  __shared__ double tau_s[256];
  __shared__ double2 alpha_s[256];

  for (int64_t e = tid; e < (int64_t)m * n; e += QR_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    double2 v = p.A[(int64_t)r * p.a_rs + (int64_t)c * p.a_cs];
    if (p.conjA) v.y = -v.y;
    Aw[e] = v;
  }
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    double2 *col = Aw + (int64_t)j * m;
    double s = 0.0;
    for (int r = j + 1 + tid; r < m; r += QR_THREADS) s += col[r].x * col[r].x + col[r].y * col[r].y;
    s = wsum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double tail = 0.0;
      for (int w = 0; w < NW; ++w) tail += red[w];
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
        for (int r = j + lane; r < m; r += 64) {
          const double2 v = col[r];
          double2 a = cc[r];
          a.x -= v.x * dr - v.y * di;
          a.y -= v.x * di + v.y * dr;
          cc[r] = a;
        }
      }
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

bool lds_ok = false;

}  // namespace

void qr_init() {
  lds_ok = hipFuncSetAttribute((const void *)qr_kernel<true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               QR_LDS_ELEMS * (int)sizeof(double2)) == hipSuccess;
  (void)hipGetLastError();
}

hipError_t qr(const QrArgs &a, hipStream_t s) {
  if (a.n > 256 || a.m < a.n || a.n <= 0) return hipErrorInvalidValue;
  const int64_t elems = (int64_t)a.m * a.n;
  if (lds_ok && elems <= QR_LDS_ELEMS) {
    hipLaunchKernelGGL(qr_kernel<true>, dim3(1), dim3(QR_THREADS), elems * sizeof(double2), s, a);
  } else {
    hipLaunchKernelGGL(qr_kernel<false>, dim3(1), dim3(QR_THREADS), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace tdvp
