// FP64 Householder QR of a tall complex matrix for the gauge shifts of the
// PS sweep (eq:QR; the right-to-left sweep uses the QR of C^H, i.e. an RQ).
//
// One work-group of 16 wave64 factors the matrix held column-major in the
// workspace: for column j the reflector H_j = I - tau v v^H with
// v = x - alpha e_1, alpha = -exp(i arg x_0) |x| (no cancellation in v_0),
// is built by a block reduction and applied to the trailing columns, one
// column per wave (dot by wave reduction, then an axpy).  Q is accumulated
// backwards from the identity, and the phases of alpha_j are moved into Q
// so that diag(R) is real and non-negative.  Inputs and outputs go through
// element strides with optional conjugation, so the same kernel serves
// C = L D (left-to-right) and C^H = Q R, C = R^H Q^H (right-to-left).
// The matrix stays on the device: there is no host round trip.
#include "common.h"

namespace tdvp {

namespace {

constexpr int QR_THREADS = 1024;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(QR_THREADS) void qr_kernel(QrArgs p) {
  const int m = p.m, n = p.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = QR_THREADS / 64;
  double2 *Aw = p.work;                               // m x n column-major: v's below diag
  double2 *Qw = p.work + (int64_t)m * n;              // m x n column-major
  __shared__ double red[QR_THREADS / 64];
  __shared__ double tau_s[256];
  __shared__ double2 alpha_s[256];
  __shared__ double2 v0_s[256];

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
    for (int r = j + tid; r < m; r += QR_THREADS) s += col[r].x * col[r].x + col[r].y * col[r].y;
    s = wsum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double sig = 0.0;
      for (int w = 0; w < nwaves; ++w) sig += red[w];
      const double2 x0 = col[j];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nx = sqrt(sig);
      double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
      const double2 v0 = make_double2(x0.x - al.x, x0.y - al.y);
      const double vn2 = sig - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
      tau_s[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      alpha_s[j] = al;
      v0_s[j] = v0;
      col[j] = v0;
    }
    __syncthreads();
    const double tau = tau_s[j];
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += nwaves) {
        double2 *cc = Aw + (int64_t)c * m;
        double dr = 0.0, di = 0.0;   // v^H a_c
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

  // Q = H_0 H_1 ... H_{n-1} [I; 0], accumulated from the last reflector.
  for (int64_t e = tid; e < (int64_t)m * n; e += QR_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    Qw[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau == 0.0) continue;
    const double2 *v = Aw + (int64_t)j * m;     // v_j in rows j..m-1 (row j holds v0)
    for (int c = j + wave; c < n; c += nwaves) {
      double2 *qc = Qw + (int64_t)c * m;
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
    __syncthreads();
  }

  // outputs with diag(R) made real and non-negative: Q[:, j] *= ph_j, R[j, :] *= conj(ph_j)
  for (int64_t e = tid; e < (int64_t)m * n; e += QR_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    const double2 al = alpha_s[c];
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
    const double2 q = Qw[e];
    double2 o = make_double2(q.x * ph.x - q.y * ph.y, q.x * ph.y + q.y * ph.x);
    if (p.conjQ) o.y = -o.y;
    p.Q[(int64_t)r * p.q_rs + (int64_t)c * p.q_cs] = o;
  }
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
}

}  // namespace

hipError_t qr(const QrArgs &a, hipStream_t s) {
  if (a.n > 256 || a.m < a.n || a.n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(qr_kernel, dim3(1), dim3(QR_THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace tdvp
