// Small device utilities: fills, copies, and single-work-group reductions used
// by the observables (populations, norm, energy; Sec. III.A) and by the
// normalisation of the gauge centre.  Reductions run in one work-group in a
// fixed order, so they are deterministic.
#include "common.h"
#include "util.h"

namespace tdvp {

namespace {

constexpr int RT = 1024;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double bsum(double v) {
  __shared__ double sh[RT / 64];
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < RT / 64; ++w) t += sh[w];
  return t;
}

__global__ void fill_one_kernel(void *p, int t, int64_t is) {
  if (t == F64) reinterpret_cast<double2 *>(p)[threadIdx.x * is] = make_double2(1.0, 0.0);
  else reinterpret_cast<float2 *>(p)[threadIdx.x * is] = make_float2(1.0f, 0.0f);
}

__global__ void copy_kernel(double2 *dst, const double2 *src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

template <typename TY>
__global__ __launch_bounds__(RT) void dot_partials_kernel(const double2 *a, const TY *y, int P,
                                                          int64_t pstride, int64_t n, double *out,
                                                          int64_t ia, int64_t iy, int64_t io) {
  a += blockIdx.x * ia;
  y += blockIdx.x * iy;
  out += blockIdx.x * io;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += RT) {
    double yr = 0.0, yi = 0.0;
    for (int p = 0; p < P; ++p) {
      const TY v = y[(int64_t)p * pstride + e];
      yr += (double)v.x;
      yi += (double)v.y;
    }
    s += a[e].x * yr + a[e].y * yi;
  }
  s = bsum(s);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(RT) void dot2d_kernel(const double2 *a, const double2 *b, int rows,
                                                   int cols, int64_t rs, int64_t cs, double *out,
                                                   int64_t ia, int64_t ib, int64_t io) {
  a += blockIdx.x * ia;
  b += blockIdx.x * ib;
  out += blockIdx.x * io;
  double s = 0.0;
  const int64_t tot = (int64_t)rows * cols;
  for (int64_t e = threadIdx.x; e < tot; e += RT) {
    const int64_t r = e / cols, c = e % cols;
    const double2 x = a[r * rs + c * cs], y = b[r * rs + c * cs];
    s += x.x * y.x + x.y * y.y;
  }
  s = bsum(s);
  if (threadIdx.x == 0) *out = s;
}

template <typename TY>
__global__ void sum_partials_kernel(const TY *y, int P, int64_t pstride, int64_t n, double2 *out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double r = 0.0, i = 0.0;
    for (int p = 0; p < P; ++p) {
      const TY v = y[(int64_t)p * pstride + e];
      r += (double)v.x;
      i += (double)v.y;
    }
    out[e] = make_double2(r, i);
  }
}

__global__ void axpy_scalar_kernel(double *dst, const double *src, double c, int64_t is) {
  dst[threadIdx.x * is] += c * src[threadIdx.x * is];
}

__global__ __launch_bounds__(RT) void normalize_kernel(double2 *a, int64_t n) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += RT) s += a[e].x * a[e].x + a[e].y * a[e].y;
  s = bsum(s);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int64_t e = threadIdx.x; e < n; e += RT) {
    double2 v = a[e];
    v.x *= inv;
    v.y *= inv;
    a[e] = v;
  }
}

}  // namespace

hipError_t fill_one(void *p, DType t, hipStream_t s, int count, int64_t is) {
  hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(count), 0, s, p, (int)t, is);
  return hipGetLastError();
}

hipError_t copy_c128(double2 *dst, const double2 *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(copy_kernel, dim3((int)g), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t set_dev_int(int *p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t dot_partials(const double2 *a, DType ty, const void *y, int P, int64_t pstride, int64_t n,
                        double *out, hipStream_t s, int count, int64_t ia, int64_t iy, int64_t io) {
  if (ty == F64)
    hipLaunchKernelGGL(dot_partials_kernel<double2>, dim3(count), dim3(RT), 0, s, a,
                       (const double2 *)y, P, pstride, n, out, ia, iy, io);
  else
    hipLaunchKernelGGL(dot_partials_kernel<float2>, dim3(count), dim3(RT), 0, s, a,
                       (const float2 *)y, P, pstride, n, out, ia, iy, io);
  return hipGetLastError();
}

hipError_t dot2d(const double2 *a, const double2 *b, int rows, int cols, int64_t rs, int64_t cs,
                 double *out, hipStream_t s, int count, int64_t ia, int64_t ib, int64_t io) {
  hipLaunchKernelGGL(dot2d_kernel, dim3(count), dim3(RT), 0, s, a, b, rows, cols, rs, cs, out, ia, ib,
                     io);
  return hipGetLastError();
}

hipError_t sum_partials(DType ty, const void *y, int P, int64_t pstride, int64_t n, double2 *out,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (ty == F64)
    hipLaunchKernelGGL(sum_partials_kernel<double2>, dim3((int)g), dim3(256), 0, s,
                       (const double2 *)y, P, pstride, n, out);
  else
    hipLaunchKernelGGL(sum_partials_kernel<float2>, dim3((int)g), dim3(256), 0, s,
                       (const float2 *)y, P, pstride, n, out);
  return hipGetLastError();
}

hipError_t axpy_scalar(double *dst, const double *src, double c, hipStream_t s, int count, int64_t is) {
  hipLaunchKernelGGL(axpy_scalar_kernel, dim3(1), dim3(count), 0, s, dst, src, c, is);
  return hipGetLastError();
}

hipError_t normalize_c128(double2 *a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(RT), 0, s, a, n);
  return hipGetLastError();
}

// One work-group: thread t looks at the instances t, t + RT, ...
__global__ __launch_bounds__(RT) void numeric_check_kernel(const int *flag, int64_t fstride,
                                                           const double *vals, int64_t vs, int nv,
                                                           int count, int *out) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  int bad = 0;
  for (int r = threadIdx.x; r < count; r += RT) {
    if (flag[(int64_t)r * fstride] != 0) bad = 1;
    for (int v = 0; v < nv; ++v)
      if (!isfinite(vals[(int64_t)r * vs + v])) bad = 1;
  }
  if (bad) any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) *out = any;
}

hipError_t numeric_check(const int *flag, int64_t fstride, const double *vals, int64_t vs, int nv,
                         int count, int *out, hipStream_t s) {
  hipLaunchKernelGGL(numeric_check_kernel, dim3(1), dim3(RT), 0, s, flag, fstride, vals, vs, nv,
                     count, out);
  return hipGetLastError();
}

}  // namespace tdvp
