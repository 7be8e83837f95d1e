// Declarations of the small device utilities (util.hip).
#pragma once

namespace tdvp {

// p[r * is] = 1 + 0i for r < count
hipError_t fill_one(void *p, DType t, hipStream_t s, int count = 1, int64_t is = 0);
hipError_t copy_c128(double2 *dst, const double2 *src, int64_t n, hipStream_t s);
hipError_t set_dev_int(int *p, int v, hipStream_t s);
// *out = Re sum_e conj(a_e) sum_p y[p][e]   (y: P partials of n elements, stride pstride)
hipError_t dot_partials(const double2 *a, DType ty, const void *y, int P, int64_t pstride,
                        int64_t n, double *out, hipStream_t s, int count = 1, int64_t ia = 0,
                        int64_t iy = 0, int64_t io = 0);
// *out = Re sum_{r,c} conj(a[r rs + c cs]) b[r rs + c cs]
hipError_t dot2d(const double2 *a, const double2 *b, int rows, int cols, int64_t rs, int64_t cs,
                 double *out, hipStream_t s, int count = 1, int64_t ia = 0, int64_t ib = 0,
                 int64_t io = 0);
// out[e] = sum_p y[p][e]
hipError_t sum_partials(DType ty, const void *y, int P, int64_t pstride, int64_t n, double2 *out,
                        hipStream_t s);
// dst[r is] += c src[r is] for r < count
hipError_t axpy_scalar(double *dst, const double *src, double c, hipStream_t s, int count = 1,
                       int64_t is = 0);
hipError_t normalize_c128(double2 *a, int64_t n, hipStream_t s);                  // a /= |a|
// *out = 1 if any of the count instance flags (flag + r * fstride ints) is set
// or any of vals[r * vs + 0 .. nv-1] is not finite, else 0
hipError_t numeric_check(const int *flag, int64_t fstride, const double *vals, int64_t vs, int nv,
                         int count, int *out, hipStream_t s);

}  // namespace tdvp
