// Internal declarations shared by the libtdvp translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/tdvp.h"

namespace tdvp {

constexpr int KMAX = 32;          // largest Krylov dimension compiled in
constexpr int LZ_GRID = 512;      // most work-groups of lz_start / lz_update / lz_finish
constexpr int LZ_PARTS = 512;     // most per-work-group partials of one reduction
constexpr int LZ_BLOCK = 256;
static_assert(LZ_GRID <= LZ_PARTS, "one dot partial per work-group of the vector kernels");

enum DType { F64 = 0, F32 = 1 };

// Independent problem instances of identical shape handled by one launch
// (the disorder ensemble): instance r reads/writes every operand at
// base + r * (its instance stride, in elements of that operand; the skip
// flag stride is in ints).  count = 1 with zero strides is one problem.
struct Inst {
  int count = 1;
  int64_t a = 0, b = 0, c = 0, skip = 0;
};

// Grouped launches: one launch covers up to GMAX groups of instances whose
// shapes differ between groups (the bond-dimension classes of a disorder
// ensemble).  The grid is one-dimensional: group k owns the flat blocks
// [start[k], start[k + 1]), which it reads as its own (gx, gy, gz) grid in
// the order x fastest, then y, then z, as a launch of that group alone
// would; every group has its own argument set.
constexpr int GMAX = 4;
struct BlockXYZ {
  int x, y, z, gx, gy, gz;
};
template <typename A> struct Grp {
  A a[GMAX];
  int ng = 0;
  int gx[GMAX] = {}, gy[GMAX] = {}, gz[GMAX] = {};
  int start[GMAX + 1] = {};
#ifdef __HIPCC__
  __device__ __forceinline__ BlockXYZ locate(int flat, int &k) const {
    k = 0;
    while (k + 1 < ng && flat >= start[k + 1]) ++k;
    const int local = flat - start[k];
    BlockXYZ b;
    b.gx = gx[k];
    b.gy = gy[k];
    b.gz = gz[k];
    b.x = local % b.gx;
    b.y = (local / b.gx) % b.gy;
    b.z = local / (b.gx * b.gy);
    return b;
  }
#endif
  // append a group with grid (x, y, z); false if full
  bool add(const A &args, int x, int y, int z) {
    if (ng >= GMAX || x <= 0 || y <= 0 || z <= 0) return ng < GMAX;
    a[ng] = args;
    gx[ng] = x;
    gy[ng] = y;
    gz[ng] = z;
    start[ng + 1] = start[ng] + x * y * z;
    ++ng;
    return true;
  }
  int blocks() const { return start[ng]; }
};
#ifdef __HIPCC__
__device__ __forceinline__ BlockXYZ native_block() {
  BlockXYZ b;
  b.x = blockIdx.x;
  b.y = blockIdx.y;
  b.z = blockIdx.z;
  b.gx = gridDim.x;
  b.gy = gridDim.y;
  b.gz = gridDim.z;
  return b;
}
#endif

// Complex GEMM  C[b][m,n] = sum_k opA(A)[b][m,k] * opB(B)[b][k,n]
// with arbitrary element strides (in complex elements) and optional
// conjugation.  Batches b = 0..batch-1.  Optional `skip`: if non-null and
// *skip != 0 the kernel returns at once (used to predicate Krylov steps).
struct LzPartials;

struct GemmArgs {
  const void *A; const void *B; void *C;
  int M, N, K, batch;
  int64_t sam, sak, sbk, sbn, scm, scn;
  int64_t bsa, bsb, bsc;     // batch strides
  int conjA, conjB;
  const int *skip;
  Inst inst;                 // a = A, b = B, c = C strides
  int tile;                  // 0: by problem size; 32: 32x32 tiles; 64, 96, 128: 64x64 tiles with
                             // K steps of 16, 32, 64 (the last two in FP32 arithmetic only)
  int mode;                  // 0: C = op(A) op(B); 1: C = C - op(A) op(B); 2: C = -op(A) op(B)
  // Lanczos projection epilogue (lzU != NULL; mode 0, batch 1, C row-major
  // with scn = 1, so that element (m, n) is entry m N + n of a length-M N
  // vector): C is not written; instead w = op(A) op(B) goes in FP64 to basis
  // vector lzj + 1 of lzU (vectors of length M N, consecutive), and every
  // work-group writes its partials <u_i, w> (i <= lzj) and |w|^2 to slot
  // (tile index) of lzpp->dot / lzpp->w2, and the tile count to
  // lzpp->ndot.  lzU and lzpp step by lzwss bytes per instance.
  double2 *lzU;
  LzPartials *lzpp;
  int lzj;
  int64_t lzwss;
};

hipError_t cgemm(DType ta, DType tb, DType tc, const GemmArgs &g, hipStream_t s);
// One launch for up to GMAX argument sets of the same types (FP32 output
// with split-BF16 arithmetic when bf3 != 0); tile: one tile choice for the
// launch (0: by the largest group).
hipError_t cgemm_grouped(DType ta, DType tb, DType tc, const GemmArgs *g, int ng, int bf3, hipStream_t s);
// Same product with split-BF16 matrix-core arithmetic and FP32 accumulation
// (about 17 significant bits per operand); FP32 output only.
hipError_t cgemm_bf3(DType ta, DType tb, DType tc, const GemmArgs &g, hipStream_t s);

// Sparse MPO-channel contraction (stage 2 of H_eff / environment update):
//   out[wo][so][a][c] = sum_{wi, si} Wt(wo, so, si, wi) * in[wi][si][a][c]
// where Wt reads the MPO tensor W (Wl, d, d, Wr) c128 either as
// W[wo][so][si][wi] (w_in_right = 1: input channel is the right MPO bond) or
// W[wi][so][si][wo] (w_in_right = 0).  Strides in complex elements.
struct WApplyArgs {
  const void *in; void *out; const void *W;
  int Wl, Wr, d, A, C;
  int w_in_right;
  int64_t si_w, si_s, si_a, si_c;   // input strides (w, s, a, c)
  int64_t so_w, so_s, so_a, so_c;   // output strides
  const int *skip;
  Inst inst;                        // a = in, b = W, c = out strides
};
hipError_t wapply(DType t, const WApplyArgs &a, hipStream_t s);
hipError_t wapply_grouped(DType t, const WApplyArgs *a, int ng, hipStream_t s);

// Lanczos state kept in device memory for the solve in flight.  Scalars
// are written by work-group 0 of the kernel that reduces them; every
// work-group of a kernel derives the same values from the same partials in
// the same order, so all of them take the same decisions.
struct LzState {
  double alpha[KMAX];
  double beta[KMAX];
  double scale[KMAX + 1];     // v_j = scale_j * u_j
  double aw[KMAX];            // |H v_j|
  double xnorm;
  int stop;                   // != 0: the basis is final (k vectors)
  int k;
  int keff;                   // largest basis for this solve: min(kmax, dim)
  double z_re, z_im, tol;
  int *nonfinite;             // the context's sticky flag (CtxHeader), set by lz_start
};

// First bytes of the caller's workspace: context-wide device flags.
struct CtxHeader {
  int nonfinite;              // sticky: a Lanczos norm of some solve was NaN or Inf
                              // (cleared only by tdvp_set_workspace)
  int numeric_out;            // result of the last numeric_check
};
constexpr size_t CTX_HEADER_BYTES = 256;

// Per-work-group partial sums.  Norm partials (lz_start, lz_update) and dot
// partials (lz_dots) live in separate arrays so a kernel never reads the
// array it writes.
struct LzPartials {
  double nrm[LZ_GRID];
  // second buffer of the norm partials for lz_update with close: step k
  // writes (k odd ? nrm : nrm_odd) and closes step k - 1 from the other
  // buffer, so no work-group overwrites partials that another still reads
  double nrm_odd[LZ_GRID];
  double2 dot[KMAX + 1][LZ_PARTS];   // <u_i, H u_j> partials, [i][work-group]
  double w2[LZ_PARTS];          // |H u_j|^2 partials (lz_dots, or lz_update on the fused path)
  int ndot;                     // partials written by a GEMM projection epilogue
};

// Lanczos kernels over `inst.count` instances: instance r uses the state,
// partials, basis and partial outputs at (base + r * wss bytes) and the
// input/output vectors x, y at + r * xs / ys elements.
struct LzInst {
  int count = 1;
  int64_t wss = 0, xs = 0, ys = 0;
};
// trows > 0 (lz_start, lz_finish): the basis is stored column-major, index
// c * trows + r for the element (r, c) of the row-major n / trows-column x, y.
hipError_t lz_start(LzState *st, LzPartials *pp, const double2 *x, double2 *u0, int64_t n,
                    double zr, double zi, double tol, int keff, int trows, int *nonfinite,
                    const LzInst &in, hipStream_t s);
hipError_t lz_dots(LzState *st, LzPartials *pp, DType ty, const void *ypart, int P, int64_t pstride,
                   double2 *U, int64_t ldu, int j, int64_t n, const LzInst &in, hipStream_t s);
// Gd: number of per-work-group dot partials written by the kernel before
// (0 = the lz_dots grid for n; < 0: pp->ndot, written by a GEMM projection
// epilogue).  Yp != NULL (fused path): H u_j is the sum of the P partial
// vectors Yp + p n (instance stride in.wss bytes), and the kernel also
// writes the |H u_j|^2 partials.  close != 0 (after a GEMM projection
// epilogue, which has no step close of its own): the kernel first closes
// step j - 1 as lz_dots does (beta, scale_j, stop tests).
hipError_t lz_update(LzState *st, LzPartials *pp, double2 *U, int64_t ldu, int j, int64_t n, int Gd,
                     const double2 *Yp, int P, const LzInst &in, hipStream_t s, int close = 0);
int lz_grid(int64_t n, int count);   // work-groups per instance of the Lanczos vector kernels

// Argument sets of the Lanczos kernels for grouped launches (one per group;
// every group of a launch is at the same Krylov index j).
struct LzStartArgs {
  LzState *st; LzPartials *pp; const double2 *x; double2 *u0; int64_t n;
  double zr, zi, tol; int keff, trows; int *nonfinite; LzInst in;
};
struct LzDotsArgs {
  LzState *st; LzPartials *pp; const void *ypart; int P; int64_t pstride;
  double2 *U; int64_t ldu; int j; int64_t n; LzInst in;
};
struct LzUpdateArgs {
  LzState *st; LzPartials *pp; double2 *U; int64_t ldu; int j; int64_t n; int Gd;
  const double2 *Yp; int P; LzInst in; int close = 0;
};
struct LzFinishArgs {
  LzState *st; const double2 *U; int64_t ldu; int64_t n; int keff; double2 *y; int32_t *k_used;
  int trows; LzInst in;
};
hipError_t lz_start_grouped(const LzStartArgs *a, int ng, hipStream_t s);
hipError_t lz_dots_grouped(DType ty, const LzDotsArgs *a, int ng, hipStream_t s);
hipError_t lz_update_grouped(const LzUpdateArgs *a, int ng, hipStream_t s);
hipError_t lz_finish_grouped(const LzFinishArgs *a, int ng, hipStream_t s);
hipError_t lz_finish(LzState *st, const double2 *U, int64_t ldu, int64_t n, int keff, double2 *y,
                     int32_t *k_used, int trows, const LzInst &in, hipStream_t s);

// Fused Lanczos step: H u_j and its partial projections in one launch,
// grid (Mr P, instances).  u_j = U + j n, column-major (rows Ml d).  Work-group
// (p, r') forms the part of column r' of H u_j that comes from the bra-side
// indices l in [p nl, (p + 1) nl) (the sum over l split P ways) and writes it
// to Yp + p n; its dots with u_0..u_j go to partial slot p Mr + r'.  The
// operator is H[i] with W given by its nonzero table (row, col, coef from
// wtable) or, with row == NULL, the bond operator (d = 1, Wl == Wr).
constexpr size_t HEFF_SMALL_LDS = 150 * 1024;
constexpr int HS_PMAX = 8;              // most parts P
struct HeffSmallArgs {
  LzState *st; LzPartials *pp; double2 *U;
  double2 *Yp;                          // P partial vectors of n (workspace)
  int64_t n; int j;
  int Gprev, Gw;                        // norm and |H u|^2 partials written by the kernel before
  int P, nl;                            // parts, bra indices per part
  int staged;                           // 1: x and L slices staged through LDS
  const void *L, *R;                    // environments (context element type)
  const int *row, *col; const double2 *coef;   // CSR table of W (wtable), in the workspace
  int Ml, d, Mr, Wl, Wr;
  int64_t wss, sL, sR;                  // instance strides: workspace bytes, env elements
};
size_t heff_small_lds(const HeffSmallArgs &a, int tm_bytes);
bool heff_small_fits(const HeffSmallArgs &a, int tm_bytes);
hipError_t heff_small(DType t, const HeffSmallArgs &a, int count, hipStream_t s);
// One launch over ng argument sets (count[k] instances each, the same
// Krylov index j and the same `staged` choice in every set).
hipError_t heff_small_grouped(DType t, const HeffSmallArgs *a, const int *count, int ng, hipStream_t s);
// CSR table of W[wl][s'][s][wr] (instance stride sW elements) over rows
// wl d + s' (Wl d <= 256, Wl d d Wr <= WT_MAX): row pointers rowp[Wl d + 1],
// then col (s Wr + wr) and coef of each nonzero in index order.  Outputs at
// instance stride wss bytes.
constexpr int WT_MAX = 8192;
hipError_t wtable(const double2 *W, int Wl, int d, int Wr, int64_t sW, int *rowp, int *col,
                  double2 *coef, int64_t wss, int count, hipStream_t s);
struct WtableArgs {
  const double2 *W; int rows, cap; int64_t sW; int *rowp; int *col; double2 *coef; int64_t wss;
  int count;
};
hipError_t wtable_grouped(const WtableArgs *a, int ng, hipStream_t s);

// QR of an m x n (m >= n, n <= 256) c128 matrix given by strides; writes
// Q (m x n) and R (n x n) through output strides, with optional conjugation
// on input and outputs.  Householder in one work-group while m n fits its
// LDS, else shifted Cholesky QR; work: cholqr_work_elems(m, n) c128.
struct QrArgs {
  const double2 *A; int64_t a_rs, a_cs; int conjA;
  double2 *Q; int64_t q_rs, q_cs; int conjQ;
  double2 *R; int64_t r_rs, r_cs; int conjR;
  int m, n;
  double2 *work;
  Inst inst;      // a = A, b = Q, c = R strides; skip = work stride (elements)
};
hipError_t qr(const QrArgs &a, hipStream_t s);
// Shifted Cholesky QR (three passes) for m >= n, n <= 256; the work area
// (QrArgs::work, instance stride inst.skip) must hold cholqr_work_elems c128.
bool cholqr_ok(int m, int n);
int64_t cholqr_work_elems(int m, int n);
hipError_t cholqr(const QrArgs &a, hipStream_t s);
void cholqr_init();   // called by qr_init
void qr_init();       // once per process, outside stream capture

// TDVP-MU (mu.hip).  Regularised inverses P = V Lam~^{-1} U^H of n x n
// bond matrices D = U Lam V^H (row-major c128, n <= 64), Lam~ = Lam +
// sqrt(eps) exp(-Lam / sqrt(eps)) (eq:reg2): up to REGINV_BATCH independent
// matrices per launch, one work-group each.
constexpr int REGINV_BATCH = 64;
struct RegInvBatch {
  const double2 *D[REGINV_BATCH];
  double2 *P[REGINV_BATCH];
  int n[REGINV_BATCH];
  int count;
  double eps;
};
hipError_t mu_reginv(const RegInvBatch &b, hipStream_t s);
// Truncated SVD of a two-site tensor X (m x n row-major c128, m, n <= 64):
// the keep largest singular values, descending; mode 0: A = U (m x keep),
// B = Lam V^H (keep x n); mode 1: A = U Lam, B = V^H.  The sum of the
// squared singular values dropped is added to *discarded (device, may be null).
hipError_t svd_split(const double2 *X, int m, int n, int keep, int mode, double2 *A, double2 *B,
                     double *discarded, hipStream_t s);
// W = two MPO sites merged: W[w][(s1 s2)][(t1 t2)][v] = sum_u W1[w][s1][t1][u] W2[u][s2][t2][v].
hipError_t merge_mpo(const double2 *W1, const double2 *W2, int wl, int d1, int wm, int d2, int wr, double2 *W,
                     hipStream_t s);
// out = -i (X - Y), n elements (Y == null: out = -i X)
hipError_t mu_finish(const double2 *X, const double2 *Y, double2 *out, int64_t n, hipStream_t s);
constexpr int LINCOMB_MAX = 7;
struct LinComb {              // out = x0 + sum_{j < m} a[j] x[j]  (real coefficients; x0 null: 0)
  double2 *out; const double2 *x0;
  const double2 *x[LINCOMB_MAX];
  double a[LINCOMB_MAX];
  int m;
};
hipError_t lincomb(const LinComb &lc, int64_t n, hipStream_t s);
constexpr int RK_PARTS = 1024;  // most partial sums of rk_err_partials
// Per-work-group partial sums of |err_e / (atol + rtol max(|y_e|, |ynew_e|))|^2
// into part[0 .. g-1]; returns g (or -1 on a launch error).
int rk_err_partials(const double2 *err, const double2 *y, const double2 *ynew, int64_t n, double rtol,
                    double atol, double *part, hipStream_t s);

}  // namespace tdvp

#include "util.h"
