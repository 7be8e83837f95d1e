// C ABI of libtdvp and the host driver of the TDVP-PS sweep.
//
// The driver only enqueues kernels on the context's stream; nothing in a
// step synchronises with the host.  Per site of a half sweep (eq:ps_trotter,
// eq:tdvp2_C, eq:tdvp2_D, eq:QR):
//   forward  : Lanczos exp(-i h H[i]) on C_i     (H[i] x = 3 contraction stages)
//   gauge    : QR (left-to-right) or QR of C^H (right-to-left), FP64
//   env      : h[1:i] or h[i:N] update (3 contraction stages)
//   backward : Lanczos exp(+i h K) on the bond matrix D (2 stages per K x)
//   centre   : C_{i+1} = D R_{i+1}  (or C_{i-1} = L_{i-1} D), one GEMM whose
//              result feeds the next forward solve directly.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <initializer_list>
#include <mutex>
#include <new>
#include <functional>
#include <vector>

#include "common.h"

using namespace tdvp;

namespace {
// One timed launch: HIP events on the context stream around a kernel of the
// selected class, with the algorithmic FLOP and byte counts of that launch.
struct ProfRec {
  hipEvent_t a, b;
  double flops, bytes;
  int reps;                       // launches between the two events (same work each)
};
}  // namespace

// Scratch memory of tdvp_lanczos_expm_noalloc: a fixed device array (one
// copy per GPU, held until the process ends), used in place of the
// context's workspace by callers that cannot allocate.  Host code never
// names it directly; its device address comes from hipGetSymbolAddress.
constexpr size_t TDVP_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[TDVP_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];   // device address of `scratch` on each device (null: not looked up)

// Look up the device address of `scratch` on `device` (current) once.
bool scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return false;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[device]) return true;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
  scratch_ptr[device] = p;
  return true;
}
void *scratch_of(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_ptr[device];
}
}  // namespace

struct tdvp_ctx {
  int device;
  hipStream_t stream;
  tdvp_precision prec;
  char *ws;
  size_t ws_bytes;
  int prof_class;                 // 0: timing off
  int prof_reps;                  // back-to-back repeats of a timed launch of a class that may repeat
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> pool;
  size_t pool_used;
  int32_t *klog;                  // device log of Krylov dimensions (may be null)
  int klog_cap, klog_pos;
  int graph_mode;                 // replay a captured step graph
  hipGraph_t graph;
  hipGraphExec_t gexec;
  std::vector<uint64_t> gkey;     // what the captured graph was built for
  int fused_off;                  // 1: never use the fused small-bond Lanczos step
  int s3_per_channel;             // 1: stage 3 of H x in one part per left MPO channel
  // autotuner: per problem key (kind, shapes, instance count, types) the
  // candidate that ran fastest when the key was first met outside a graph
  // capture; later launches (and captured graphs) reuse it
  int autotune;
  int tune_now;                   // predicated launches may be timed (a step that cannot be stopped)
  std::map<std::vector<int64_t>, int> tuned;
  hipEvent_t tune_ev[2];
  // second lane of the grouped ensemble step (default priority, created on
  // first use) and the events that fork it from and join it to `stream`
  hipStream_t aux;
  hipEvent_t fork_ev, join_ev;
  // lanes of the TDVP-MU site derivatives (default priority, created on
  // first use) and their fork / join events
  hipStream_t mu_lane[3] = {};
  hipEvent_t mu_ev[4] = {};
};

namespace {

#define CK(x)                                  \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return TDVP_E_DEVICE; \
  } while (0)

#define CS(x)                      \
  do {                             \
    tdvp_status s_ = (x);          \
    if (s_ != TDVP_OK) return s_;  \
  } while (0)

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

DType env_type(const tdvp_ctx *c) { return c->prec == TDVP_FP64 ? F64 : F32; }
int env_bytes(const tdvp_ctx *c) { return c->prec == TDVP_FP64 ? 16 : 8; }

// Workspace carve-up for a problem whose largest local vector has n complex
// entries and largest MPO bond is wmax.
struct Layout {
  size_t st, pp, U, T1, T2, Y, D, tmp, qr, obs, total;
  size_t ybytes;     // bytes of each of T1, T2, Y
  int64_t n;
};

Layout layout(int64_t n, int wmax, int kmax, int es) {
  Layout L;
  size_t o = 0;
  L.n = n;
  L.ybytes = (size_t)wmax * n * es;
  o += CTX_HEADER_BYTES;   // instance 0: the context header; others: unused
  L.st = o; o += al256(sizeof(LzState));
  L.pp = o; o += al256(sizeof(LzPartials));
  L.U = o; o += al256((size_t)(kmax + 1) * n * 16);
  L.T1 = o; o += al256((size_t)wmax * n * es);
  L.T2 = o; o += al256((size_t)wmax * n * es);
  L.Y = o; o += al256((size_t)wmax * n * es);
  L.D = o; o += al256((size_t)n * 16);
  L.tmp = o; o += al256((size_t)n * 16);
  L.qr = o; o += al256((size_t)10 * n * 16 + 16 * 1024);  // QR: Cholesky QR 3 m n + 6 n^2 + 16 complex, n^2 <= m n
  L.obs = o; o += al256((size_t)3 * n * 16 + 4096);
  L.total = o;
  return L;
}

template <typename T> T *at(tdvp_ctx *c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }
CtxHeader *header(tdvp_ctx *c) { return reinterpret_cast<CtxHeader *>(c->ws); }

hipEvent_t pool_event(tdvp_ctx *c) {
  if (c->pool_used == c->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->pool.push_back(e);
  }
  return c->pool[c->pool_used++];
}

// Start/stop a timed launch of class `cls` (no-op unless that class is profiled).
int prof_begin(tdvp_ctx *c, int cls) {
  if (c->prof_class != cls) return -1;
  ProfRec r{pool_event(c), pool_event(c), 0.0, 0.0, 1};
  if (!r.a || !r.b) return -1;
  hipEventRecord(r.a, c->stream);
  c->prof.push_back(r);
  return (int)c->prof.size() - 1;
}
// Timed launches of the classes whose launches may be repeated (they
// overwrite outputs they do not read: GEMM, MPO pass, fused Lanczos step)
// run prof_reps times back to back, so that the event interval measures the
// kernels rather than one dispatch each.
template <typename F> hipError_t timed_repeat(tdvp_ctx *c, int idx, F launch) {
  hipError_t e = launch();
  if (idx < 0) return e;
  for (int r = 1; r < c->prof_reps && e == hipSuccess; ++r) e = launch();
  c->prof[idx].reps = c->prof_reps;
  return e;
}
void prof_end(tdvp_ctx *c, int idx, double flops, double bytes) {
  if (idx < 0) return;
  hipEventRecord(c->prof[idx].b, c->stream);
  c->prof[idx].flops = flops;
  c->prof[idx].bytes = bytes;
}

int esz(DType t) { return t == F64 ? 16 : 8; }

// The contraction GEMMs (FP32 output) of the split-BF16 mode run on the bf16
// matrix cores; every other GEMM as requested.
hipError_t gemm_any(tdvp_ctx *c, DType ta, DType tb, DType tc, const GemmArgs &g) {
  if (c->prec == TDVP_BF16X3 && tc == F32) return cgemm_bf3(ta, tb, tc, g, c->stream);
  return cgemm(ta, tb, tc, g, c->stream);
}

// Autotuning: may the launch about to be issued be timed now?  Only outside
// a graph capture, and for a launch predicated on the Lanczos stop flag only
// where the caller has marked the step as one that cannot be stopped.
bool can_tune(tdvp_ctx *c, const void *skip) {
  if (!c->autotune || (skip && !c->tune_now)) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  for (hipEvent_t &e : c->tune_ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return false;
  return true;
}
// Average time of `launch` (one warm-up call, then reps timed calls) in ms;
// a failed launch returns a huge time so it is never chosen.
template <typename F> double time_launch(tdvp_ctx *c, F launch, int reps = 3) {
  if (launch() != hipSuccess) return 1e30;
  hipEventRecord(c->tune_ev[0], c->stream);
  for (int r = 0; r < reps; ++r)
    if (launch() != hipSuccess) return 1e30;
  hipEventRecord(c->tune_ev[1], c->stream);
  float ms = 0.f;
  if (hipEventSynchronize(c->tune_ev[1]) != hipSuccess ||
      hipEventElapsedTime(&ms, c->tune_ev[0], c->tune_ev[1]) != hipSuccess)
    return 1e30;
  return ms / reps;
}

// cgemm with timing: algorithmic FLOP 8 M N K per batch; bytes = operands once + output once.
// With the autotuner on, the tile shape (32x32, or 64x64 with K steps of 16,
// 32 or 64 in FP32) of a new problem key is chosen by timing each (a GEMM
// overwrites C, so repeats are harmless).
hipError_t gemm_t(tdvp_ctx *c, DType ta, DType tb, DType tc, const GemmArgs &g0,
                  int prof_cls = TDVP_PROF_GEMM) {
  GemmArgs g = g0;
  if (c->autotune) {
    const std::vector<int64_t> key = {0, ta, tb, tc, g.M, g.N, g.K, g.batch, g.inst.count,
                                      g.sak == 1, g.sbn == 1, g.scn == 1, (int64_t)c->prec,
                                      g.lzU != nullptr};
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
      g.tile = it->second;
    } else if (can_tune(c, g.skip)) {
      // the built-in choice stays unless another shape is clearly faster
      // (timings of small GEMMs carry launch noise)
      const int64_t tiles64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
      const int def = tiles64 >= 240 ? 64 : 32;
      g.tile = def;
      const double tdef = time_launch(c, [&] { return gemm_any(c, ta, tb, tc, g); }, 5);
      int best = def;
      double tbest = tdef;
      for (int cand : {32, 64, 96, 128}) {
        if (cand == def || (cand > 64 && (tc != F32 || c->prec == TDVP_BF16X3))) continue;   // FP32 only
        g.tile = cand;
        const double t = time_launch(c, [&] { return gemm_any(c, ta, tb, tc, g); }, 5);
        if (t < 0.97 * tdef && t < tbest) { tbest = t; best = cand; }
      }
      c->tuned[key] = best;
      g.tile = best;
    }
  }
  const int id = prof_begin(c, prof_cls);
  const hipError_t e = timed_repeat(c, id, [&] { return gemm_any(c, ta, tb, tc, g); });
  // every instance of a batched launch does the work of one
  const double M = g.M, N = g.N, K = g.K, B = g.batch, R = g.inst.count;
  prof_end(c, id, 8.0 * M * N * K * B * R,
           R * ((g.bsa ? B : 1.0) * M * K * esz(ta) + (g.bsb ? B : 1.0) * K * N * esz(tb) + B * M * N * esz(tc)));
  return e;
}

hipError_t wapply_t(tdvp_ctx *c, DType t, const WApplyArgs &a) {
  const int id = prof_begin(c, TDVP_PROF_WAPPLY);
  const hipError_t e = timed_repeat(c, id, [&] { return wapply(t, a, c->stream); });
  const double io = (double)a.A * a.C * a.d * esz(t) * a.inst.count;
  prof_end(c, id, 0.0, io * (a.Wl + a.Wr));
  return e;
}

// Instances handled together (identical shapes): count, and the stride of
// each instance's workspace slice in bytes.  A single problem is count = 1.
struct Bi {
  int R = 1;
  int64_t ws = 0;
  int64_t wsel(int es) const { return ws / es; }   // workspace stride in elements of size es
  int64_t wsint() const { return ws / 4; }
};

Inst inst_of(const Bi &b, int64_t sa, int64_t sb, int64_t sc, int64_t sskip) {
  Inst in;
  in.count = b.R;
  in.a = sa; in.b = sb; in.c = sc; in.skip = sskip;
  return in;
}

// One linear operator of a local equation: H[i] (W != NULL) or the bond
// operator K of eq:tdvp2_D (W == NULL, d == 1, Wl == Wr).  sL, sW, sR are
// the instance strides (elements) of the two environments and of W.
struct Op {
  const void *L, *W, *R;
  int Ml, d, Mr, Wl, Wr;
  int64_t sL = 0, sW = 0, sR = 0;
  int P = 0;   // partial outputs of the stage-3 GEMM (a divisor of Wl; 0: Wl)
  int64_t size() const { return (int64_t)Ml * d * Mr; }
  int parts() const { return P > 0 ? P : Wl; }
};

// Partial outputs of Op x for a batch of R instances.  Stage 3 sums over
// the pairs (wl, l), K = Wl Ml; it is split into P equal runs of whole wl
// blocks, each run a GEMM of its own whose output is one part.  Every part
// is one more vector for the projections to read, and one part lets the
// GEMM take the projections into its epilogue, so a batch of 8 or more
// instances runs it unsplit (on the disorder ensemble's 15 x M = 32 and
// 12 x M = 64 classes this measured 3 % faster overall than splitting them
// to fill the chip); otherwise P is the smallest divisor of Wl that gives
// about four 32 x 32 output tiles per compute unit (1024 in all).
int stage3_parts(const Op &op, int R, int per_channel) {
  if (per_channel) return op.Wl;
  if (R >= 8) return 1;
  const int64_t tiles = (int64_t)((op.Ml + 31) / 32) * ((op.d * op.Mr + 31) / 32) * R;
  for (int p = 1; p < op.Wl; ++p)
    if (op.Wl % p == 0 && tiles * p >= 1024) return p;
  return op.Wl;
}

// The launches of Op x (stage-1 GEMM, MPO pass, stage-3 GEMM; the bond
// operator has no MPO pass) for the instances b with workspace base `base`:
// y_parts[p] (p < Wl) in the Y buffer with sum_p y_parts[p] = Op x.  x is
// c128 with instance stride sx.
struct OpLaunch {
  GemmArgs g1, g3;
  WApplyArgs w;
  bool has_w;
};

OpLaunch op_args(const tdvp_ctx *c, char *base, const Layout &lay, const Op &op, const double2 *x,
                 int64_t sx, const int *skip, const Bi &b) {
  const int es = env_bytes(c);
  const int64_t n = op.size();
  void *T1 = base + lay.T1, *T2 = base + lay.T2, *Y = base + lay.Y;
  const int64_t wse = b.wsel(es), wsk = skip ? b.wsint() : 0;
  OpLaunch L{};
  L.has_w = op.W != nullptr;
  if (op.W) {
    // stage 1: T1[wr][l s][r'] = sum_r x[l s][r] R[r'][wr][r]
    GemmArgs &g = L.g1;
    g.A = x; g.B = op.R; g.C = T1;
    g.M = op.Ml * op.d; g.N = op.Mr; g.K = op.Mr; g.batch = op.Wr;
    g.sam = op.Mr; g.sak = 1; g.sbk = 1; g.sbn = (int64_t)op.Wr * op.Mr;
    g.scm = op.Mr; g.scn = 1;
    g.bsa = 0; g.bsb = op.Mr; g.bsc = n;
    g.skip = skip;
    g.inst = inst_of(b, sx, op.sR, wse, wsk);
    // stage 2: T2[wl][l][s'][r'] = sum_{s, wr} W[wl][s'][s][wr] T1[wr][l][s][r']
    WApplyArgs &w = L.w;
    w.in = T1; w.out = T2; w.W = op.W;
    w.Wl = op.Wl; w.Wr = op.Wr; w.d = op.d; w.A = op.Ml; w.C = op.Mr;
    w.w_in_right = 1;
    w.si_w = n; w.si_s = op.Mr; w.si_a = (int64_t)op.d * op.Mr; w.si_c = 1;
    w.so_w = n; w.so_s = op.Mr; w.so_a = (int64_t)op.d * op.Mr; w.so_c = 1;
    w.skip = skip;
    w.inst = inst_of(b, wse, op.sW, wse, wsk);
    // stage 3: Y[p][l'][s' r'] = sum_{(wl, l) in run p} L[l'][wl][l] T2[wl][l][s' r']
    // (K = (Wl / P) Ml per part; the pairs (wl, l) are contiguous in both operands)
    GemmArgs &h = L.g3;
    const int64_t kc = (int64_t)(op.Wl / op.parts()) * op.Ml;
    h.A = op.L; h.B = T2; h.C = Y;
    h.M = op.Ml; h.N = op.d * op.Mr; h.K = (int)kc; h.batch = op.parts();
    h.sam = (int64_t)op.Wl * op.Ml; h.sak = 1; h.sbk = (int64_t)op.d * op.Mr; h.sbn = 1;
    h.scm = (int64_t)op.d * op.Mr; h.scn = 1;
    h.bsa = kc; h.bsb = kc * h.sbk; h.bsc = n;
    h.skip = skip;
    h.inst = inst_of(b, op.sL, wse, wse, wsk);
  } else {
    // bond operator: T1[w][l][r'] = sum_r D[l][r] R[r'][w][r]; Y[w][l'][r'] = sum_l L[l'][w][l] T1[w][l][r']
    GemmArgs &g = L.g1;
    g.A = x; g.B = op.R; g.C = T1;
    g.M = op.Ml; g.N = op.Mr; g.K = op.Mr; g.batch = op.Wr;
    g.sam = op.Mr; g.sak = 1; g.sbk = 1; g.sbn = (int64_t)op.Wr * op.Mr;
    g.scm = op.Mr; g.scn = 1;
    g.bsa = 0; g.bsb = op.Mr; g.bsc = n;
    g.skip = skip;
    g.inst = inst_of(b, sx, op.sR, wse, wsk);
    GemmArgs &h = L.g3;
    const int64_t kc = (int64_t)(op.Wl / op.parts()) * op.Ml;
    h.A = op.L; h.B = T1; h.C = Y;
    h.M = op.Ml; h.N = op.Mr; h.K = (int)kc; h.batch = op.parts();
    h.sam = (int64_t)op.Wl * op.Ml; h.sak = 1; h.sbk = op.Mr; h.sbn = 1;
    h.scm = op.Mr; h.scn = 1;
    h.bsa = kc; h.bsb = kc * h.sbk; h.bsc = n;
    h.skip = skip;
    h.inst = inst_of(b, op.sL, wse, wse, wsk);
  }
  return L;
}

// y_parts[p] (p < Wl) with sum_p y_parts[p] = Op x.  x is c128 with instance stride sx.
// With lzU set (a Krylov step of run_lanczos whose stage 3 runs in one
// part): stage 3 writes H x to basis vector lzj + 1 instead, with the
// projection partials (GEMM epilogue).
tdvp_status apply_op(tdvp_ctx *c, const Layout &lay, const Op &op, const double2 *x, int64_t sx,
                     const int *skip, const Bi &b, double2 *lzU = nullptr, LzPartials *lzpp = nullptr,
                     int lzj = 0) {
  const DType et = env_type(c), ct = et;
  OpLaunch L = op_args(c, c->ws, lay, op, x, sx, skip, b);
  if (lzU) {
    L.g3.lzU = lzU;
    L.g3.lzpp = lzpp;
    L.g3.lzj = lzj;
    L.g3.lzwss = b.ws;
  }
  CK(gemm_t(c, F64, et, ct, L.g1, TDVP_PROF_GEMM_HEFF));
  if (L.has_w) CK(wapply_t(c, ct, L.w));
  CK(gemm_t(c, et, ct, ct, L.g3, TDVP_PROF_GEMM_HEFF));
  return TDVP_OK;
}

// May the Krylov steps of `op` (stage 3 in P parts) take the projection
// epilogue: one part, not split-BF16 (its GEMM has no epilogue), and few
// enough output tiles for one partial each.
bool lz_epilogue_ok(const tdvp_ctx *c, const Op &op) {
  return op.parts() == 1 && c->prec != TDVP_BF16X3 &&
         (int64_t)((op.Ml + 31) / 32) * ((op.d * op.Mr + 31) / 32) <= LZ_PARTS;
}

// Arguments of the fused Lanczos step (heff_small) for Op, if it applies:
// its tiles fit in LDS, the nonzero table of W fits in the Y buffer and the
// P partial vectors in the T1 buffer (both unused on this path).  The sum
// over the bra index l is split into P parts so that Mr P work-groups per
// instance cover the chip.  Fills everything except st, pp, U, j.
// Measured on the 77-site chain: the fused step wins up to bond dimension
// 64 (FP64 and FP32); at 128 the tiled GEMM path is faster, for H[i] and for
// the bond operator alike.  A batch whose output columns (Mr per instance)
// already number 256 or more fills the chip with the general path's tiles:
// on the disorder ensemble (FP32) the general path took 0.86x the kernel
// time of the fused step for 15 instances of M = 32 and 0.54x for 12 of
// M = 64.
constexpr int FUSED_MAX_MR = 64;
constexpr int FUSED_MAX_MR_BOND = 64;
constexpr int FUSED_MAX_COLS = 256;

bool fused_args(const tdvp_ctx *c, const Layout &lay, const Op &op, const Bi &b, HeffSmallArgs &a,
                char *base = nullptr) {
  if (!base) base = c->ws;
  if (c->fused_off || op.Mr > (op.W ? FUSED_MAX_MR : FUSED_MAX_MR_BOND)) return false;
  if ((int64_t)op.Mr * b.R >= FUSED_MAX_COLS) return false;
  if (!op.W && (op.Wl != op.Wr || op.d != 1)) return false;
  a = HeffSmallArgs{};
  a.L = op.L; a.R = op.R;
  a.Ml = op.Ml; a.d = op.d; a.Mr = op.Mr; a.Wl = op.Wl; a.Wr = op.Wr;
  a.n = op.size();
  a.Gprev = lz_grid(a.n, b.R);
  a.Gw = lz_grid(a.n, b.R);
  a.wss = b.ws; a.sL = op.sL; a.sR = op.sR;
  // P is chosen so that all instances together cover the chip: one chain
  // gets up to 8 parts per column, a large batch 1 (each part adds
  // redundant reads of the basis columns, so a batch that already fills
  // the chip runs faster unsplit)
  const int64_t cols = (int64_t)op.Mr * b.R;
  int P = (int)std::min<int64_t>(HS_PMAX, std::max<int64_t>(1, (256 + cols - 1) / cols));
  P = std::min(P, std::max(1, op.Ml / 4));
  while (P > 1 && ((int64_t)P * op.Mr > LZ_PARTS || (size_t)P * a.n * 16 > lay.ybytes)) --P;
  a.nl = (op.Ml + P - 1) / P;
  a.P = (op.Ml + a.nl - 1) / a.nl;
  if ((size_t)a.P * a.n * 16 > lay.ybytes) return false;
  a.staged = 1;
  if (!heff_small_fits(a, env_bytes(c) / 2)) {
    a.staged = 0;
    if (!heff_small_fits(a, env_bytes(c) / 2)) return false;
  }
  a.Yp = reinterpret_cast<double2 *>(base + lay.T1);
  if (op.W) {
    const size_t rows = (size_t)op.Wl * op.d, cap = (size_t)op.d * op.Wr;
    const size_t o_col = al256((rows + 1) * 4), o_coef = o_col + al256(rows * cap * 4);
    if (o_coef + rows * cap * 16 > lay.ybytes) return false;
    char *tb = base + lay.Y;
    a.row = reinterpret_cast<const int *>(tb);
    a.col = reinterpret_cast<const int *>(tb + o_col);
    a.coef = reinterpret_cast<const double2 *>(tb + o_coef);
  }
  return true;
}

// y = exp(z Op) x for every instance; x, y c128 with instance strides sx, sy.
tdvp_status run_lanczos(tdvp_ctx *c, const Layout &lay, const Op &op_in, double zr, double zi,
                        int kmax, double tol, const void *x, int64_t sx, void *y, int64_t sy,
                        int32_t *kused, const Bi &b) {
  Op op = op_in;
  op.P = stage3_parts(op, b.R, c->s3_per_channel);
  const int64_t n = op.size();
  const int keff = (int)std::min<int64_t>(kmax, n);
  LzState *st = at<LzState>(c, lay.st);
  LzPartials *pp = at<LzPartials>(c, lay.pp);
  double2 *U = at<double2>(c, lay.U);
  LzInst li;
  li.count = b.R; li.wss = b.ws; li.xs = sx; li.ys = sy;
  const double vb = 16.0 * n * b.R;
  HeffSmallArgs fa;
  const bool fused = fused_args(c, lay, op, b, fa);
  const bool epi = !fused && lz_epilogue_ok(c, op);
  const int trows = fused ? op.Ml * op.d : 0;
  if (fused && op.W)
    CK(wtable((const double2 *)op.W, op.Wl, op.d, op.Wr, op.sW, const_cast<int *>(fa.row),
              const_cast<int *>(fa.col), const_cast<double2 *>(fa.coef), b.ws, b.R, c->stream));
  int id = prof_begin(c, TDVP_PROF_LZ_ENDS);
  CK(lz_start(st, pp, (const double2 *)x, U, n, zr, zi, tol, keff, trows, &header(c)->nonfinite, li,
              c->stream));
  prof_end(c, id, 4.0 * n * b.R, 2.0 * vb);
  fa.st = st; fa.pp = pp; fa.U = U;
  for (int j = 0; j < keff; ++j) {
    if (fused) {
      // algorithmic work: the three contraction stages and j+1 projections;
      // bytes: u_j, both environments, W, H u_j, and u_0..u_j once
      const double Ml = op.Ml, d = op.d, Mr = op.Mr, Wl = op.Wl, Wr = op.Wr;
      const double fl = 8.0 * (Ml * d * Mr * Wr * Mr + Wl * Ml * Ml * d * Mr) + 8.0 * (j + 1) * n;
      const double by = (Ml * Wl * Ml + Mr * Wr * Mr) * env_bytes(c) +
                        (op.W ? Wl * d * d * Wr * 16.0 : 0.0);
      id = prof_begin(c, TDVP_PROF_LZ_FUSED);
      fa.j = j;
      CK(timed_repeat(c, id, [&] { return heff_small(env_type(c), fa, b.R, c->stream); }));
      prof_end(c, id, fl * b.R, by * b.R + (j + 2) * vb);
      id = prof_begin(c, TDVP_PROF_LZ_UPDATE);
      CK(lz_update(st, pp, U, n, j, n, op.Mr * fa.P, fa.Yp, fa.P, li, c->stream));
      prof_end(c, id, 8.0 * (j + 1) * n * b.R, 2.0 * vb + (j + 1) * vb);
      continue;
    }
    c->tune_now = j == 0;   // the first Krylov step is never stopped
    if (epi) {
      // stage 3 writes H u_j to U[j+1] with the projection partials; the
      // update kernel closes step j - 1 itself
      const tdvp_status so = apply_op(c, lay, op, U + (int64_t)j * n, b.wsel(16), &st->stop, b, U, pp, j);
      c->tune_now = 0;
      CS(so);
      id = prof_begin(c, TDVP_PROF_LZ_UPDATE);
      CK(lz_update(st, pp, U, n, j, n, -1, nullptr, 0, li, c->stream, 1));
      prof_end(c, id, 8.0 * (j + 1) * n * b.R, 2.0 * vb + (j + 1) * vb);
      continue;
    }
    const tdvp_status so = apply_op(c, lay, op, U + (int64_t)j * n, b.wsel(16), &st->stop, b);
    c->tune_now = 0;
    CS(so);
    id = prof_begin(c, TDVP_PROF_LZ_DOTS);
    CK(lz_dots(st, pp, env_type(c), c->ws + lay.Y, op.parts(), n, U, n, j, n, li, c->stream));
    prof_end(c, id, 8.0 * (j + 1) * n * b.R,
             (double)op.parts() * n * env_bytes(c) * b.R + vb + (j + 1) * vb);
    id = prof_begin(c, TDVP_PROF_LZ_UPDATE);
    CK(lz_update(st, pp, U, n, j, n, 0, nullptr, 0, li, c->stream));
    prof_end(c, id, 8.0 * (j + 1) * n * b.R, 2.0 * vb + (j + 1) * vb);
  }
  if (!kused && c->klog && c->klog_pos + b.R <= c->klog_cap) {
    kused = c->klog + c->klog_pos;
    c->klog_pos += b.R;
  }
  id = prof_begin(c, TDVP_PROF_LZ_ENDS);
  CK(lz_finish(st, U, n, n, keff, (double2 *)y, kused, trows, li, c->stream));
  prof_end(c, id, 8.0 * keff * n * b.R, keff * vb + vb);
  return TDVP_OK;
}

// dir = +1: out (Mr, Wr, Mr) = h[1:i] from in (Ml, Wl, Ml).  dir = -1: out (Ml, Wl, Ml) from in (Mr, Wr, Mr).
// Instance strides (elements): sin, sout (environments), sA (site tensor), sW (MPO).
tdvp_status env_update(tdvp_ctx *c, const Layout &lay, int dir, const void *in, const void *A,
                       const void *W, int Ml, int d, int Mr, int Wl, int Wr, void *out,
                       const Bi &b, int64_t sin, int64_t sA, int64_t sW, int64_t sout) {
  const DType et = env_type(c), ct = et;
  const int64_t n = (int64_t)Ml * d * Mr;
  const int64_t wse = b.wsel(env_bytes(c));
  void *T1 = c->ws + lay.T1, *T2 = c->ws + lay.T2;
  if (dir > 0) {
    // T1[l'][wl][s][li] = sum_l L[l'][wl][l] A[l][s][li]
    GemmArgs g{};
    g.A = in; g.B = A; g.C = T1;
    g.M = Ml * Wl; g.N = d * Mr; g.K = Ml; g.batch = 1;
    g.sam = Ml; g.sak = 1; g.sbk = (int64_t)d * Mr; g.sbn = 1; g.scm = (int64_t)d * Mr; g.scn = 1;
    g.inst = inst_of(b, sin, sA, wse, 0);
    CK(gemm_t(c, et, F64, ct, g));
    // T2[l'][s'][wr][li] = sum_{wl, s} W[wl][s'][s][wr] T1[l'][wl][s][li]
    WApplyArgs w{};
    w.in = T1; w.out = T2; w.W = W;
    w.Wl = Wl; w.Wr = Wr; w.d = d; w.A = Ml; w.C = Mr; w.w_in_right = 0;
    w.si_w = (int64_t)d * Mr; w.si_s = Mr; w.si_a = (int64_t)Wl * d * Mr; w.si_c = 1;
    w.so_w = Mr; w.so_s = (int64_t)Wr * Mr; w.so_a = (int64_t)d * Wr * Mr; w.so_c = 1;
    w.inst = inst_of(b, wse, sW, wse, 0);
    CK(wapply_t(c, ct, w));
    // out[q][wr][li] = sum_{l', s'} conj(A[l'][s'][q]) T2[l'][s'][wr][li]
    GemmArgs h{};
    h.A = A; h.B = T2; h.C = out;
    h.M = Mr; h.N = Wr * Mr; h.K = Ml * d; h.batch = 1;
    h.sam = 1; h.sak = Mr; h.conjA = 1; h.sbk = (int64_t)Wr * Mr; h.sbn = 1;
    h.scm = (int64_t)Wr * Mr; h.scn = 1;
    h.inst = inst_of(b, sA, wse, sout, 0);
    CK(gemm_t(c, F64, ct, et, h));
  } else {
    // T1[wr][k][t][q] = sum_r A[k][t][r] R[q][wr][r]   (as stage 1 of H[i] x)
    GemmArgs g{};
    g.A = A; g.B = in; g.C = T1;
    g.M = Ml * d; g.N = Mr; g.K = Mr; g.batch = Wr;
    g.sam = Mr; g.sak = 1; g.sbk = 1; g.sbn = (int64_t)Wr * Mr;
    g.scm = Mr; g.scn = 1; g.bsa = 0; g.bsb = Mr; g.bsc = n;
    g.inst = inst_of(b, sA, sin, wse, 0);
    CK(gemm_t(c, F64, et, ct, g));
    // T2[wl][k][s][q] = sum_{t, wr} W[wl][s][t][wr] T1[wr][k][t][q]
    WApplyArgs w{};
    w.in = T1; w.out = T2; w.W = W;
    w.Wl = Wl; w.Wr = Wr; w.d = d; w.A = Ml; w.C = Mr; w.w_in_right = 1;
    w.si_w = n; w.si_s = Mr; w.si_a = (int64_t)d * Mr; w.si_c = 1;
    w.so_w = n; w.so_s = Mr; w.so_a = (int64_t)d * Mr; w.so_c = 1;
    w.inst = inst_of(b, wse, sW, wse, 0);
    CK(wapply_t(c, ct, w));
    // out[b][wl][k] = sum_{s, q} conj(A[b][s][q]) T2[wl][k][s][q]
    GemmArgs h{};
    h.A = A; h.B = T2; h.C = out;
    h.M = Ml; h.N = Wl * Ml; h.K = d * Mr; h.batch = 1;
    h.sam = (int64_t)d * Mr; h.sak = 1; h.conjA = 1; h.sbk = 1; h.sbn = (int64_t)d * Mr;
    h.scm = (int64_t)Wl * Ml; h.scn = 1;
    h.inst = inst_of(b, sA, wse, sout, 0);
    CK(gemm_t(c, F64, ct, et, h));
  }
  return TDVP_OK;
}

// Householder QR of an m x n complex matrix plus forming the thin Q:
// 2 (4 m n^2 - 4 n^3 / 3) complex-equivalent real FLOP (factor + Q).
double qr_flops(double m, double n) { return 2.0 * 8.0 * (m * n * n - n * n * n / 3.0); }

tdvp_status run_qr(tdvp_ctx *c, QrArgs &q) {
  const int id = prof_begin(c, TDVP_PROF_QR);
  CK(qr(q, c->stream));
  prof_end(c, id, qr_flops(q.m, q.n) * q.inst.count,
           16.0 * (2.0 * q.m * q.n + (double)q.n * q.n) * q.inst.count);
  return TDVP_OK;
}

// Left-to-right gauge: C (Ml d x Mr, row-major) = Q D; Q written back to C.
// sC: instance stride of C; D lives in the workspace.
tdvp_status qr_left(tdvp_ctx *c, const Layout &lay, double2 *C, int Ml, int d, int Mr, double2 *D,
                    const Bi &b, int64_t sC) {
  QrArgs q{};
  q.A = C; q.a_rs = Mr; q.a_cs = 1;
  q.Q = C; q.q_rs = Mr; q.q_cs = 1;
  q.R = D; q.r_rs = Mr; q.r_cs = 1;
  q.m = Ml * d; q.n = Mr;
  q.work = at<double2>(c, lay.qr);
  q.inst = inst_of(b, sC, sC, b.wsel(16), b.wsel(16));
  return run_qr(c, q);
}

// Right-to-left gauge: C (Ml x d Mr) = D Rt with Rt right-isometric (written
// back to C) and D = R^H from the QR of C^H.
tdvp_status qr_right(tdvp_ctx *c, const Layout &lay, double2 *C, int Ml, int d, int Mr, double2 *D,
                     const Bi &b, int64_t sC) {
  const int64_t cols = (int64_t)d * Mr;
  QrArgs q{};
  q.A = C; q.a_rs = 1; q.a_cs = cols; q.conjA = 1;
  q.Q = C; q.q_rs = 1; q.q_cs = cols; q.conjQ = 1;
  q.R = D; q.r_rs = 1; q.r_cs = Ml; q.conjR = 1;
  q.m = (int)cols; q.n = Ml;
  q.work = at<double2>(c, lay.qr);
  q.inst = inst_of(b, sC, sC, b.wsel(16), b.wsel(16));
  return run_qr(c, q);
}

// out (m x nn) = A (m x k) B (k x nn), all c128 row-major; instance strides sa, sb, so.
tdvp_status matmul(tdvp_ctx *c, const double2 *A, const double2 *B, double2 *out, int m, int k, int nn,
                   const Bi &b = Bi(), int64_t sa = 0, int64_t sb = 0, int64_t so = 0) {
  GemmArgs g{};
  g.A = A; g.B = B; g.C = out;
  g.M = m; g.N = nn; g.K = k; g.batch = 1;
  g.sam = k; g.sak = 1; g.sbk = nn; g.sbn = 1; g.scm = nn; g.scn = 1;
  g.inst = inst_of(b, sa, sb, so, 0);
  CK(gemm_t(c, F64, F64, F64, g));
  return TDVP_OK;
}

struct Chain {
  int n;
  std::vector<int> phys, bond, wbond;
  int64_t nmax;
  int wmax, mmax;
};

tdvp_status check_chain(const tdvp_mps *mps, const tdvp_mpo *mpo, Chain *ch) {
  if (!mps || !mps->phys || !mps->bond || !mps->site || mps->n <= 0) return TDVP_E_ARG;
  const int n = mps->n;
  ch->n = n;
  ch->phys.assign(mps->phys, mps->phys + n);
  ch->bond.assign(mps->bond, mps->bond + n + 1);
  if (ch->bond[0] != 1 || ch->bond[n] != 1) return TDVP_E_SHAPE;
  ch->nmax = 1;
  ch->mmax = 1;
  for (int i = 0; i < n; ++i) {
    if (ch->phys[i] < 1 || ch->bond[i] < 1 || !mps->site[i]) return TDVP_E_SHAPE;
    ch->nmax = std::max<int64_t>(ch->nmax, (int64_t)ch->bond[i] * ch->phys[i] * ch->bond[i + 1]);
    ch->nmax = std::max<int64_t>(ch->nmax, (int64_t)ch->bond[i] * ch->bond[i]);
    ch->mmax = std::max(ch->mmax, ch->bond[i]);
    // QR shapes of both sweep directions must be tall
    if (i < n - 1 && (int64_t)ch->bond[i] * ch->phys[i] < ch->bond[i + 1]) return TDVP_E_SHAPE;
    if (i > 0 && (int64_t)ch->phys[i] * ch->bond[i + 1] < ch->bond[i]) return TDVP_E_SHAPE;
  }
  if (ch->mmax > 256) return TDVP_E_UNSUPPORTED;
  ch->wmax = 1;
  if (mpo) {
    if (mpo->n != n || !mpo->phys || !mpo->bond || !mpo->site) return TDVP_E_ARG;
    ch->wbond.assign(mpo->bond, mpo->bond + n + 1);
    if (ch->wbond[0] != 1 || ch->wbond[n] != 1) return TDVP_E_SHAPE;
    for (int i = 0; i < n; ++i) {
      if (mpo->phys[i] != ch->phys[i] || !mpo->site[i] || ch->wbond[i] < 1) return TDVP_E_SHAPE;
      ch->wmax = std::max(ch->wmax, ch->wbond[i]);
      if ((int64_t)ch->wbond[i + 1] * ch->phys[i] > 1024 || (int64_t)ch->wbond[i] * ch->phys[i] > 1024)
        return TDVP_E_UNSUPPORTED;
    }
  }
  return TDVP_OK;
}

tdvp_status need(const tdvp_ctx *c, const Layout &lay) {
  if (!c->ws) return TDVP_E_WORKSPACE;
  if (c->ws_bytes < lay.total) return TDVP_E_WORKSPACE;
  return TDVP_OK;
}



}  // namespace

extern "C" {

const char *tdvp_status_string(tdvp_status s) {
  switch (s) {
    case TDVP_OK: return "ok";
    case TDVP_E_ARG: return "invalid argument";
    case TDVP_E_SHAPE: return "inconsistent shapes";
    case TDVP_E_DEVICE: return "HIP runtime error";
    case TDVP_E_WORKSPACE: return "workspace missing or too small";
    case TDVP_E_NUMERIC: return "non-finite value";
    case TDVP_E_UNSUPPORTED: return "size beyond compiled limits";
  }
  return "unknown status";
}

tdvp_status tdvp_create(tdvp_ctx **ctx, int device, void *hip_stream, tdvp_precision prec) {
  if (!ctx) return TDVP_E_ARG;
  if (prec != TDVP_FP64 && prec != TDVP_FP32 && prec != TDVP_BF16X3) return TDVP_E_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TDVP_E_DEVICE;
  tdvp_ctx *c = new (std::nothrow) tdvp_ctx;
  if (!c) return TDVP_E_DEVICE;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->prec = prec;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->prof_class = 0;
  c->prof_reps = 1;
  c->pool_used = 0;
  c->klog = nullptr;
  c->klog_cap = 0;
  c->klog_pos = 0;
  c->graph_mode = 0;
  c->fused_off = 0;
  c->s3_per_channel = 0;
  c->autotune = 0;
  c->tune_now = 0;
  c->tune_ev[0] = c->tune_ev[1] = nullptr;
  c->graph = nullptr;
  c->gexec = nullptr;
  c->aux = nullptr;
  c->fork_ev = c->join_ev = nullptr;
  if (hipSetDevice(device) != hipSuccess) { delete c; return TDVP_E_DEVICE; }
  static const bool inited = (qr_init(), true);   // once per process (thread-safe static)
  (void)inited;
  // device address of the no-allocation scratch array on this device (once
  // per device); a failure only disables tdvp_lanczos_expm_noalloc
  (void)scratch_init(device);
  *ctx = c;
  return TDVP_OK;
}

tdvp_status tdvp_destroy(tdvp_ctx *ctx) {
  if (!ctx) return TDVP_E_ARG;
  for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
  for (hipEvent_t e : ctx->tune_ev)
    if (e) hipEventDestroy(e);
  if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) hipGraphDestroy(ctx->graph);
  if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) hipEventDestroy(ctx->join_ev);
  if (ctx->aux) hipStreamDestroy(ctx->aux);
  for (hipStream_t l : ctx->mu_lane)
    if (l) hipStreamDestroy(l);
  for (hipEvent_t e : ctx->mu_ev)
    if (e) hipEventDestroy(e);
  delete ctx;
  return TDVP_OK;
}

tdvp_status tdvp_set_stream(tdvp_ctx *ctx, void *hip_stream) {
  if (!ctx) return TDVP_E_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return TDVP_OK;
}

int tdvp_env_elem_bytes(const tdvp_ctx *ctx) { return ctx ? env_bytes(ctx) : 0; }

tdvp_status tdvp_set_krylov_log(tdvp_ctx *ctx, int32_t *dev, int capacity) {
  if (!ctx || capacity < 0 || (capacity > 0 && !dev)) return TDVP_E_ARG;
  ctx->klog = capacity > 0 ? dev : nullptr;
  ctx->klog_cap = capacity;
  ctx->klog_pos = 0;
  return TDVP_OK;
}

tdvp_status tdvp_profile(tdvp_ctx *ctx, int kernel_class) {
  if (!ctx || kernel_class < 0 || kernel_class > TDVP_PROF_GEMM_HEFF) return TDVP_E_ARG;
  ctx->prof_class = kernel_class;
  ctx->prof.clear();
  ctx->pool_used = 0;
  return TDVP_OK;
}

tdvp_status tdvp_profile_reps(tdvp_ctx *ctx, int reps) {
  if (!ctx || reps < 1 || reps > 64) return TDVP_E_ARG;
  ctx->prof_reps = reps;
  return TDVP_OK;
}

tdvp_status tdvp_profile_read(tdvp_ctx *ctx, double *ms, int64_t *launches, double *flops, double *bytes) {
  if (!ctx || !ms || !launches || !flops || !bytes) return TDVP_E_ARG;
  CK(hipStreamSynchronize(ctx->stream));
  double t = 0.0, f = 0.0, b = 0.0;
  for (const ProfRec &r : ctx->prof) {
    float e = 0.0f;
    CK(hipEventElapsedTime(&e, r.a, r.b));
    t += e / r.reps;
    f += r.flops;
    b += r.bytes;
  }
  *ms = t;
  *launches = (int64_t)ctx->prof.size();
  *flops = f;
  *bytes = b;
  return TDVP_OK;
}

tdvp_status tdvp_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 int kmax, size_t *bytes) {
  if (!ctx || !bytes || kmax < 1 || kmax > KMAX) return TDVP_E_ARG;
  Chain ch;
  CS(check_chain(mps, mpo, &ch));
  *bytes = layout(ch.nmax, ch.wmax, kmax, env_bytes(ctx)).total;
  return TDVP_OK;
}

tdvp_status tdvp_set_workspace(tdvp_ctx *ctx, void *dev, size_t bytes) {
  if (!ctx || !dev) return TDVP_E_ARG;
  if (((uintptr_t)dev & 255) != 0) return TDVP_E_ARG;
  if (bytes < CTX_HEADER_BYTES + al256(sizeof(LzState))) return TDVP_E_WORKSPACE;
  ctx->ws = (char *)dev;
  ctx->ws_bytes = bytes;
  CK(hipSetDevice(ctx->device));
  CK(hipMemsetAsync(ctx->ws, 0, CTX_HEADER_BYTES, ctx->stream));
  CK(set_dev_int(&reinterpret_cast<LzState *>(ctx->ws + CTX_HEADER_BYTES)->stop, 1, ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_env_update(tdvp_ctx *ctx, int dir, const void *env_in, const void *A, const void *W,
                            int Ml, int d, int Mr, int Wl, int Wr, void *env_out) {
  if (!ctx || !env_in || !A || !W || !env_out || (dir != 1 && dir != -1)) return TDVP_E_ARG;
  if (Ml < 1 || d < 1 || Mr < 1 || Wl < 1 || Wr < 1) return TDVP_E_SHAPE;
  if ((int64_t)std::max(Wl, Wr) * d > 1024) return TDVP_E_UNSUPPORTED;
  const Layout lay = layout((int64_t)Ml * d * Mr, std::max(Wl, Wr), 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  return env_update(ctx, lay, dir, env_in, A, W, Ml, d, Mr, Wl, Wr, env_out, Bi(), 0, 0, 0, 0);
}

tdvp_status tdvp_heff_apply(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv, int Ml,
                            int d, int Mr, int Wl, int Wr, const void *x, void *y) {
  if (!ctx || !Lenv || !Renv || !x || !y) return TDVP_E_ARG;
  if (Ml < 1 || d < 1 || Mr < 1 || Wl < 1 || Wr < 1) return TDVP_E_SHAPE;
  if (!W && (d != 1 || Wl != Wr)) return TDVP_E_SHAPE;
  if ((int64_t)std::max(Wl, Wr) * d > 1024) return TDVP_E_UNSUPPORTED;
  const Op op{Lenv, W, Renv, Ml, d, Mr, Wl, Wr};
  const Layout lay = layout(op.size(), std::max(Wl, Wr), 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  CS(apply_op(ctx, lay, op, (const double2 *)x, 0, nullptr, Bi()));
  CK(sum_partials(env_type(ctx), ctx->ws + lay.Y, op.parts(), op.size(), op.size(), (double2 *)y,
                  ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_lanczos_expm(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv, int Ml,
                              int d, int Mr, int Wl, int Wr, double z_re, double z_im, int kmax,
                              double tol, const void *x, void *y, int32_t *k_used_dev) {
  if (!ctx || !Lenv || !Renv || !x || !y) return TDVP_E_ARG;
  if (kmax < 1 || kmax > KMAX || !(tol >= 0.0)) return TDVP_E_ARG;
  if (Ml < 1 || d < 1 || Mr < 1 || Wl < 1 || Wr < 1) return TDVP_E_SHAPE;
  if (!W && (d != 1 || Wl != Wr)) return TDVP_E_SHAPE;
  if ((int64_t)std::max(Wl, Wr) * d > 1024) return TDVP_E_UNSUPPORTED;
  const Op op{Lenv, W, Renv, Ml, d, Mr, Wl, Wr};
  const Layout lay = layout(op.size(), std::max(Wl, Wr), kmax, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  return run_lanczos(ctx, lay, op, z_re, z_im, kmax, tol, x, 0, y, 0, k_used_dev, Bi());
}

tdvp_status tdvp_lanczos_expm_noalloc(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv,
                                      int Ml, int d, int Mr, int Wl, int Wr, double z_re, double z_im,
                                      int kmax, double tol, const void *x, void *y, int32_t *k_used_dev) {
  if (!ctx || !Lenv || !Renv || !x || !y) return TDVP_E_ARG;
  if (kmax < 1 || kmax > KMAX || !(tol >= 0.0)) return TDVP_E_ARG;
  if (Ml < 1 || d < 1 || Mr < 1 || Wl < 1 || Wr < 1) return TDVP_E_SHAPE;
  if (!W && (d != 1 || Wl != Wr)) return TDVP_E_SHAPE;
  if ((int64_t)std::max(Wl, Wr) * d > 1024) return TDVP_E_UNSUPPORTED;
  const Op op{Lenv, W, Renv, Ml, d, Mr, Wl, Wr};
  const Layout lay = layout(op.size(), std::max(Wl, Wr), kmax, env_bytes(ctx));
  if (lay.total > TDVP_SCRATCH_BYTES) return TDVP_E_WORKSPACE;
  CK(hipSetDevice(ctx->device));
  char *sp = static_cast<char *>(scratch_of(ctx->device));
  if (!sp) return TDVP_E_DEVICE;
  // run the solve on the scratch array in place of the context's workspace;
  // no timing or tuning (both create events and time launches)
  char *ws = ctx->ws;
  const size_t wsb = ctx->ws_bytes;
  const int prof = ctx->prof_class, tune = ctx->autotune;
  ctx->ws = sp;
  ctx->ws_bytes = TDVP_SCRATCH_BYTES;
  ctx->prof_class = 0;
  ctx->autotune = 0;
  // the header's non-finite flag starts at zero for every call (a kernel,
  // not a memset, so that the call can be captured into a graph)
  tdvp_status st = TDVP_OK;
  if (set_dev_int(&header(ctx)->nonfinite, 0, ctx->stream) != hipSuccess) st = TDVP_E_DEVICE;
  if (st == TDVP_OK)
    st = run_lanczos(ctx, lay, op, z_re, z_im, kmax, tol, x, 0, y, 0, k_used_dev, Bi());
  ctx->ws = ws;
  ctx->ws_bytes = wsb;
  ctx->prof_class = prof;
  ctx->autotune = tune;
  return st;
}

tdvp_status tdvp_qr(tdvp_ctx *ctx, const void *A, int m, int n, void *Q, void *R) {
  if (!ctx || !A || !Q || !R) return TDVP_E_ARG;
  if (n < 1 || m < n) return TDVP_E_SHAPE;
  if (n > 256) return TDVP_E_UNSUPPORTED;
  const Layout lay = layout((int64_t)m * n, 1, 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  QrArgs q{};
  q.A = (const double2 *)A; q.a_rs = n; q.a_cs = 1;
  q.Q = (double2 *)Q; q.q_rs = n; q.q_cs = 1;
  q.R = (double2 *)R; q.r_rs = n; q.r_cs = 1;
  q.m = m; q.n = n;
  q.work = at<double2>(ctx, lay.qr);
  CK(qr(q, ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_right_canonicalize(tdvp_ctx *ctx, const tdvp_mps *mps) {
  if (!ctx) return TDVP_E_ARG;
  Chain ch;
  CS(check_chain(mps, nullptr, &ch));
  const Layout lay = layout(ch.nmax, 1, 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  double2 *D = at<double2>(ctx, lay.D), *tmp = at<double2>(ctx, lay.tmp);
  for (int i = ch.n - 1; i >= 1; --i) {
    const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
    CS(qr_right(ctx, lay, (double2 *)mps->site[i], Ml, d, Mr, D, Bi(), 0));
    const int Mp = ch.bond[i - 1], dp = ch.phys[i - 1];
    CS(matmul(ctx, (const double2 *)mps->site[i - 1], D, tmp, Mp * dp, Ml, Ml));
    CK(copy_c128((double2 *)mps->site[i - 1], tmp, (int64_t)Mp * dp * Ml, ctx->stream));
  }
  CK(normalize_c128((double2 *)mps->site[0], (int64_t)ch.phys[0] * ch.bond[1], ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_left_canonicalize(tdvp_ctx *ctx, const tdvp_mps *mps) {
  if (!ctx) return TDVP_E_ARG;
  Chain ch;
  CS(check_chain(mps, nullptr, &ch));
  const Layout lay = layout(ch.nmax, 1, 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  double2 *R = at<double2>(ctx, lay.D), *tmp = at<double2>(ctx, lay.tmp);
  const int n = ch.n;
  for (int i = 0; i + 1 < n; ++i) {
    const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
    if ((int64_t)Ml * d < Mr) return TDVP_E_SHAPE;
    CS(qr_left(ctx, lay, (double2 *)mps->site[i], Ml, d, Mr, R, Bi(), 0));
    const int64_t cols = (int64_t)ch.phys[i + 1] * ch.bond[i + 2];
    CS(matmul(ctx, R, (const double2 *)mps->site[i + 1], tmp, Mr, Mr, (int)cols));
    CK(copy_c128((double2 *)mps->site[i + 1], tmp, (int64_t)Mr * cols, ctx->stream));
  }
  CK(normalize_c128((double2 *)mps->site[n - 1], (int64_t)ch.bond[n - 1] * ch.phys[n - 1] * ch.bond[n],
                    ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_envs_build(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                            const tdvp_envs *envs) {
  if (!ctx || !envs || !envs->left || !envs->right) return TDVP_E_ARG;
  Chain ch;
  CS(check_chain(mps, mpo, &ch));
  const Layout lay = layout(ch.nmax, ch.wmax, 1, env_bytes(ctx));
  CS(need(ctx, lay));
  CK(hipSetDevice(ctx->device));
  const int n = ch.n;
  if (!envs->left[0] || !envs->right[n]) return TDVP_E_ARG;
  CK(fill_one(envs->left[0], env_type(ctx), ctx->stream));
  CK(fill_one(envs->right[n], env_type(ctx), ctx->stream));
  for (int i = n - 1; i >= 1; --i) {
    if (!envs->right[i] || !envs->right[i + 1]) return TDVP_E_ARG;
    CS(env_update(ctx, lay, -1, envs->right[i + 1], mps->site[i], mpo->site[i], ch.bond[i], ch.phys[i],
                  ch.bond[i + 1], ch.wbond[i], ch.wbond[i + 1], envs->right[i], Bi(), 0, 0, 0, 0));
  }
  return TDVP_OK;
}

namespace {

// Per-instance strides (elements) of every tensor of the chain, for a
// batch of identical-shape chains stored at constant strides.
struct Strides {
  std::vector<int64_t> site, mpo, envl, envr;
  void zeros(int n) { site.assign(n, 0); mpo.assign(n, 0); envl.assign(n + 1, 0); envr.assign(n + 1, 0); }
};

// Enqueue nsteps symmetric PS steps (eq:ps_trotter) on the context stream
// for b.R instances (instance 0 given by the descriptors, the others at the
// strides s).
tdvp_status enqueue_steps(tdvp_ctx *ctx, const Layout &lay, const Chain &ch, const tdvp_mps *mps,
                          const tdvp_mpo *mpo, const tdvp_envs *envs, double dt, int nsteps,
                          int kmax, double tol, const Bi &b, const Strides &s) {
  const int n = ch.n;
  double2 *D = at<double2>(ctx, lay.D), *tmp = at<double2>(ctx, lay.tmp);
  const int64_t wsx = b.wsel(16);   // instance stride of workspace c128 buffers
  const double h = 0.5 * dt;
  auto site = [&](int i) { return (double2 *)mps->site[i]; };
  for (int step = 0; step < nsteps; ++step) {
    // left-to-right half sweep
    const double2 *xin = site(0);
    int64_t sxin = s.site[0];
    for (int i = 0; i < n; ++i) {
      const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
      const bool last = (i == n - 1);
      Op f{envs->left[i], mpo->site[i], envs->right[i + 1], Ml, d, Mr, ch.wbond[i], ch.wbond[i + 1]};
      f.sL = s.envl[i]; f.sW = s.mpo[i]; f.sR = s.envr[i + 1];
      CS(run_lanczos(ctx, lay, f, 0.0, -(last ? dt : h), kmax, tol, xin, sxin, site(i), s.site[i],
                     nullptr, b));
      if (last) break;
      CS(qr_left(ctx, lay, site(i), Ml, d, Mr, D, b, s.site[i]));
      CS(env_update(ctx, lay, +1, envs->left[i], site(i), mpo->site[i], Ml, d, Mr, ch.wbond[i],
                    ch.wbond[i + 1], envs->left[i + 1], b, s.envl[i], s.site[i], s.mpo[i],
                    s.envl[i + 1]));
      const int Wb = ch.wbond[i + 1];
      Op k{envs->left[i + 1], nullptr, envs->right[i + 1], Mr, 1, Mr, Wb, Wb};
      k.sL = s.envl[i + 1]; k.sR = s.envr[i + 1];
      CS(run_lanczos(ctx, lay, k, 0.0, +h, kmax, tol, D, wsx, D, wsx, nullptr, b));
      const int dn = ch.phys[i + 1], Mn = ch.bond[i + 2];
      CS(matmul(ctx, D, site(i + 1), tmp, Mr, Mr, dn * Mn, b, wsx, s.site[i + 1], wsx));
      xin = tmp;
      sxin = wsx;
    }
    // right-to-left half sweep (the last site was advanced by dt above)
    for (int i = n - 1; i >= 0; --i) {
      const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
      if (i < n - 1) {
        Op f{envs->left[i], mpo->site[i], envs->right[i + 1], Ml, d, Mr, ch.wbond[i], ch.wbond[i + 1]};
        f.sL = s.envl[i]; f.sW = s.mpo[i]; f.sR = s.envr[i + 1];
        CS(run_lanczos(ctx, lay, f, 0.0, -h, kmax, tol, xin, sxin, site(i), s.site[i], nullptr, b));
      }
      if (i == 0) break;
      CS(qr_right(ctx, lay, site(i), Ml, d, Mr, D, b, s.site[i]));
      CS(env_update(ctx, lay, -1, envs->right[i + 1], site(i), mpo->site[i], Ml, d, Mr, ch.wbond[i],
                    ch.wbond[i + 1], envs->right[i], b, s.envr[i + 1], s.site[i], s.mpo[i],
                    s.envr[i]));
      const int Wb = ch.wbond[i];
      Op k{envs->left[i], nullptr, envs->right[i], Ml, 1, Ml, Wb, Wb};
      k.sL = s.envl[i]; k.sR = s.envr[i];
      CS(run_lanczos(ctx, lay, k, 0.0, +h, kmax, tol, D, wsx, D, wsx, nullptr, b));
      const int Mp = ch.bond[i - 1], dp = ch.phys[i - 1];
      CS(matmul(ctx, site(i - 1), D, tmp, Mp * dp, Ml, Ml, b, s.site[i - 1], wsx, wsx));
      xin = tmp;
      sxin = wsx;
    }
  }
  return TDVP_OK;
}

}  // namespace

tdvp_status tdvp_set_graph(tdvp_ctx *ctx, int enable) {
  if (!ctx) return TDVP_E_ARG;
  ctx->graph_mode = enable ? 1 : 0;
  return TDVP_OK;
}

tdvp_status tdvp_set_fused(tdvp_ctx *ctx, int enable) {
  if (!ctx) return TDVP_E_ARG;
  ctx->fused_off = enable ? 0 : 1;
  return TDVP_OK;
}

tdvp_status tdvp_set_stage3_split(tdvp_ctx *ctx, int per_channel) {
  if (!ctx) return TDVP_E_ARG;
  ctx->s3_per_channel = per_channel ? 1 : 0;
  return TDVP_OK;
}

tdvp_status tdvp_set_autotune(tdvp_ctx *ctx, int enable) {
  if (!ctx) return TDVP_E_ARG;
  ctx->autotune = enable ? 1 : 0;
  return TDVP_OK;
}

tdvp_status tdvp_autotune_count(const tdvp_ctx *ctx, int32_t *count) {
  if (!ctx || !count) return TDVP_E_ARG;
  *count = (int32_t)ctx->tuned.size();
  return TDVP_OK;
}

tdvp_status tdvp_ps_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                         const tdvp_envs *envs, double dt, int nsteps, int kmax, double tol) {
  return tdvp_ps_step_batched(ctx, 1, mps, mpo, envs, dt, nsteps, kmax, tol);
}

}  // extern "C"

namespace {

// Observables for b.R instances (see tdvp_observe); out has instance stride so.
tdvp_status observe_impl(tdvp_ctx *ctx, const Layout &lay, const Chain &ch, const tdvp_mps *mps,
                         const tdvp_mpo *mpo, const tdvp_envs *envs, const int32_t *el_sites, int n_el,
                         double *out_dev, int64_t so, const double *shifts, const Bi &b,
                         const Strides &s) {
  const int n = ch.n;
  const int64_t wsx = b.wsel(16);
  const double2 *C0 = (const double2 *)mps->site[0];
  const int64_t n0 = (int64_t)ch.phys[0] * ch.bond[1];
  CK(dot2d(C0, C0, 1, (int)n0, 0, 1, out_dev + 0, ctx->stream, b.R, s.site[0], s.site[0], so));
  Op e{envs->left[0], mpo->site[0], envs->right[1], 1, ch.phys[0], ch.bond[1], ch.wbond[0], ch.wbond[1]};
  e.sL = s.envl[0]; e.sW = s.mpo[0]; e.sR = s.envr[1];
  CS(apply_op(ctx, lay, e, C0, s.site[0], nullptr, b));
  CK(dot_partials(C0, env_type(ctx), ctx->ws + lay.Y, e.parts(), e.size(), e.size(), out_dev + 1,
                  ctx->stream, b.R, s.site[0], b.wsel(env_bytes(ctx)), so));
  for (int r = 0; r < b.R; ++r)
    CK(axpy_scalar(out_dev + 1 + r * so, out_dev + r * so, shifts[r], ctx->stream));
  if (n_el == 0) return TDVP_OK;
  int last = 0;
  for (int m = 0; m < n_el; ++m) last = std::max(last, (int)el_sites[m]);
  double2 *E = at<double2>(ctx, lay.obs), *E2 = E + lay.n, *T = E + 2 * lay.n;
  CK(fill_one(E, F64, ctx->stream, b.R, wsx));
  for (int i = 0; i <= last && i < n; ++i) {
    const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
    const double2 *A = (const double2 *)mps->site[i];
    // T[l'][s][r] = sum_l E[l'][l] A[l][s][r]
    CS(matmul(ctx, E, A, T, Ml, Ml, d * Mr, b, wsx, s.site[i], wsx));
    for (int m = 0; m < n_el; ++m)
      if (el_sites[m] == i)
        CK(dot2d(A + Mr, T + Mr, Ml, Mr, (int64_t)d * Mr, 1, out_dev + 2 + m, ctx->stream, b.R,
                 s.site[i], wsx, so));
    if (i == last) break;
    GemmArgs g{};   // E2[r'][r] = sum conj(A[l'][s][r']) T[l'][s][r]
    g.A = A; g.B = T; g.C = E2;
    g.M = Mr; g.N = Mr; g.K = Ml * d; g.batch = 1;
    g.sam = 1; g.sak = Mr; g.conjA = 1; g.sbk = Mr; g.sbn = 1; g.scm = Mr; g.scn = 1;
    g.inst = inst_of(b, s.site[i], wsx, wsx, 0);
    CK(gemm_t(ctx, F64, F64, F64, g));
    std::swap(E, E2);
  }
  return TDVP_OK;
}

// Instance strides of a batch of nb identical-shape chains: instance r's
// tensor = instance 0's + r * stride, checked for every r.  Returns false if
// the tensors are not laid out that way.
bool batch_strides(int nb, const tdvp_mps *mps, const tdvp_mpo *mpo, const tdvp_envs *envs,
                   const Chain &ch, int es, Strides *s) {
  const int n = ch.n;
  s->zeros(n);
  if (nb <= 1) return true;
  auto stride = [&](const void *p0, const void *p1, int esz, int64_t *out) {
    const int64_t d = (const char *)p1 - (const char *)p0;
    if (d % esz != 0) return false;
    *out = d / esz;
    return true;
  };
  for (int i = 0; i < n; ++i) {
    if (!stride(mps[0].site[i], mps[1].site[i], 16, &s->site[i])) return false;
    if (!stride(mpo[0].site[i], mpo[1].site[i], 16, &s->mpo[i])) return false;
  }
  for (int bb = 0; bb <= n; ++bb) {
    if (!stride(envs[0].left[bb], envs[1].left[bb], es, &s->envl[bb])) return false;
    if (!stride(envs[0].right[bb], envs[1].right[bb], es, &s->envr[bb])) return false;
  }
  for (int r = 2; r < nb; ++r) {
    for (int i = 0; i < n; ++i) {
      if ((const char *)mps[r].site[i] != (const char *)mps[0].site[i] + 16 * r * s->site[i]) return false;
      if ((const char *)mpo[r].site[i] != (const char *)mpo[0].site[i] + 16 * r * s->mpo[i]) return false;
    }
    for (int bb = 0; bb <= n; ++bb) {
      if ((const char *)envs[r].left[bb] != (const char *)envs[0].left[bb] + (int64_t)es * r * s->envl[bb])
        return false;
      if ((const char *)envs[r].right[bb] != (const char *)envs[0].right[bb] + (int64_t)es * r * s->envr[bb])
        return false;
    }
  }
  return true;
}

tdvp_status check_batch(tdvp_ctx *ctx, int nb, const tdvp_mps *mps, const tdvp_mpo *mpo,
                        const tdvp_envs *envs, Chain *ch, Strides *s) {
  if (!ctx || nb < 1 || !mps || !mpo || !envs) return TDVP_E_ARG;
  CS(check_chain(&mps[0], &mpo[0], ch));
  for (int r = 0; r < nb; ++r) {
    Chain c2;
    CS(check_chain(&mps[r], &mpo[r], &c2));
    if (c2.phys != ch->phys || c2.bond != ch->bond || c2.wbond != ch->wbond) return TDVP_E_SHAPE;
    if (!envs[r].left || !envs[r].right) return TDVP_E_ARG;
    for (int bb = 0; bb <= ch->n; ++bb)
      if (!envs[r].left[bb] || !envs[r].right[bb]) return TDVP_E_ARG;
  }
  if (!batch_strides(nb, mps, mpo, envs, *ch, env_bytes(ctx), s)) return TDVP_E_ARG;
  return TDVP_OK;
}

}  // namespace

namespace {

// Graph key fields common to every step entry point.
void step_key_head(const tdvp_ctx *ctx, double dt, double tol, int kmax, std::vector<uint64_t> *key) {
  uint64_t bits;
  std::memcpy(&bits, &dt, 8); key->push_back(bits);
  std::memcpy(&bits, &tol, 8); key->push_back(bits);
  key->push_back((uint64_t)kmax);
  key->push_back((uint64_t)(int)ctx->prec);
  key->push_back((uint64_t)ctx->fused_off);
  key->push_back((uint64_t)ctx->s3_per_channel);
  key->push_back((uint64_t)ctx->autotune);
  key->push_back((uint64_t)(uintptr_t)ctx->ws);
  key->push_back((uint64_t)(uintptr_t)ctx->stream);
}

// nsteps steps through a captured graph of one step (captured the first
// time `key` is met; with the autotuner on, one eager step first so that
// new problem keys are timed outside the capture).  enqueue(k) enqueues k
// steps eagerly.
template <typename F>
tdvp_status run_graphed(tdvp_ctx *ctx, const std::vector<uint64_t> &key, int nsteps, F enqueue) {
  if (!ctx->gexec || key != ctx->gkey) {
    if (ctx->autotune && nsteps > 0) {
      CS(enqueue(1));
      --nsteps;
    }
    if (ctx->gexec) { hipGraphExecDestroy(ctx->gexec); ctx->gexec = nullptr; }
    if (ctx->graph) { hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
    ctx->gkey.clear();
    CK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
    const tdvp_status st = enqueue(1);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
    if (st != TDVP_OK) { if (g) hipGraphDestroy(g); return st; }
    if (ec != hipSuccess || !g) return TDVP_E_DEVICE;
    ctx->graph = g;
    CK(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
    ctx->gkey = key;
  }
  for (int st = 0; st < nsteps; ++st) CK(hipGraphLaunch(ctx->gexec, ctx->stream));
  return TDVP_OK;
}

// ---------------------------------------------------------------------------
// Ensembles of uneven bond dimension: groups of instances (one group per
// bond-dimension class; identical shapes and constant strides inside a
// group, the same chain layout and MPO channel dims across groups) advanced
// together.  Every Krylov solve of a sweep position is one grouped sequence
// for all groups: per Krylov step one fused-step launch for the groups on
// the fused path, one launch per contraction stage and one projection
// launch for the groups on the general path, and one orthogonalisation
// launch for all; the gauge shifts, environment updates and centre moves
// run per group.
struct GroupRun {
  Chain ch;
  Layout lay;
  Bi b;
  Strides s;
  const tdvp_mps *mps;
  const tdvp_mpo *mpo;
  const tdvp_envs *envs;
  char *base;                      // workspace slice of the group's first instance
};

struct LzJob {
  Op op;
  const void *x;
  int64_t sx;
  void *y;
  int64_t sy;
  const GroupRun *g;
};

tdvp_status run_lanczos_grouped(tdvp_ctx *c, const std::vector<LzJob> &jobs_in, double zr, double zi,
                                int kmax, double tol) {
  std::vector<LzJob> jobs = jobs_in;
  for (LzJob &J : jobs) J.op.P = stage3_parts(J.op, J.g->b.R, c->s3_per_channel);   // as run_lanczos
  const int ng = (int)jobs.size();
  if (ng == 0) return TDVP_OK;
  if (ng > GMAX) return TDVP_E_UNSUPPORTED;
  const DType et = env_type(c), ct = et;
  const bool bf3 = c->prec == TDVP_BF16X3;
  HeffSmallArgs fa[GMAX];
  bool fused[GMAX];
  LzStartArgs sa[GMAX];
  LzFinishArgs fi[GMAX];
  LzInst li[GMAX];
  LzState *st[GMAX];
  LzPartials *pp[GMAX];
  double2 *U[GMAX];
  int64_t nn[GMAX];
  int kall = 0;
  WtableArgs wt[GMAX];
  int nwt = 0;
  for (int k = 0; k < ng; ++k) {
    const LzJob &J = jobs[k];
    const GroupRun &G = *J.g;
    const int64_t n = J.op.size();
    nn[k] = n;
    const int keff = (int)std::min<int64_t>(kmax, n);
    kall = std::max(kall, keff);
    fused[k] = fused_args(c, G.lay, J.op, G.b, fa[k], G.base);
    const int trows = fused[k] ? J.op.Ml * J.op.d : 0;
    st[k] = reinterpret_cast<LzState *>(G.base + G.lay.st);
    pp[k] = reinterpret_cast<LzPartials *>(G.base + G.lay.pp);
    U[k] = reinterpret_cast<double2 *>(G.base + G.lay.U);
    li[k].count = G.b.R; li[k].wss = G.b.ws; li[k].xs = J.sx; li[k].ys = J.sy;
    sa[k] = LzStartArgs{st[k], pp[k], (const double2 *)J.x, U[k], n, zr, zi, tol, keff, trows,
                        &header(c)->nonfinite, li[k]};
    fi[k] = LzFinishArgs{st[k], U[k], n, n, keff, (double2 *)J.y, nullptr, trows, li[k]};
    if (fused[k]) {
      fa[k].st = st[k]; fa[k].pp = pp[k]; fa[k].U = U[k];
      if (J.op.W)
        wt[nwt++] = WtableArgs{(const double2 *)J.op.W, J.op.Wl * J.op.d, J.op.d * J.op.Wr, J.op.sW,
                               const_cast<int *>(fa[k].row), const_cast<int *>(fa[k].col),
                               const_cast<double2 *>(fa[k].coef), G.b.ws, G.b.R};
    }
  }
  if (nwt) CK(wtable_grouped(wt, nwt, c->stream));
  CK(lz_start_grouped(sa, ng, c->stream));
  for (int j = 0; j < kall; ++j) {
    // fused path: one launch per staging variant
    for (int stg = 0; stg < 2; ++stg) {
      HeffSmallArgs ha[GMAX];
      int cnt[GMAX], nh = 0;
      for (int k = 0; k < ng; ++k)
        if (fused[k] && fa[k].staged == stg) {
          ha[nh] = fa[k];
          ha[nh].j = j;
          cnt[nh++] = jobs[k].g->b.R;
        }
      if (nh) {
        const int id = prof_begin(c, TDVP_PROF_LZ_FUSED);
        CK(timed_repeat(c, id, [&] { return heff_small_grouped(et, ha, cnt, nh, c->stream); }));
        double fl = 0.0, by = 0.0;
        for (int q = 0; q < nh; ++q) {
          const double Ml = ha[q].Ml, d = ha[q].d, Mr = ha[q].Mr, Wl = ha[q].Wl, Wr = ha[q].Wr, n = ha[q].n;
          fl += cnt[q] * (8.0 * (Ml * d * Mr * Wr * Mr + Wl * Ml * Ml * d * Mr) + 8.0 * (j + 1) * n);
          by += cnt[q] * ((Ml * Wl * Ml + Mr * Wr * Mr) * env_bytes(c) + (j + 2) * 16.0 * n);
        }
        prof_end(c, id, fl, by);
      }
    }
    // general path: contraction stages and projections
    GemmArgs g1[GMAX], g3[GMAX];
    WApplyArgs wa[GMAX];
    LzDotsArgs da[GMAX];
    int ngen = 0, nw = 0;
    for (int k = 0; k < ng; ++k) {
      if (fused[k]) continue;
      const LzJob &J = jobs[k];
      const GroupRun &G = *J.g;
      const OpLaunch L = op_args(c, G.base, G.lay, J.op, U[k] + (int64_t)j * nn[k], G.b.wsel(16),
                                 &st[k]->stop, G.b);
      g1[ngen] = L.g1;
      g3[ngen] = L.g3;
      if (L.has_w) wa[nw++] = L.w;
      da[ngen] = LzDotsArgs{st[k], pp[k], G.base + G.lay.Y, J.op.parts(), nn[k], U[k], nn[k], j, nn[k], li[k]};
      ++ngen;
    }
    if (ngen) {
      // algorithmic work of a grouped GEMM: 8 M N K per batch and instance;
      // operands read once, result written once
      auto gw = [&](const GemmArgs *g, DType ta, DType tb, DType tc, double *fl, double *by) {
        *fl = *by = 0.0;
        for (int q = 0; q < ngen; ++q) {
          const double M = g[q].M, N = g[q].N, K = g[q].K, B = g[q].batch, R = g[q].inst.count;
          *fl += 8.0 * M * N * K * B * R;
          *by += R * ((g[q].bsa ? B : 1.0) * M * K * esz(ta) + (g[q].bsb ? B : 1.0) * K * N * esz(tb) +
                      B * M * N * esz(tc));
        }
      };
      double fl, gb;
      int id = prof_begin(c, TDVP_PROF_GEMM_HEFF);
      CK(timed_repeat(c, id, [&] { return cgemm_grouped(F64, et, ct, g1, ngen, bf3 && ct == F32, c->stream); }));
      gw(g1, F64, et, ct, &fl, &gb);
      prof_end(c, id, fl, gb);
      if (nw) {
        id = prof_begin(c, TDVP_PROF_WAPPLY);
        CK(timed_repeat(c, id, [&] { return wapply_grouped(ct, wa, nw, c->stream); }));
        double by = 0.0;
        for (int q = 0; q < nw; ++q)
          by += (double)wa[q].A * wa[q].C * wa[q].d * esz(ct) * (wa[q].Wl + wa[q].Wr) * wa[q].inst.count;
        prof_end(c, id, 0.0, by);
      }
      id = prof_begin(c, TDVP_PROF_GEMM_HEFF);
      CK(timed_repeat(c, id, [&] { return cgemm_grouped(et, ct, ct, g3, ngen, bf3 && ct == F32, c->stream); }));
      gw(g3, et, ct, ct, &fl, &gb);
      prof_end(c, id, fl, gb);
      id = prof_begin(c, TDVP_PROF_LZ_DOTS);
      CK(lz_dots_grouped(ct, da, ngen, c->stream));
      fl = gb = 0.0;
      for (int q = 0; q < ngen; ++q) {
        const double n = (double)da[q].n, R = da[q].in.count;
        fl += 8.0 * (j + 1) * n * R;
        gb += R * ((double)da[q].P * n * env_bytes(c) + (j + 2) * 16.0 * n);
      }
      prof_end(c, id, fl, gb);
    }
    LzUpdateArgs ua[GMAX];
    for (int k = 0; k < ng; ++k) {
      if (fused[k])
        ua[k] = LzUpdateArgs{st[k], pp[k], U[k], nn[k], j, nn[k], jobs[k].op.Mr * fa[k].P, fa[k].Yp, fa[k].P, li[k]};
      else
        ua[k] = LzUpdateArgs{st[k], pp[k], U[k], nn[k], j, nn[k], 0, nullptr, 0, li[k]};
    }
    const int id = prof_begin(c, TDVP_PROF_LZ_UPDATE);
    CK(lz_update_grouped(ua, ng, c->stream));
    double fl = 0.0, by = 0.0;
    for (int k = 0; k < ng; ++k) {
      fl += 8.0 * (j + 1) * nn[k] * li[k].count;
      by += (j + 3) * 16.0 * nn[k] * li[k].count;
    }
    prof_end(c, id, fl, by);
  }
  const int id = prof_begin(c, TDVP_PROF_LZ_ENDS);
  CK(lz_finish_grouped(fi, ng, c->stream));
  double fl = 0.0, by = 0.0;
  for (int k = 0; k < ng; ++k) {
    fl += 8.0 * fi[k].keff * nn[k] * li[k].count;
    by += (fi[k].keff + 1) * 16.0 * nn[k] * li[k].count;
  }
  prof_end(c, id, fl, by);
  return TDVP_OK;
}

// Run per-group helpers (QR, environment update, centre move) on group g's
// workspace: the helpers address the workspace through ctx->ws.
template <typename F> tdvp_status on_group(tdvp_ctx *c, const GroupRun &g, F f) {
  char *ws = c->ws;
  c->ws = g.base;
  const tdvp_status st = f();
  c->ws = ws;
  return st;
}

tdvp_status enqueue_steps_grouped(tdvp_ctx *ctx, std::vector<GroupRun> &gr, double dt, int nsteps,
                                  int kmax, double tol) {
  const int ng = (int)gr.size();
  const int n = gr[0].ch.n;
  const double h = 0.5 * dt;
  auto site = [&](const GroupRun &g, int i) { return (double2 *)g.mps->site[i]; };
  auto Dp = [&](const GroupRun &g) { return reinterpret_cast<double2 *>(g.base + g.lay.D); };
  auto Tp = [&](const GroupRun &g) { return reinterpret_cast<double2 *>(g.base + g.lay.tmp); };
  for (int step = 0; step < nsteps; ++step) {
    std::vector<const double2 *> xin(ng);
    std::vector<int64_t> sxin(ng);
    for (int q = 0; q < ng; ++q) { xin[q] = site(gr[q], 0); sxin[q] = gr[q].s.site[0]; }
    // left-to-right half sweep
    for (int i = 0; i < n; ++i) {
      const bool last = (i == n - 1);
      std::vector<LzJob> jobs;
      for (int q = 0; q < ng; ++q) {
        const GroupRun &g = gr[q];
        Op f{g.envs->left[i], g.mpo->site[i], g.envs->right[i + 1], g.ch.bond[i], g.ch.phys[i],
             g.ch.bond[i + 1], g.ch.wbond[i], g.ch.wbond[i + 1]};
        f.sL = g.s.envl[i]; f.sW = g.s.mpo[i]; f.sR = g.s.envr[i + 1];
        jobs.push_back(LzJob{f, xin[q], sxin[q], site(g, i), g.s.site[i], &g});
      }
      CS(run_lanczos_grouped(ctx, jobs, 0.0, -(last ? dt : h), kmax, tol));
      if (last) break;
      std::vector<LzJob> bj;
      for (int q = 0; q < ng; ++q) {
        const GroupRun &g = gr[q];
        const int Ml = g.ch.bond[i], d = g.ch.phys[i], Mr = g.ch.bond[i + 1];
        CS(on_group(ctx, g, [&] {
          CS(qr_left(ctx, g.lay, site(g, i), Ml, d, Mr, Dp(g), g.b, g.s.site[i]));
          return env_update(ctx, g.lay, +1, g.envs->left[i], site(g, i), g.mpo->site[i], Ml, d, Mr,
                            g.ch.wbond[i], g.ch.wbond[i + 1], g.envs->left[i + 1], g.b, g.s.envl[i],
                            g.s.site[i], g.s.mpo[i], g.s.envl[i + 1]);
        }));
        const int Wb = g.ch.wbond[i + 1];
        Op k{g.envs->left[i + 1], nullptr, g.envs->right[i + 1], Mr, 1, Mr, Wb, Wb};
        k.sL = g.s.envl[i + 1]; k.sR = g.s.envr[i + 1];
        bj.push_back(LzJob{k, Dp(g), g.b.wsel(16), Dp(g), g.b.wsel(16), &g});
      }
      CS(run_lanczos_grouped(ctx, bj, 0.0, +h, kmax, tol));
      for (int q = 0; q < ng; ++q) {
        const GroupRun &g = gr[q];
        const int Mr = g.ch.bond[i + 1], dn = g.ch.phys[i + 1], Mn = g.ch.bond[i + 2];
        const int64_t wsx = g.b.wsel(16);
        CS(on_group(ctx, g, [&] {
          return matmul(ctx, Dp(g), site(g, i + 1), Tp(g), Mr, Mr, dn * Mn, g.b, wsx, g.s.site[i + 1], wsx);
        }));
        xin[q] = Tp(g);
        sxin[q] = wsx;
      }
    }
    // right-to-left half sweep (the last site was advanced by dt above)
    for (int i = n - 1; i >= 0; --i) {
      if (i < n - 1) {
        std::vector<LzJob> jobs;
        for (int q = 0; q < ng; ++q) {
          const GroupRun &g = gr[q];
          Op f{g.envs->left[i], g.mpo->site[i], g.envs->right[i + 1], g.ch.bond[i], g.ch.phys[i],
               g.ch.bond[i + 1], g.ch.wbond[i], g.ch.wbond[i + 1]};
          f.sL = g.s.envl[i]; f.sW = g.s.mpo[i]; f.sR = g.s.envr[i + 1];
          jobs.push_back(LzJob{f, xin[q], sxin[q], site(g, i), g.s.site[i], &g});
        }
        CS(run_lanczos_grouped(ctx, jobs, 0.0, -h, kmax, tol));
      }
      if (i == 0) break;
      std::vector<LzJob> bj;
      for (int q = 0; q < ng; ++q) {
        const GroupRun &g = gr[q];
        const int Ml = g.ch.bond[i], d = g.ch.phys[i], Mr = g.ch.bond[i + 1];
        CS(on_group(ctx, g, [&] {
          CS(qr_right(ctx, g.lay, site(g, i), Ml, d, Mr, Dp(g), g.b, g.s.site[i]));
          return env_update(ctx, g.lay, -1, g.envs->right[i + 1], site(g, i), g.mpo->site[i], Ml, d, Mr,
                            g.ch.wbond[i], g.ch.wbond[i + 1], g.envs->right[i], g.b, g.s.envr[i + 1],
                            g.s.site[i], g.s.mpo[i], g.s.envr[i]);
        }));
        const int Wb = g.ch.wbond[i];
        Op k{g.envs->left[i], nullptr, g.envs->right[i], Ml, 1, Ml, Wb, Wb};
        k.sL = g.s.envl[i]; k.sR = g.s.envr[i];
        bj.push_back(LzJob{k, Dp(g), g.b.wsel(16), Dp(g), g.b.wsel(16), &g});
      }
      CS(run_lanczos_grouped(ctx, bj, 0.0, +h, kmax, tol));
      for (int q = 0; q < ng; ++q) {
        const GroupRun &g = gr[q];
        const int Ml = g.ch.bond[i], Mp = g.ch.bond[i - 1], dp = g.ch.phys[i - 1];
        const int64_t wsx = g.b.wsel(16);
        CS(on_group(ctx, g, [&] {
          return matmul(ctx, site(g, i - 1), Dp(g), Tp(g), Mp * dp, Ml, Ml, g.b, g.s.site[i - 1], wsx, wsx);
        }));
        xin[q] = Tp(g);
        sxin[q] = wsx;
      }
    }
  }
  return TDVP_OK;
}

// The groups of a grouped step in two lanes that run concurrently: groups
// whose bond dimensions are all small (<= 64: latency-bound solves, on the
// fused step for a small batch) on the context stream, the others
// (contraction GEMMs, MFMA bound) on the auxiliary stream, forked from and
// joined to the context stream
// (in graph mode the two lanes become parallel branches of the graph).
// Without profiling, the Krylov log or a second lane, one lane.
tdvp_status enqueue_lanes(tdvp_ctx *ctx, std::vector<GroupRun> &gr, double dt, int nsteps, int kmax,
                          double tol) {
  std::vector<GroupRun> small, large;
  for (const GroupRun &g : gr) (g.ch.mmax <= FUSED_MAX_MR ? small : large).push_back(g);
  if (small.empty() || large.empty() || ctx->prof_class != 0 || ctx->fused_off || !ctx->aux || !ctx->stream)
    return enqueue_steps_grouped(ctx, gr, dt, nsteps, kmax, tol);
  hipStream_t main = ctx->stream;
  CK(hipEventRecord(ctx->fork_ev, main));
  CK(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
  ctx->stream = ctx->aux;
  const tdvp_status sl = enqueue_steps_grouped(ctx, large, dt, nsteps, kmax, tol);
  ctx->stream = main;
  // join the auxiliary lane even on an error, so that a capture ends cleanly
  const hipError_t e1 = hipEventRecord(ctx->join_ev, ctx->aux);
  const tdvp_status ss = sl == TDVP_OK ? enqueue_steps_grouped(ctx, small, dt, nsteps, kmax, tol) : sl;
  const hipError_t e2 = hipStreamWaitEvent(main, ctx->join_ev, 0);
  if (ss != TDVP_OK) return ss;
  if (e1 != hipSuccess || e2 != hipSuccess) return TDVP_E_DEVICE;
  return TDVP_OK;
}

// Validate the groups of a grouped call and lay out their workspaces.
tdvp_status plan_groups(tdvp_ctx *ctx, int ng, const int32_t *counts, const tdvp_mps *mps,
                        const tdvp_mpo *mpo, const tdvp_envs *envs, int kmax,
                        std::vector<GroupRun> *gr, size_t *bytes) {
  if (!ctx || ng < 1 || ng > GMAX || !counts || !mps || !mpo) return TDVP_E_ARG;
  gr->clear();
  size_t off = 0;
  int first = 0;
  for (int q = 0; q < ng; ++q) {
    if (counts[q] < 1) return TDVP_E_ARG;
    GroupRun g;
    if (envs) {
      CS(check_batch(ctx, counts[q], mps + first, mpo + first, envs + first, &g.ch, &g.s));
    } else {
      CS(check_chain(&mps[first], &mpo[first], &g.ch));
    }
    if (q > 0 && (g.ch.n != (*gr)[0].ch.n || g.ch.phys != (*gr)[0].ch.phys || g.ch.wbond != (*gr)[0].ch.wbond))
      return TDVP_E_SHAPE;
    g.lay = layout(g.ch.nmax, g.ch.wmax, kmax, env_bytes(ctx));
    g.b.R = counts[q];
    g.b.ws = (int64_t)g.lay.total;
    g.mps = mps + first;
    g.mpo = mpo + first;
    g.envs = envs ? envs + first : nullptr;
    g.base = ctx->ws ? ctx->ws + off : nullptr;
    off += (size_t)counts[q] * g.lay.total;
    first += counts[q];
    gr->push_back(g);
  }
  *bytes = off;
  return TDVP_OK;
}

}  // namespace

extern "C" {

tdvp_status tdvp_observe(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, const tdvp_envs *envs,
                         const int32_t *el_sites, int n_el, double *out_dev) {
  return tdvp_observe_batched(ctx, 1, mps, mpo, envs, el_sites, n_el, out_dev);
}

tdvp_status tdvp_observe_batched(tdvp_ctx *ctx, int nb, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 const tdvp_envs *envs, const int32_t *el_sites, int n_el,
                                 double *out_dev) {
  if (!ctx || !out_dev || n_el < 0 || (n_el > 0 && !el_sites)) return TDVP_E_ARG;
  Chain ch;
  Strides s;
  CS(check_batch(ctx, nb, mps, mpo, envs, &ch, &s));
  for (int m = 0; m < n_el; ++m)
    if (el_sites[m] < 0 || el_sites[m] >= ch.n || ch.phys[el_sites[m]] != 2) return TDVP_E_SHAPE;
  const Layout lay = layout(ch.nmax, ch.wmax, 1, env_bytes(ctx));
  Bi b;
  b.R = nb;
  b.ws = (int64_t)lay.total;
  if (!ctx->ws || ctx->ws_bytes < (size_t)nb * lay.total) return TDVP_E_WORKSPACE;
  CK(hipSetDevice(ctx->device));
  std::vector<double> shifts(nb);
  for (int r = 0; r < nb; ++r) shifts[r] = mpo[r].energy_shift;
  CS(observe_impl(ctx, lay, ch, mps, mpo, envs, el_sites, n_el, out_dev, 2 + n_el, shifts.data(), b, s));
  // non-finite check: the context's sticky Lanczos flag and every observable
  // just written; the host waits for the stream here
  CtxHeader *hdr = header(ctx);
  CK(numeric_check(&hdr->nonfinite, 0, out_dev, 2 + n_el, 2 + n_el, nb, &hdr->numeric_out,
                   ctx->stream));
  int bad = 0;
  CK(hipMemcpyAsync(&bad, &hdr->numeric_out, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  return bad ? TDVP_E_NUMERIC : TDVP_OK;
}

tdvp_status tdvp_ps_step_batched(tdvp_ctx *ctx, int nb, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 const tdvp_envs *envs, double dt, int nsteps, int kmax, double tol) {
  if (nsteps < 0 || kmax < 1 || kmax > KMAX || !(tol >= 0.0) || !std::isfinite(dt)) return TDVP_E_ARG;
  Chain ch;
  Strides s;
  CS(check_batch(ctx, nb, mps, mpo, envs, &ch, &s));
  const Layout lay = layout(ch.nmax, ch.wmax, kmax, env_bytes(ctx));
  Bi b;
  b.R = nb;
  b.ws = (int64_t)lay.total;
  if (!ctx->ws || ctx->ws_bytes < (size_t)nb * lay.total) return TDVP_E_WORKSPACE;
  CK(hipSetDevice(ctx->device));
  ctx->klog_pos = 0;
  if (!ctx->graph_mode || ctx->prof_class != 0 || ctx->klog || !ctx->stream || nsteps == 0)
    return enqueue_steps(ctx, lay, ch, &mps[0], &mpo[0], &envs[0], dt, nsteps, kmax, tol, b, s);
  std::vector<uint64_t> key;
  auto put = [&](const void *p) { key.push_back((uint64_t)(uintptr_t)p); };
  step_key_head(ctx, dt, tol, kmax, &key);
  key.push_back((uint64_t)nb);
  for (int i = 0; i < ch.n; ++i) {
    put(mps[0].site[i]); put(mpo[0].site[i]);
    key.push_back((uint64_t)s.site[i]); key.push_back((uint64_t)s.mpo[i]);
    key.push_back((uint64_t)ch.phys[i]);
  }
  for (int bb = 0; bb <= ch.n; ++bb) {
    put(envs[0].left[bb]); put(envs[0].right[bb]);
    key.push_back((uint64_t)s.envl[bb]); key.push_back((uint64_t)s.envr[bb]);
    key.push_back((uint64_t)ch.bond[bb] << 32 | (uint32_t)ch.wbond[bb]);
  }
  return run_graphed(ctx, key, nsteps, [&](int k) {
    return enqueue_steps(ctx, lay, ch, &mps[0], &mpo[0], &envs[0], dt, k, kmax, tol, b, s);
  });
}

}  // extern "C"

extern "C" {

tdvp_status tdvp_workspace_bytes_grouped(const tdvp_ctx *ctx, int ngroups, const int32_t *counts,
                                         const tdvp_mps *mps, const tdvp_mpo *mpo, int kmax,
                                         size_t *bytes) {
  if (!bytes || kmax < 1 || kmax > KMAX) return TDVP_E_ARG;
  std::vector<GroupRun> gr;
  return plan_groups(const_cast<tdvp_ctx *>(ctx), ngroups, counts, mps, mpo, nullptr, kmax, &gr, bytes);
}

tdvp_status tdvp_ps_step_grouped(tdvp_ctx *ctx, int ngroups, const int32_t *counts, const tdvp_mps *mps,
                                 const tdvp_mpo *mpo, const tdvp_envs *envs, double dt, int nsteps,
                                 int kmax, double tol) {
  if (nsteps < 0 || kmax < 1 || kmax > KMAX || !(tol >= 0.0) || !std::isfinite(dt) || !envs)
    return TDVP_E_ARG;
  std::vector<GroupRun> gr;
  size_t bytes = 0;
  CS(plan_groups(ctx, ngroups, counts, mps, mpo, envs, kmax, &gr, &bytes));
  if (!ctx->ws || ctx->ws_bytes < bytes) return TDVP_E_WORKSPACE;
  CK(hipSetDevice(ctx->device));
  ctx->klog_pos = 0;
  if (!ctx->aux) {
    CK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    CK(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
  }
  if (!ctx->graph_mode || ctx->prof_class != 0 || !ctx->stream || nsteps == 0)
    return enqueue_lanes(ctx, gr, dt, nsteps, kmax, tol);
  std::vector<uint64_t> key;
  auto put = [&](const void *p) { key.push_back((uint64_t)(uintptr_t)p); };
  step_key_head(ctx, dt, tol, kmax, &key);
  key.push_back(0x67726f7570ull);   // grouped
  for (const GroupRun &g : gr) {
    key.push_back((uint64_t)g.b.R);
    for (int i = 0; i < g.ch.n; ++i) {
      put(g.mps->site[i]); put(g.mpo->site[i]);
      key.push_back((uint64_t)g.s.site[i]); key.push_back((uint64_t)g.s.mpo[i]);
      key.push_back((uint64_t)g.ch.phys[i]);
    }
    for (int bb = 0; bb <= g.ch.n; ++bb) {
      put(g.envs->left[bb]); put(g.envs->right[bb]);
      key.push_back((uint64_t)g.s.envl[bb]); key.push_back((uint64_t)g.s.envr[bb]);
      key.push_back((uint64_t)g.ch.bond[bb] << 32 | (uint32_t)g.ch.wbond[bb]);
    }
  }
  return run_graphed(ctx, key, nsteps, [&](int k) { return enqueue_lanes(ctx, gr, dt, k, kmax, tol); });
}

tdvp_status tdvp_observe_grouped(tdvp_ctx *ctx, int ngroups, const int32_t *counts, const tdvp_mps *mps,
                                 const tdvp_mpo *mpo, const tdvp_envs *envs, const int32_t *el_sites,
                                 int n_el, double *out_dev) {
  if (!out_dev || n_el < 0 || (n_el > 0 && !el_sites) || !envs) return TDVP_E_ARG;
  std::vector<GroupRun> gr;
  size_t bytes = 0;
  CS(plan_groups(ctx, ngroups, counts, mps, mpo, envs, 1, &gr, &bytes));
  if (!ctx->ws || ctx->ws_bytes < bytes) return TDVP_E_WORKSPACE;
  for (int m = 0; m < n_el; ++m)
    if (el_sites[m] < 0 || el_sites[m] >= gr[0].ch.n || gr[0].ch.phys[el_sites[m]] != 2) return TDVP_E_SHAPE;
  CK(hipSetDevice(ctx->device));
  const int so = 2 + n_el;
  int first = 0, total = 0;
  for (const GroupRun &g : gr) {
    std::vector<double> shifts(g.b.R);
    for (int r = 0; r < g.b.R; ++r) shifts[r] = g.mpo[r].energy_shift;
    CS(on_group(ctx, g, [&] {
      return observe_impl(ctx, g.lay, g.ch, g.mps, g.mpo, g.envs, el_sites, n_el, out_dev + (int64_t)first * so,
                          so, shifts.data(), g.b, g.s);
    }));
    first += g.b.R;
    total += g.b.R;
  }
  CtxHeader *hdr = header(ctx);
  CK(numeric_check(&hdr->nonfinite, 0, out_dev, so, so, total, &hdr->numeric_out, ctx->stream));
  int bad = 0;
  CK(hipMemcpyAsync(&bad, &hdr->numeric_out, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  return bad ? TDVP_E_NUMERIC : TDVP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// TDVP-MU (Sec. II.A.2, "TDVP-MU"), variable-mean-field integration.
//
// State: left-canonical site tensors L_0..L_{n-2} and the centre C_{n-1}.
// One right-hand side (eq:tdvp1_C, eq:tdvp1_mu_L with eq:reg2):
//   1. left environments h[1:i] from the L's (eq:tdvp1_h1i);
//   2. an RQ sweep from the right end, C_{n-1} = D_{n-1} R_{n-1},
//      L_{i} D_{i+1} = D_i R_i, giving right isometries R_i and the bond
//      matrices D_b between sites b-1 and b;
//   3. right environments from the R's (eq:tdvp1_hiN);
//   4. per site i < n-1: P = V Lam~^{-1} U^H from D_{i+1} = U Lam V^H,
//      G = H[i] (L_i D_{i+1}), X = G P, dL_i/dt = -i (X - L_i (L_i^H X));
//   5. dC_{n-1}/dt = -i H[n-1] C_{n-1}.
// The integrator is the Dormand-Prince 5(4) pair with the usual step-size
// control (error norm scaled by atol + rtol max(|y|, |y_new|), safety 0.9,
// step factor within [0.2, 10], first step from the two-evaluation rule);
// the step decision is taken on the host after each step (one sync).
//
// Constant mean field, second order: steps 1-3 and the regularised inverse
// of step 4 (the mean fields) are taken at one state and held; with them
// each site's equation involves that site alone.  The fields of the state
// at t carry every site to t + tau/2, the fields of that midpoint state
// carry the state at t to t + tau.  The site tensors L_i follow their
// frozen-field equations with the Dormand-Prince pair, all sites together
// on one packed vector with one step size (the equations do not couple, so
// this is their joint solution; the error control takes the worst site);
// the centre follows its linear one by the Lanczos propagator.
namespace {

constexpr int MU_LANES = 4;        // streams the site derivatives are spread over

struct MuPlan {
  Chain ch;
  Layout lay;                       // local-problem region (contraction, QR scratch)
  std::vector<size_t> lenv, renv, rt, dbuf, pbuf, site_off;   // byte offsets / element offsets (site_off)
  // per-lane site temporaries; lane 0 contracts in lay, lane k in lane_lay[k]
  // (lay with its own T1, T2, Y buffers)
  Layout lane_lay[MU_LANES];
  size_t C[MU_LANES], G[MU_LANES], X[MU_LANES], Y[MU_LANES], T[MU_LANES];
  size_t vec[12];                   // packed vectors: y, ys, ynew, err, k1..k7, start state (CMF)
  size_t part;                      // RK error partial sums
  int64_t ntot;                     // packed length (complex elements)
  size_t total;
};

constexpr int MU_MAXM = 64;         // bond dimensions the regularised inverse handles

// kmax: Krylov dimension the local-problem region must hold (1 without the
// centre's Lanczos propagator).
tdvp_status mu_plan(const tdvp_ctx *c, const tdvp_mps *mps, const tdvp_mpo *mpo, MuPlan *pl, int kmax = 1) {
  if (!c || !mpo) return TDVP_E_ARG;
  CS(check_chain(mps, mpo, &pl->ch));
  if (c->prec != TDVP_FP64) return TDVP_E_UNSUPPORTED;
  const Chain &ch = pl->ch;
  const int n = ch.n;
  if (n < 2) return TDVP_E_SHAPE;
  if (ch.mmax > MU_MAXM) return TDVP_E_UNSUPPORTED;
  pl->lay = layout(ch.nmax, ch.wmax, kmax, 16);
  size_t o = pl->lay.total;
  auto take = [&](size_t bytes) { const size_t r = o; o += al256(bytes); return r; };
  pl->lenv.assign(n + 1, 0);
  pl->renv.assign(n + 1, 0);
  pl->dbuf.assign(n + 1, 0);
  pl->pbuf.assign(n + 1, 0);
  pl->rt.assign(n, 0);
  pl->site_off.assign(n + 1, 0);
  for (int b = 0; b <= n; ++b) {
    const size_t e = (size_t)ch.bond[b] * ch.wbond[b] * ch.bond[b] * 16;
    pl->lenv[b] = take(e);
    pl->renv[b] = take(e);
    pl->dbuf[b] = take((size_t)ch.bond[b] * ch.bond[b] * 16);
    pl->pbuf[b] = take((size_t)ch.bond[b] * ch.bond[b] * 16);
  }
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t sz = (int64_t)ch.bond[i] * ch.phys[i] * ch.bond[i + 1];
    pl->rt[i] = take((size_t)sz * 16);
    pl->site_off[i] = tot;
    tot += sz;
  }
  pl->site_off[n] = tot;
  pl->ntot = tot;
  const size_t m2 = (size_t)ch.mmax * ch.mmax * 16, nv = (size_t)ch.nmax * 16;
  for (int k = 0; k < MU_LANES; ++k) {
    pl->lane_lay[k] = pl->lay;
    if (k > 0) {
      pl->lane_lay[k].T1 = take(pl->lay.ybytes);
      pl->lane_lay[k].T2 = take(pl->lay.ybytes);
      pl->lane_lay[k].Y = take(pl->lay.ybytes);
    }
    pl->T[k] = take(m2);
    pl->C[k] = take(nv);
    pl->G[k] = take(nv);
    pl->X[k] = take(nv);
    pl->Y[k] = take(nv);
  }
  for (size_t &v : pl->vec) v = take((size_t)tot * 16);
  pl->part = take(RK_PARTS * sizeof(double));
  pl->total = o;
  return TDVP_OK;
}

// Mean fields of the left-canonical state A (host table of n device
// pointers): steps 1-3 and, per site i < n-1, the regularised inverse factor
// P_i = V Lam~^{-1} U^H of D_{i+1} (pbuf[i+1]).
tdvp_status mu_fields(tdvp_ctx *c, const MuPlan &pl, const tdvp_mpo *mpo, const double2 *const *A,
                      double eps) {
  const Chain &ch = pl.ch;
  const int n = ch.n;
  const Layout &lay = pl.lay;
  auto B = [&](size_t off) { return reinterpret_cast<double2 *>(c->ws + off); };
  // 1. left environments
  CK(fill_one(B(pl.lenv[0]), F64, c->stream));
  for (int i = 0; i + 1 < n; ++i)
    CS(env_update(c, lay, +1, B(pl.lenv[i]), A[i], mpo->site[i], ch.bond[i], ch.phys[i], ch.bond[i + 1],
                  ch.wbond[i], ch.wbond[i + 1], B(pl.lenv[i + 1]), Bi(), 0, 0, 0, 0));
  // 2. RQ sweep: rt[i] = R_i, dbuf[i] = D_i (bond i, between sites i-1 and i)
  for (int i = n - 1; i >= 1; --i) {
    const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
    const int64_t sz = (int64_t)Ml * d * Mr;
    if (i == n - 1) CK(copy_c128(B(pl.rt[i]), A[i], sz, c->stream));
    else CS(matmul(c, A[i], B(pl.dbuf[i + 1]), B(pl.rt[i]), Ml * d, Mr, Mr));
    CS(qr_right(c, lay, B(pl.rt[i]), Ml, d, Mr, B(pl.dbuf[i]), Bi(), 0));
  }
  // 3. right environments
  CK(fill_one(B(pl.renv[n]), F64, c->stream));
  for (int i = n - 1; i >= 1; --i)
    CS(env_update(c, lay, -1, B(pl.renv[i + 1]), B(pl.rt[i]), mpo->site[i], ch.bond[i], ch.phys[i],
                  ch.bond[i + 1], ch.wbond[i], ch.wbond[i + 1], B(pl.renv[i]), Bi(), 0, 0, 0, 0));
  // regularised inverse factors of step 4: independent per bond, so the
  // bonds go side by side (one work-group each)
  for (int i0 = 0; i0 + 1 < n; i0 += REGINV_BATCH) {
    RegInvBatch rb{};
    rb.eps = eps;
    for (int i = i0; i + 1 < n && rb.count < REGINV_BATCH; ++i) {
      rb.D[rb.count] = B(pl.dbuf[i + 1]);
      rb.P[rb.count] = B(pl.pbuf[i + 1]);
      rb.n[rb.count] = ch.bond[i + 1];
      ++rb.count;
    }
    CK(mu_reginv(rb, c->stream));
  }
  return TDVP_OK;
}

// d(site i)/dt of one site with the mean fields last computed (steps 4
// and 5), on c->stream with the temporaries of lane k.
tdvp_status mu_site_one(tdvp_ctx *c, const MuPlan &pl, int k, const tdvp_mpo *mpo, int i, const double2 *A,
                        double2 *out) {
  const Chain &ch = pl.ch;
  const int n = ch.n;
  const Layout &lay = pl.lane_lay[k];
  auto B = [&](size_t off) { return reinterpret_cast<double2 *>(c->ws + off); };
  const int Ml = ch.bond[i], d = ch.phys[i], Mr = ch.bond[i + 1];
  const int64_t sz = (int64_t)Ml * d * Mr;
  const double2 *x = A;
  if (i + 1 < n) {
    CS(matmul(c, A, B(pl.dbuf[i + 1]), B(pl.C[k]), Ml * d, Mr, Mr));
    x = B(pl.C[k]);
  }
  const Op op{B(pl.lenv[i]), mpo->site[i], B(pl.renv[i + 1]), Ml, d, Mr, ch.wbond[i], ch.wbond[i + 1]};
  CS(apply_op(c, lay, op, x, 0, nullptr, Bi()));
  CK(sum_partials(F64, c->ws + lay.Y, op.parts(), sz, sz, B(pl.G[k]), c->stream));
  if (i + 1 == n) {
    CK(mu_finish(B(pl.G[k]), nullptr, out, sz, c->stream));   // 5.
    return TDVP_OK;
  }
  CS(matmul(c, B(pl.G[k]), B(pl.pbuf[i + 1]), B(pl.X[k]), Ml * d, Mr, Mr));
  GemmArgs g{};   // T = L_i^H X  (Mr x Mr)
  g.A = A; g.B = B(pl.X[k]); g.C = B(pl.T[k]);
  g.M = Mr; g.N = Mr; g.K = Ml * d; g.batch = 1;
  g.sam = 1; g.sak = Mr; g.conjA = 1; g.sbk = Mr; g.sbn = 1; g.scm = Mr; g.scn = 1;
  CK(gemm_t(c, F64, F64, F64, g));
  CS(matmul(c, A, B(pl.T[k]), B(pl.Y[k]), Ml * d, Mr, Mr));
  CK(mu_finish(B(pl.X[k]), B(pl.Y[k]), out, sz, c->stream));
  return TDVP_OK;
}

// out[i] = d(site i)/dt for sites i0 <= i < i1 of the state A with the mean
// fields mu_fields last computed.  The site equations are independent, and
// each one's launches are small (a few dozen work-groups), so the sites go
// round-robin over MU_LANES streams forked from and joined to c->stream.
tdvp_status mu_site_rhs(tdvp_ctx *c, const MuPlan &pl, const tdvp_mpo *mpo, const double2 *const *A,
                        double2 *const *out, int i0, int i1) {
  const int lanes = std::max(1, std::min(MU_LANES, i1 - i0));
  hipStream_t main = c->stream;
  if (lanes > 1) {
    for (int k = 0; k < MU_LANES; ++k)
      if (!c->mu_ev[k]) CK(hipEventCreateWithFlags(&c->mu_ev[k], hipEventDisableTiming));
    for (int k = 0; k + 1 < MU_LANES; ++k)
      if (!c->mu_lane[k]) CK(hipStreamCreateWithFlags(&c->mu_lane[k], hipStreamNonBlocking));
    CK(hipEventRecord(c->mu_ev[0], main));
    for (int k = 1; k < lanes; ++k) CK(hipStreamWaitEvent(c->mu_lane[k - 1], c->mu_ev[0], 0));
  }
  tdvp_status st = TDVP_OK;
  for (int i = i0; i < i1 && st == TDVP_OK; ++i) {
    const int k = (i - i0) % lanes;
    c->stream = k == 0 ? main : c->mu_lane[k - 1];
    st = mu_site_one(c, pl, k, mpo, i, A[i], out[i]);
  }
  c->stream = main;
  for (int k = 1; k < lanes; ++k) {
    CK(hipEventRecord(c->mu_ev[k], c->mu_lane[k - 1]));
    CK(hipStreamWaitEvent(main, c->mu_ev[k], 0));
  }
  return st;
}

// out[i] = d(site i)/dt for the left-canonical state A (host tables of n device pointers).
tdvp_status mu_rhs_impl(tdvp_ctx *c, const MuPlan &pl, const tdvp_mpo *mpo, const double2 *const *A,
                        double2 *const *out, double eps) {
  CS(mu_fields(c, pl, mpo, A, eps));
  return mu_site_rhs(c, pl, mpo, A, out, 0, pl.ch.n);
}

tdvp_status mu_prepare(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, MuPlan *pl, int kmax = 1) {
  CS(mu_plan(ctx, mps, mpo, pl, kmax));
  if (!ctx->ws || ctx->ws_bytes < pl->total) return TDVP_E_WORKSPACE;
  CK(hipSetDevice(ctx->device));
  return TDVP_OK;
}

// Integrates dy/dt = f(y) from 0 to t_final on the packed vector y (N
// complex entries; initial values in place) with the Dormand-Prince 5(4)
// pair, using the plan's vectors 1..10 as stages; *res receives the buffer
// that holds the result (y itself or one of those vectors).
tdvp_status dp45(tdvp_ctx *ctx, const MuPlan &pl, double2 *y, int64_t N, double t_final, double rtol,
                 double atol, int max_steps, const std::function<tdvp_status(const double2 *, double2 *)> &f,
                 double2 **res, int64_t *nacc_out, int64_t *nrej_out) {
  auto V = [&](int k) { return reinterpret_cast<double2 *>(ctx->ws + pl.vec[k]); };
  double2 *ys = V(1), *ynew = V(2), *err = V(3);
  double2 *K[7];
  for (int j = 0; j < 7; ++j) K[j] = V(4 + j);
  double *part = reinterpret_cast<double *>(ctx->ws + pl.part);
  int64_t nacc = 0, nrej = 0;
  // RMS of (e / (atol + rtol max(|a|, |b|))) over the packed vector
  auto wnorm = [&](const double2 *e, const double2 *a, const double2 *b, double *res) -> tdvp_status {
    const int g = rk_err_partials(e, a, b, N, rtol, atol, part, ctx->stream);
    if (g < 0) return TDVP_E_DEVICE;
    std::vector<double> h(g);
    CK(hipMemcpyAsync(h.data(), part, g * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    double sum = 0.0;
    for (double v : h) sum += v;
    *res = std::sqrt(sum / (double)N);
    return TDVP_OK;
  };
  auto lin = [&](double2 *out, const double2 *x0, std::initializer_list<std::pair<double, const double2 *>> terms)
      -> tdvp_status {
    LinComb lc{};
    lc.out = out;
    lc.x0 = x0;
    for (const auto &t : terms) {
      if (t.first == 0.0) continue;
      lc.a[lc.m] = t.first;
      lc.x[lc.m] = t.second;
      ++lc.m;
    }
    CK(lincomb(lc, N, ctx->stream));
    return TDVP_OK;
  };
  // Dormand-Prince 5(4) tableau
  static const double A2[1] = {1.0 / 5};
  static const double A3[2] = {3.0 / 40, 9.0 / 40};
  static const double A4[3] = {44.0 / 45, -56.0 / 15, 32.0 / 9};
  static const double A5[4] = {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729};
  static const double A6[5] = {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656};
  static const double B5[6] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84};
  static const double E7[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                               22.0 / 525, -1.0 / 40};
  double t = 0.0;
  CS(f(y, K[0]));
  if (t_final > 0.0) {
    // first step from the two-evaluation rule (order 4 error estimate)
    double d0, d1, d2;
    CS(wnorm(y, y, y, &d0));
    CS(wnorm(K[0], y, y, &d1));
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = std::min(h0, t_final);
    CS(lin(ys, y, {{h0, K[0]}}));
    CS(f(ys, K[1]));
    CS(lin(err, K[1], {{-1.0, K[0]}}));
    CS(wnorm(err, y, y, &d2));
    d2 /= h0;
    const double h1 = (d1 <= 1e-15 && d2 <= 1e-15) ? std::max(1e-6, h0 * 1e-3)
                                                   : std::pow(0.01 / std::max(d1, d2), 1.0 / 5);
    double h = std::min(std::min(100 * h0, h1), t_final);
    bool rejected = false;
    while (t < t_final) {
      if (nacc + nrej >= max_steps) return TDVP_E_NUMERIC;
      const double min_step = 10.0 * std::fabs(std::nextafter(t, 2 * t_final + 1.0) - t);
      if (h < min_step) return TDVP_E_NUMERIC;
      double hs = h;
      if (t + hs > t_final) hs = t_final - t;
      CS(lin(ys, y, {{hs * A2[0], K[0]}}));
      CS(f(ys, K[1]));
      CS(lin(ys, y, {{hs * A3[0], K[0]}, {hs * A3[1], K[1]}}));
      CS(f(ys, K[2]));
      CS(lin(ys, y, {{hs * A4[0], K[0]}, {hs * A4[1], K[1]}, {hs * A4[2], K[2]}}));
      CS(f(ys, K[3]));
      CS(lin(ys, y, {{hs * A5[0], K[0]}, {hs * A5[1], K[1]}, {hs * A5[2], K[2]}, {hs * A5[3], K[3]}}));
      CS(f(ys, K[4]));
      CS(lin(ys, y, {{hs * A6[0], K[0]}, {hs * A6[1], K[1]}, {hs * A6[2], K[2]}, {hs * A6[3], K[3]},
                     {hs * A6[4], K[4]}}));
      CS(f(ys, K[5]));
      CS(lin(ynew, y, {{hs * B5[0], K[0]}, {hs * B5[2], K[2]}, {hs * B5[3], K[3]}, {hs * B5[4], K[4]},
                       {hs * B5[5], K[5]}}));
      CS(f(ynew, K[6]));
      CS(lin(err, nullptr, {{hs * E7[0], K[0]}, {hs * E7[2], K[2]}, {hs * E7[3], K[3]},
                            {hs * E7[4], K[4]}, {hs * E7[5], K[5]}, {hs * E7[6], K[6]}}));
      double en;
      CS(wnorm(err, y, ynew, &en));
      if (!std::isfinite(en)) return TDVP_E_NUMERIC;
      if (en < 1.0) {
        double fac = en == 0.0 ? 10.0 : std::min(10.0, 0.9 * std::pow(en, -0.2));
        if (rejected) fac = std::min(1.0, fac);
        t += hs;
        std::swap(y, ynew);
        std::swap(K[0], K[6]);        // first stage of the next step (FSAL)
        h = hs * fac;
        rejected = false;
        ++nacc;
      } else {
        h = hs * std::max(0.2, 0.9 * std::pow(en, -0.2));
        rejected = true;
        ++nrej;
      }
    }
  }
  *res = y;
  *nacc_out += nacc;
  *nrej_out += nrej;
  return TDVP_OK;
}

}  // namespace

extern "C" {

tdvp_status tdvp_mu_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                    size_t *bytes) {
  if (!bytes) return TDVP_E_ARG;
  MuPlan pl;
  CS(mu_plan(ctx, mps, mpo, &pl));
  *bytes = pl.total;
  return TDVP_OK;
}

tdvp_status tdvp_mu_rhs(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double eps,
                        void *const *out_site) {
  if (!out_site || !(eps > 0.0)) return TDVP_E_ARG;
  MuPlan pl;
  CS(mu_prepare(ctx, mps, mpo, &pl));
  const int n = pl.ch.n;
  std::vector<const double2 *> A(n);
  std::vector<double2 *> out(n);
  for (int i = 0; i < n; ++i) {
    if (!out_site[i]) return TDVP_E_ARG;
    A[i] = (const double2 *)mps->site[i];
    out[i] = (double2 *)out_site[i];
  }
  return mu_rhs_impl(ctx, pl, mpo, A.data(), out.data(), eps);
}

tdvp_status tdvp_mu_evolve(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double t_final,
                           double eps, double rtol, double atol, int max_steps, int64_t *stats) {
  if (!(t_final >= 0.0) || !(eps > 0.0) || !(rtol > 0.0) || !(atol >= 0.0) || max_steps < 1)
    return TDVP_E_ARG;
  MuPlan pl;
  CS(mu_prepare(ctx, mps, mpo, &pl));
  const int n = pl.ch.n;
  const int64_t N = pl.ntot;
  auto V = [&](int k) { return reinterpret_cast<double2 *>(ctx->ws + pl.vec[k]); };
  double2 *y = V(0);
  // site pointer tables into a packed vector
  auto sites_of = [&](double2 *v, std::vector<double2 *> &t) {
    t.resize(n);
    for (int i = 0; i < n; ++i) t[i] = v + pl.site_off[i];
  };
  for (int i = 0; i < n; ++i)
    CK(copy_c128(y + pl.site_off[i], (const double2 *)mps->site[i], pl.site_off[i + 1] - pl.site_off[i],
                 ctx->stream));
  int64_t nfev = 0, nacc = 0, nrej = 0;
  auto f = [&](const double2 *in, double2 *outv) -> tdvp_status {
    std::vector<double2 *> ti, to;
    sites_of(const_cast<double2 *>(in), ti);
    sites_of(outv, to);
    ++nfev;
    return mu_rhs_impl(ctx, pl, mpo, ti.data(), to.data(), eps);
  };
  CS(dp45(ctx, pl, y, N, t_final, rtol, atol, max_steps, f, &y, &nacc, &nrej));
  for (int i = 0; i < n; ++i)
    CK(copy_c128((double2 *)mps->site[i], y + pl.site_off[i], pl.site_off[i + 1] - pl.site_off[i],
                 ctx->stream));
  if (stats) {
    stats[0] = nacc;
    stats[1] = nrej;
    stats[2] = nfev;
  }
  return TDVP_OK;
}

tdvp_status tdvp_mu_cmf_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                        int kmax, size_t *bytes) {
  if (!bytes || kmax < 1 || kmax > KMAX) return TDVP_E_ARG;
  MuPlan pl;
  CS(mu_plan(ctx, mps, mpo, &pl, kmax));
  *bytes = pl.total;
  return TDVP_OK;
}

tdvp_status tdvp_mu_cmf_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double tau, double eps,
                             double rtol, double atol, int max_steps, int kmax, double tol, int64_t *stats) {
  if (!(tau > 0.0) || !(eps > 0.0) || !(rtol > 0.0) || !(atol >= 0.0) || max_steps < 1 || kmax < 1 ||
      kmax > KMAX || !(tol >= 0.0))
    return TDVP_E_ARG;
  MuPlan pl;
  CS(mu_prepare(ctx, mps, mpo, &pl, kmax));
  const Chain &ch = pl.ch;
  const int n = ch.n;
  const int64_t NL = pl.site_off[n - 1];   // the left-isometric sites lead the packed vector
  auto V = [&](int k) { return reinterpret_cast<double2 *>(ctx->ws + pl.vec[k]); };
  auto B = [&](size_t off) { return reinterpret_cast<double2 *>(ctx->ws + off); };
  double2 *y0 = V(11);
  for (int i = 0; i < n; ++i)
    CK(copy_c128(y0 + pl.site_off[i], (const double2 *)mps->site[i], pl.site_off[i + 1] - pl.site_off[i],
                 ctx->stream));
  auto table = [&](const double2 *v) {
    std::vector<const double2 *> t(n);
    for (int i = 0; i < n; ++i) t[i] = v + pl.site_off[i];
    return t;
  };
  int64_t nfev = 0, nacc = 0, nrej = 0;
  // frozen-field derivative of the sites 0 .. n-2
  auto f = [&](const double2 *in, double2 *outv) -> tdvp_status {
    const std::vector<const double2 *> ti = table(in);
    std::vector<double2 *> to(n);
    for (int i = 0; i < n; ++i) to[i] = outv + pl.site_off[i];
    ++nfev;
    return mu_site_rhs(ctx, pl, mpo, ti.data(), to.data(), 0, n - 1);
  };
  // the start state carried over time h with the fields last computed
  auto propagate = [&](double h, double2 **res) -> tdvp_status {
    double2 *y = V(0);
    CK(copy_c128(y, y0, pl.ntot, ctx->stream));
    CS(dp45(ctx, pl, y, NL, h, rtol, atol, max_steps, f, res, &nacc, &nrej));
    const Op op{B(pl.lenv[n - 1]), mpo->site[n - 1], B(pl.renv[n]), ch.bond[n - 1], ch.phys[n - 1],
                ch.bond[n], ch.wbond[n - 1], ch.wbond[n]};
    return run_lanczos(ctx, pl.lay, op, 0.0, -h, kmax, tol, y0 + NL, 0, *res + NL, 0, nullptr, Bi());
  };
  double2 *half = nullptr, *full = nullptr;
  CS(mu_fields(ctx, pl, mpo, table(y0).data(), eps));
  CS(propagate(0.5 * tau, &half));
  CS(mu_fields(ctx, pl, mpo, table(half).data(), eps));
  CS(propagate(tau, &full));
  for (int i = 0; i < n; ++i)
    CK(copy_c128((double2 *)mps->site[i], full + pl.site_off[i], pl.site_off[i + 1] - pl.site_off[i],
                 ctx->stream));
  if (stats) {
    stats[0] = nacc;
    stats[1] = nrej;
    stats[2] = nfev;
  }
  return TDVP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Two-site TDVP-PS (the two-site form of the projector splitting, Sec. II.A.2
// after eq:tdvp2_D): forward factors on pairs of sites with the merged
// two-site operator, a truncated SVD split (eq:SVD) after each, backward
// factors on the one-site centre.  Sweep order as in the one-site step;
// the two forward factors of the last pair are merged.
namespace {

struct Ps2Plan {
  Chain ch;
  Layout lay;          // local-problem region sized for the two-site problems
  size_t W2, X;        // merged MPO pair, two-site tensor
  size_t total;
};

tdvp_status ps2_plan(const tdvp_ctx *c, const tdvp_mps *mps, const tdvp_mpo *mpo, int kmax, Ps2Plan *pl) {
  if (!c || !mpo || kmax < 1 || kmax > KMAX) return TDVP_E_ARG;
  CS(check_chain(mps, mpo, &pl->ch));
  if (c->prec != TDVP_FP64) return TDVP_E_UNSUPPORTED;
  const Chain &ch = pl->ch;
  const int n = ch.n;
  if (n < 2) return TDVP_E_SHAPE;
  int64_t n2max = ch.nmax, w2max = 1;
  for (int i = 0; i + 1 < n; ++i) {
    const int64_t m = (int64_t)ch.bond[i] * ch.phys[i], k = (int64_t)ch.phys[i + 1] * ch.bond[i + 2];
    if (ch.bond[i + 1] > m || ch.bond[i + 1] > k) return TDVP_E_SHAPE;
    if (m > 64 || k > 64) return TDVP_E_UNSUPPORTED;       // the one-work-group SVD
    const int64_t D = (int64_t)ch.phys[i] * ch.phys[i + 1];
    if ((int64_t)std::max(ch.wbond[i], ch.wbond[i + 2]) * D > 1024) return TDVP_E_UNSUPPORTED;
    n2max = std::max(n2max, m * k);
    w2max = std::max(w2max, (int64_t)ch.wbond[i] * D * D * ch.wbond[i + 2]);
  }
  pl->lay = layout(n2max, ch.wmax, kmax, 16);
  size_t o = pl->lay.total;
  auto take = [&](size_t bytes) { const size_t r = o; o += al256(bytes); return r; };
  pl->W2 = take((size_t)w2max * 16);
  pl->X = take((size_t)n2max * 16);
  pl->total = o;
  return TDVP_OK;
}

}  // namespace

extern "C" {

tdvp_status tdvp_ps2_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, int kmax,
                                     size_t *bytes) {
  if (!bytes) return TDVP_E_ARG;
  Ps2Plan pl;
  CS(ps2_plan(ctx, mps, mpo, kmax, &pl));
  *bytes = pl.total;
  return TDVP_OK;
}

tdvp_status tdvp_svd_split(tdvp_ctx *ctx, const void *X, int m, int n, int keep, int mode, void *A, void *B,
                           double *discarded_dev) {
  if (!ctx || !X || !A || !B || (mode != 0 && mode != 1)) return TDVP_E_ARG;
  if (m < 1 || n < 1 || keep < 1 || keep > m || keep > n) return TDVP_E_SHAPE;
  if (m > 64 || n > 64) return TDVP_E_UNSUPPORTED;
  CK(hipSetDevice(ctx->device));
  CK(svd_split((const double2 *)X, m, n, keep, mode, (double2 *)A, (double2 *)B, discarded_dev, ctx->stream));
  return TDVP_OK;
}

tdvp_status tdvp_ps2_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, const tdvp_envs *envs,
                          double dt, int nsteps, int kmax, double tol, double *discarded_dev) {
  if (nsteps < 0 || !(tol >= 0.0) || !std::isfinite(dt) || !envs || !envs->left || !envs->right)
    return TDVP_E_ARG;
  Ps2Plan pl;
  CS(ps2_plan(ctx, mps, mpo, kmax, &pl));
  if (!ctx->ws || ctx->ws_bytes < pl.total) return TDVP_E_WORKSPACE;
  const Chain &ch = pl.ch;
  const int n = ch.n;
  for (int b = 0; b <= n; ++b)
    if (!envs->left[b] || !envs->right[b]) return TDVP_E_ARG;
  CK(hipSetDevice(ctx->device));
  const Layout &lay = pl.lay;
  hipStream_t st = ctx->stream;
  double2 *X = at<double2>(ctx, pl.X), *W2 = at<double2>(ctx, pl.W2);
  auto S = [&](int i) { return (double2 *)mps->site[i]; };
  auto W = [&](int i) { return (const double2 *)mpo->site[i]; };
  const double h = 0.5 * dt;
  // X = C_i A_{i+1}: (M_i d_i) x (M_{i+1}) times (M_{i+1}) x (d_{i+1} M_{i+2})
  auto pair = [&](int i) -> tdvp_status {
    CS(matmul(ctx, S(i), S(i + 1), X, ch.bond[i] * ch.phys[i], ch.bond[i + 1], ch.phys[i + 1] * ch.bond[i + 2]));
    CK(merge_mpo(W(i), W(i + 1), ch.wbond[i], ch.phys[i], ch.wbond[i + 1], ch.phys[i + 1], ch.wbond[i + 2], W2, st));
    return TDVP_OK;
  };
  auto forward2 = [&](int i, double t) -> tdvp_status {
    const Op op{envs->left[i], W2, envs->right[i + 2], ch.bond[i], ch.phys[i] * ch.phys[i + 1], ch.bond[i + 2],
                ch.wbond[i], ch.wbond[i + 2]};
    return run_lanczos(ctx, lay, op, 0.0, -t, kmax, tol, X, 0, X, 0, nullptr, Bi());
  };
  auto backward1 = [&](int i) -> tdvp_status {
    const Op op{envs->left[i], W(i), envs->right[i + 1], ch.bond[i], ch.phys[i], ch.bond[i + 1], ch.wbond[i],
                ch.wbond[i + 1]};
    return run_lanczos(ctx, lay, op, 0.0, +h, kmax, tol, S(i), 0, S(i), 0, nullptr, Bi());
  };
  auto split = [&](int i, int mode) -> tdvp_status {
    CK(svd_split(X, ch.bond[i] * ch.phys[i], ch.phys[i + 1] * ch.bond[i + 2], ch.bond[i + 1], mode, S(i), S(i + 1),
                 discarded_dev, st));
    return TDVP_OK;
  };
  auto left_env = [&](int i) {
    return env_update(ctx, lay, +1, envs->left[i], S(i), W(i), ch.bond[i], ch.phys[i], ch.bond[i + 1], ch.wbond[i],
                      ch.wbond[i + 1], envs->left[i + 1], Bi(), 0, 0, 0, 0);
  };
  auto right_env = [&](int i) {   // right[i] from right[i+1] and the right-isometric site i
    return env_update(ctx, lay, -1, envs->right[i + 1], S(i), W(i), ch.bond[i], ch.phys[i], ch.bond[i + 1],
                      ch.wbond[i], ch.wbond[i + 1], envs->right[i], Bi(), 0, 0, 0, 0);
  };
  ctx->klog_pos = 0;
  CK(fill_one(envs->left[0], F64, st));
  CK(fill_one(envs->right[n], F64, st));
  for (int s = 0; s < nsteps; ++s) {
    for (int i = 0; i + 1 < n; ++i) {          // left to right
      const bool last = i + 2 == n;
      CS(pair(i));
      CS(forward2(i, last ? dt : h));
      if (last) {                              // the turn: centre on the left site of the pair
        CS(split(i, 1));
        CS(right_env(i + 1));
        break;
      }
      CS(split(i, 0));
      CS(left_env(i));
      CS(backward1(i + 1));
    }
    for (int i = n - 3; i >= 0; --i) {         // right to left
      CS(backward1(i + 1));
      CS(pair(i));
      CS(forward2(i, h));
      CS(split(i, 1));
      CS(right_env(i + 1));
    }
  }
  return TDVP_OK;
}

}  // extern "C"
