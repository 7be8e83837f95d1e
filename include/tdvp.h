/*
 * tdvp.h -- C ABI of libtdvp: one-site TDVP projector-splitting (TDVP-PS) time
 * evolution of a matrix product state on one AMD MI355X (gfx950) GPU.
 *
 * Problem statement (Li, Ren, Shuai, "Numerical Assessment for Accuracy and
 * GPU Acceleration of TD-DMRG Time Evolution Schemes"):
 *   MPS  |psi> = sum A^{s_1} A^{s_2} ... A^{s_N}               (Sec. II.A, eq:mps)
 *   MPO  H     = sum W^{s'_1 s_1} ... W^{s'_N s_N}             (Sec. II.A, eq:mpo)
 *   environments h[1:i-1], h[i+1:N]                           (eq:tdvp1_h1i, eq:tdvp1_hiN, eq:tdvp1_h)
 *   forward site equation  i dC/dt = H[i] C                   (eq:tdvp2_C, eq:tdvp1_H)
 *   backward bond equation i dD/dt = h[1:i] h[i+1:N] D         (eq:tdvp2_D)
 *   symmetric splitting of exp(-i P H tau)                    (eq:ps_trotter)
 *
 * Conventions
 *  - Sites are numbered 0..n-1, bonds 0..n; site i sits between bonds i and
 *    i+1.  bond[0] = bond[n] = 1 for both the MPS and the MPO.
 *  - Complex numbers are stored interleaved (re, im).  "c128" = two doubles,
 *    "c64" = two floats.  All arrays are row-major (last index fastest).
 *  - MPS site tensor i: c128 (bond[i], phys[i], bond[i+1]).
 *  - MPO site tensor i: c128 (W_i, d_out, d_in, W_{i+1}); d_out is the bra
 *    (row) index s' of W^{s' s} in eq:mpo.
 *  - Environment at bond b: (M_b, W_b, M_b) indexed [bra, channel, ket], bra
 *    conjugated (eq:tdvp1_h).  left[b] contracts sites 0..b-1, right[b]
 *    contracts sites b..n-1; left[0] = right[n] = 1.  Element type: c128 in
 *    TDVP_FP64 mode, c64 in the mixed modes.
 *  - Every pointer to tensor data is DEVICE memory owned by the caller; the
 *    library never allocates, frees or keeps it beyond the call, except the
 *    workspace passed to tdvp_set_workspace, which must stay valid while
 *    the context uses it.  Descriptor arrays (phys, bond, site pointer
 *    tables) are HOST memory, read during the call only.
 *  - Every call is asynchronous on the context's HIP stream unless stated
 *    otherwise; results are ready after the stream is synchronised.
 *  - Errors: argument and shape errors return at once and enqueue nothing.
 *    A failed HIP call returns TDVP_E_DEVICE.  No C++ exception crosses the
 *    ABI.  A context is not thread safe; use one per host thread.
 *  - Non-finite values: a Lanczos solve whose start vector or any Krylov
 *    norm is NaN or Inf stops, writes NaN to its output (a zero start
 *    vector still gives a zero output) and raises a sticky device flag in
 *    the context's workspace; tdvp_observe / tdvp_observe_batched report
 *    it, or a non-finite observable, as TDVP_E_NUMERIC.  The flag is
 *    cleared only by tdvp_set_workspace.
 */
#ifndef TDVP_H
#define TDVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDVP_OK = 0,
  TDVP_E_ARG = 1,        /* null pointer, negative size, bad enum           */
  TDVP_E_SHAPE = 2,      /* inconsistent bond / phys / channel dimensions   */
  TDVP_E_DEVICE = 3,     /* a HIP runtime call failed                       */
  TDVP_E_WORKSPACE = 4,  /* no workspace set, or too small for the call     */
  TDVP_E_NUMERIC = 5,    /* a non-finite value reported by tdvp_observe      */
  TDVP_E_UNSUPPORTED = 6 /* sizes beyond the compiled limits                */
} tdvp_status;

typedef enum {
  TDVP_FP64 = 0,  /* every contraction in FP64 (complex128)                   */
  TDVP_FP32 = 1,  /* contractions and environments in FP32 (complex64) with
                     FP32 accumulation; Lanczos orthogonalisation, norms,
                     the small exponential, QR and the MPS stay FP64          */
  TDVP_BF16X3 = 2 /* as TDVP_FP32, but the tiled GEMMs of the contractions run
                     on the bf16 matrix cores with each FP32 operand split
                     into two bf16 parts and three products per real product
                     (FP32 accumulation, ~17 significant bits per operand);
                     the fused small-bond Lanczos step stays FP32             */
} tdvp_precision;

typedef struct tdvp_ctx tdvp_ctx;

/* MPS descriptor (eq:mps).  site[i]: device c128 (bond[i], phys[i], bond[i+1]). */
typedef struct {
  int32_t n;
  const int32_t *phys;   /* host [n]   */
  const int32_t *bond;   /* host [n+1] */
  void *const *site;     /* host [n] of device pointers */
} tdvp_mps;

/* MPO descriptor (eq:mpo).  site[i]: device c128 (bond[i], phys[i], phys[i], bond[i+1]).
 * energy_shift: constant removed from H, added back by tdvp_observe. */
typedef struct {
  int32_t n;
  const int32_t *phys;   /* host [n]   (must equal the MPS phys) */
  const int32_t *bond;   /* host [n+1] channel dims W_b          */
  const void *const *site;
  double energy_shift;
} tdvp_mpo;

/* Environments (eq:tdvp1_h1i, eq:tdvp1_hiN): host tables of n+1 device
 * pointers each; left[b] and right[b] have (bond_mps[b], bond_mpo[b], bond_mps[b]). */
typedef struct {
  void *const *left;
  void *const *right;
} tdvp_envs;

/* Create a context on HIP device `device`, bound to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *ctx receives the handle. */
tdvp_status tdvp_create(tdvp_ctx **ctx, int device, void *hip_stream, tdvp_precision prec);
tdvp_status tdvp_destroy(tdvp_ctx *ctx);
tdvp_status tdvp_set_stream(tdvp_ctx *ctx, void *hip_stream);
const char *tdvp_status_string(tdvp_status s);
/* Bytes per environment element for the context's precision (16 or 8). */
int tdvp_env_elem_bytes(const tdvp_ctx *ctx);

/* Workspace bytes needed to run every call below on this chain with
 * Krylov dimension up to kmax (1 <= kmax <= 32).  Host-only computation. */
tdvp_status tdvp_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 int kmax, size_t *bytes);
/* Hand the context a device workspace of `bytes` bytes (256-byte aligned).
 * Enqueues its initialisation on the stream (clears the non-finite flag). */
tdvp_status tdvp_set_workspace(tdvp_ctx *ctx, void *dev, size_t bytes);

/* Environment update (eq:tdvp1_h with A = L or R, one site at a time).
 * dir = +1: env_out = h[1:i] from env_in = h[1:i-1] and the left-canonical
 *           site tensor A (Ml, d, Mr); env_in (Ml, Wl, Ml), env_out (Mr, Wr, Mr).
 * dir = -1: env_out = h[i:N] from env_in = h[i+1:N] and the right-canonical
 *           A (Ml, d, Mr); env_in (Mr, Wr, Mr), env_out (Ml, Wl, Ml).
 * A is c128; W is the MPO site tensor (Wl, d, d, Wr); envs use the context's
 * element type.  env_out must not alias env_in. */
tdvp_status tdvp_env_update(tdvp_ctx *ctx, int dir, const void *env_in, const void *A,
                            const void *W, int Ml, int d, int Mr, int Wl, int Wr, void *env_out);

/* Effective-Hamiltonian application.
 * W != NULL: y = H[i] x with H[i] = h[1:i-1] W h[i+1:N] (eq:tdvp1_H, eq:tdvp2_C);
 *   Lenv (Ml, Wl, Ml), Renv (Mr, Wr, Mr), x, y c128 (Ml, d, Mr).
 * W == NULL: the bond operator of eq:tdvp2_D, y = sum_w Lenv[:,w,:] x Renv[:,w,:]^T;
 *   d must be 1, Wl == Wr, x and y c128 (Ml, Mr).
 * y must not alias x. */
tdvp_status tdvp_heff_apply(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv,
                            int Ml, int d, int Mr, int Wl, int Wr, const void *x, void *y);

/* Krylov propagator y = exp(z Heff) x (Sec. II.A.2, local integrator of
 * eq:tdvp2_C / eq:tdvp2_D): Lanczos with full FP64 reorthogonalisation,
 * k <= min(kmax, dim) vectors, stop at breakdown beta_j <= 1e-12 |Heff v_j|
 * or, if tol > 0, when |z beta_j [exp(z T_k) e_1]_k| < tol; the small
 * exponential exp(z T_k) e_1 is evaluated on the device in FP64.
 * Operator arguments as in tdvp_heff_apply (W == NULL: bond operator).
 * x and y are c128 and may alias.  k_used_dev (device int32, may be NULL)
 * receives the number of Krylov vectors used. */
tdvp_status tdvp_lanczos_expm(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv,
                              int Ml, int d, int Mr, int Wl, int Wr, double z_re, double z_im,
                              int kmax, double tol, const void *x, void *y, int32_t *k_used_dev);

/* Variant of tdvp_lanczos_expm for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): same arguments and results, but the solve's scratch
 * memory is a fixed 64 MiB device array inside the library (one per GPU,
 * held until the process ends) instead of the context's workspace, so no
 * workspace needs to be set and nothing is allocated or freed.  Launches
 * only kernels on the context's stream (no memset, no event, no timing or
 * tuning).  TDVP_E_WORKSPACE if the problem's scratch (the size
 * tdvp_workspace_bytes gives for one site of these sizes) exceeds 64 MiB:
 * at kmax = 20 and W = 9, beyond n = Ml d Mr of about 66,000 in TDVP_FP64
 * and 84,000 in the mixed modes (every site of the bond-dimension-64
 * chains fits; 128 x 8 x 128 does not).
 * Every call on one GPU shares that GPU's array: calls that overlap on the
 * same GPU (other streams, other contexts, other host threads) race, and
 * the non-finite flag of a call is not reported by tdvp_observe. */
tdvp_status tdvp_lanczos_expm_noalloc(tdvp_ctx *ctx, const void *Lenv, const void *W, const void *Renv,
                                      int Ml, int d, int Mr, int Wl, int Wr, double z_re, double z_im,
                                      int kmax, double tol, const void *x, void *y, int32_t *k_used_dev);

/* Thin QR of a tall c128 matrix (eq:QR): A (m x n, m >= n, row-major) = Q R,
 * Q (m x n) with orthonormal columns, R (n x n) upper triangular with real
 * non-negative diagonal, n <= 256, all in FP64: Householder while the matrix
 * fits one work-group's LDS (m n <= 8704), else shifted Cholesky QR in three
 * passes (Gram matrix, Cholesky factor and its inverse, Q = A R^{-1}).
 * Q and R row-major; Q may alias A.  TDVP_E_SHAPE if n < 1 or m < n,
 * TDVP_E_UNSUPPORTED if n > 256. */
tdvp_status tdvp_qr(tdvp_ctx *ctx, const void *A, int m, int n, void *Q, void *R);

/* Right-canonicalise an MPS in place (RQ sweep n-1 -> 1, Sec. II.A) and
 * normalise the centre tensor at site 0. */
tdvp_status tdvp_right_canonicalize(tdvp_ctx *ctx, const tdvp_mps *mps);

/* Left-canonicalise an MPS in place (QR sweep 0 -> n-2, eq:QR: site i =
 * Q R, Q kept, R absorbed into site i+1) and normalise the centre tensor
 * at site n-1: the gauge of the TDVP-MU state.  Every site must satisfy
 * bond[i] * phys[i] >= bond[i+1] (TDVP_E_SHAPE otherwise). */
tdvp_status tdvp_left_canonicalize(tdvp_ctx *ctx, const tdvp_mps *mps);

/* Build every right environment right[n-1..1] of a right-canonical MPS and
 * set left[0] = right[n] = 1 (left[1..n-1] are produced by the sweep). */
tdvp_status tdvp_envs_build(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                            const tdvp_envs *envs);

/* nsteps symmetric TDVP-PS steps of size dt (eq:ps_trotter): a left-to-right
 * then a right-to-left sweep with dt/2, the two forward factors on the last
 * site merged into one exp(-i dt H[n-1]).  Entry and exit: right-canonical
 * MPS, centre at site 0, right[1..n-1] valid for it.  kmax/tol as in
 * tdvp_lanczos_expm.  MPS tensors and environments are updated in place. */
tdvp_status tdvp_ps_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                         const tdvp_envs *envs, double dt, int nsteps, int kmax, double tol);

/* Graph mode (enable != 0): tdvp_ps_step captures one whole step into a HIP
 * graph the first time it sees a given set of buffers, sizes, dt, kmax and
 * tol, and replays that graph for every later step with the same
 * arguments (the captured kernels read the buffers in place, so the caller
 * must keep them alive).  The context's stream must not be the NULL stream.
 * Steps run eagerly while a Krylov log or kernel timing is active. */
tdvp_status tdvp_set_graph(tdvp_ctx *ctx, int enable);

/* Kernel path of the local Lanczos solves (eq:tdvp2_C, eq:tdvp2_D).  With
 * enable != 0 (the default) a solve whose bond dimensions are small enough
 * (right bond dimension <= 64, MPO bonds <= 16, and the tiles of the
 * work-groups that share an output column fit in LDS) and whose batch has
 * fewer than 256 output columns in all (right bond dimension times the
 * number of instances solved together) runs each Krylov step
 * as two kernels: the fused H x with its projections, then the
 * orthogonalisation.  enable = 0 forces the general path (three contraction
 * kernels, projections, orthogonalisation) for every solve.  Both paths
 * compute the same quantities; results differ by rounding order only. */
tdvp_status tdvp_set_fused(tdvp_ctx *ctx, int enable);

/* Split of the last contraction of H[i] x on the general path (the sum over
 * the pairs (w_l, l) of the left MPO channel and the left bond index,
 * eq:tdvp1_h).  per_channel = 0 (the default): one part for a batch of 8
 * or more instances (the projections then run in the GEMM's epilogue),
 * otherwise as few equal parts as give the launch about four 32 x 32
 * output tiles per compute unit; per_channel != 0: one part per left MPO
 * channel.  The parts are added by the projection kernel.  Both
 * settings compute the same quantity; results differ by rounding order
 * only. */
tdvp_status tdvp_set_stage3_split(tdvp_ctx *ctx, int per_channel);

/* Autotuner for the tile shapes of the contraction GEMMs (a production
 * pattern, not part of the paper's method).  With enable != 0, the first
 * time a GEMM problem key (types, M, N, K, batch, instance count, operand
 * layout, precision) is met outside a graph capture, the candidate tile
 * shapes (32x32 with K steps of 32; 64x64 with K steps of 16, and in FP32
 * arithmetic also 32 and 64) are each run six times on the context stream
 * and timed with HIP events (the host waits for them); the built-in choice
 * is kept unless another shape is at least 3 % faster, and the choice is
 * kept in the context for every later launch of that key, captured graphs
 * included.  The candidates compute the same products; results differ by
 * rounding order only, so a tuned run agrees with an untuned one to
 * round-off, not bit for bit.  With a step graph enabled, the step that
 * meets new keys runs eagerly and the graph is captured after it.  The
 * fused small-bond Lanczos step keeps its built-in split (its cost depends
 * on the Krylov index, which a one-shot timing cannot see).  Default: off. */
tdvp_status tdvp_set_autotune(tdvp_ctx *ctx, int enable);
/* Number of problem keys the autotuner has decided so far (host int). */
tdvp_status tdvp_autotune_count(const tdvp_ctx *ctx, int32_t *count);

/* Observables of a right-canonical MPS (Sec. III.A): out_dev (device double
 * [2 + n_el]) receives <psi|psi>, <psi|H|psi> + energy_shift * <psi|psi>, and
 * the populations <psi|a+_m a_m|psi> of the electronic sites el_sites[m]
 * (host array of site indices; local dim 2, level 1 = occupied).  Not
 * divided by the norm.  Needs envs->right[1] valid.  This is the one call
 * of a time loop that waits for the stream: after the observables it
 * checks the context's non-finite flag and the values it wrote, and
 * returns TDVP_E_NUMERIC if any is NaN or Inf (out_dev is written either
 * way). */
tdvp_status tdvp_observe(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                         const tdvp_envs *envs, const int32_t *el_sites, int n_el,
                         double *out_dev);

/* Krylov log: while set, every Lanczos solve of tdvp_ps_step writes its
 * Krylov dimension to dev[slot] (device int32), slots counted from 0 at the
 * start of each tdvp_ps_step call in launch order (2n - 1 forward and
 * 2n - 2 backward solves per step); solves beyond `capacity` are not logged.
 * capacity = 0 switches the log off. */
tdvp_status tdvp_set_krylov_log(tdvp_ctx *ctx, int32_t *dev, int capacity);

/* Kernel timing for roofline reports.  tdvp_profile(ctx, cls) starts
 * recording HIP events on the context stream around every later launch of
 * kernel class cls (0 = off), together with the algorithmic FLOP and HBM
 * bytes of each launch (operands read once, results written once).
 * tdvp_profile_read synchronises the stream and returns the summed event
 * time (ms), the launch count and the summed FLOP and bytes. */
enum {
  TDVP_PROF_OFF = 0,
  TDVP_PROF_GEMM = 1,       /* complex MFMA contractions outside H x: environment
                               updates, centre moves, observables (cgemm_kernel) */
  TDVP_PROF_WAPPLY = 2,     /* MPO channel stage (wapply_kernel)                */
  TDVP_PROF_LZ_DOTS = 3,    /* Lanczos projections (lz_dots_kernel)             */
  TDVP_PROF_LZ_UPDATE = 4,  /* Lanczos orthogonalisation (lz_update_kernel)     */
  TDVP_PROF_LZ_ENDS = 5,    /* Lanczos start and final combination + exp(zT)e1  */
  TDVP_PROF_QR = 6,         /* Householder QR (qr_* kernels)                    */
  TDVP_PROF_LZ_FUSED = 7,   /* fused H x + projections (heff_small_kernel)      */
  TDVP_PROF_GEMM_HEFF = 8   /* the GEMM stages of H[i] x and of the bond operator
                               on the general path (cgemm_kernel)              */
};
tdvp_status tdvp_profile(tdvp_ctx *ctx, int kernel_class);
/* Repeat count for timed launches of the classes whose launches overwrite
 * outputs they do not read (TDVP_PROF_GEMM, TDVP_PROF_GEMM_HEFF,
 * TDVP_PROF_WAPPLY, TDVP_PROF_LZ_FUSED): each timed launch runs `reps` times back to back
 * between its two events and tdvp_profile_read divides by reps, so the time
 * per launch is the kernel's duration plus the gap between two queued
 * kernels rather than one whole dispatch.  1 <= reps <= 64 (default 1);
 * the results are those of one launch. */
tdvp_status tdvp_profile_reps(tdvp_ctx *ctx, int reps);
tdvp_status tdvp_profile_read(tdvp_ctx *ctx, double *ms, int64_t *launches, double *flops,
                              double *bytes);

/* Batched form of tdvp_ps_step / tdvp_observe for an ensemble of nb
 * independent chains of IDENTICAL shapes (phys, bond and MPO channel dims;
 * e.g. static-disorder realisations that share one bond dimension):
 * every kernel of the step covers all nb instances in one launch.
 * mps, mpo, envs are arrays of nb descriptors whose tensors must be laid
 * out at constant strides (instance r's tensor = instance 0's tensor +
 * r * stride, one stride per site / bond), as when each site tensor of the
 * ensemble is one (nb, ...) array; TDVP_E_ARG otherwise.  The workspace
 * must hold nb times tdvp_workspace_bytes of one chain.  Observables go to
 * out_dev[r * (2 + n_el) + ...] per instance.  Results per instance are
 * the single-chain results: bit for bit where the fused Lanczos step splits
 * a column the same way for nb chains as for one (always on the general
 * path; on the fused path the split count falls as nb grows, and results
 * then differ from a single run only in the order of one summation). */
tdvp_status tdvp_ps_step_batched(tdvp_ctx *ctx, int nb, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 const tdvp_envs *envs, double dt, int nsteps, int kmax, double tol);
tdvp_status tdvp_observe_batched(tdvp_ctx *ctx, int nb, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                 const tdvp_envs *envs, const int32_t *el_sites, int n_el,
                                 double *out_dev);

/* Two-site TDVP-PS (the two-site form of the projector splitting that
 * Sec. II.A.2 mentions after eq:tdvp2_D): nsteps symmetric steps of dt in
 * place.  Entry and exit gauge as tdvp_ps_step (right canonical, centre at
 * site 0, right environments valid; left[0] and right[n] are set here).
 * Left to right, pair i = 0 .. n-2: X = C_i A_{i+1} evolved by
 * exp(-i h H[i,i+1]) (h = dt/2; H[i,i+1] the operator of the two sites
 * with their MPO tensors merged, eq:tdvp1_H), split by an SVD truncated to
 * the bond's dimension (eq:SVD; A_i = U, C_{i+1} = Lam V^H), left
 * environment updated, C_{i+1} evolved back by exp(+i h H[i+1]); the last
 * pair takes exp(-i dt H) and splits with the centre on its left site.
 * Right to left, pair i = n-3 .. 0: C_{i+1} evolved back, X = A_i C_{i+1}
 * evolved forward, split (C_i = U Lam, B_{i+1} = V^H), right environment
 * updated.  Lanczos as tdvp_lanczos_expm (kmax, tol).  Bond dimensions stay
 * those of the MPS (the SVD chooses each bond's basis anew).
 * discarded_dev (device double, may be NULL): the squared singular values
 * dropped by every split are added to it (the caller zeroes it).
 * Limits: TDVP_FP64 contexts; every pair with bond[i] phys[i] <= 64 and
 * phys[i+1] bond[i+2] <= 64 (the SVD is a one-sided Jacobi in one
 * work-group) and max(W_i, W_{i+2}) phys[i] phys[i+1] <= 1024;
 * TDVP_E_UNSUPPORTED otherwise.  The workspace must hold
 * tdvp_ps2_workspace_bytes. */
tdvp_status tdvp_ps2_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, int kmax,
                                     size_t *bytes);
/* The split of the two-site step on its own (eq:SVD): X (device c128,
 * m x n row-major, 1 <= m, n <= 64) = U Lam V^H, the keep largest singular
 * values kept in descending order (1 <= keep <= min(m, n)); mode 0:
 * A = U (m x keep), B = Lam V^H (keep x n); mode 1: A = U Lam, B = V^H
 * (both row-major c128, device, not aliasing X).  The squared singular
 * values dropped are added to *discarded_dev (device double, may be NULL).
 * FP64 one-sided Jacobi in one work-group; enqueued on the context's
 * stream; no workspace. */
tdvp_status tdvp_svd_split(tdvp_ctx *ctx, const void *X, int m, int n, int keep, int mode, void *A, void *B,
                           double *discarded_dev);
tdvp_status tdvp_ps2_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, const tdvp_envs *envs,
                          double dt, int nsteps, int kmax, double tol, double *discarded_dev);

/* TDVP-MU (Sec. II.A.2, "TDVP-MU"): the equations of motion of a
 * left-canonical MPS (site tensors L_0 .. L_{n-2} left-isometric, the
 * centre C_{n-1} at the last site) with the matrix-unfolding
 * regularisation, integrated by the variable-mean-field scheme.
 * Right-hand side:
 *   dC_{n-1}/dt = -i H[n-1] C_{n-1}                              (eq:tdvp1_C)
 *   dL_i/dt     = -i (1 - L_i L_i^H) H[i](L_i D_i) V Lam~^{-1} U^H (eq:tdvp1_mu_L)
 * with D_i = U Lam V^H the bond matrix right of site i from an RQ sweep
 * of the state (eq:tdvp1_mu_rcano), H[i] built with environments in the
 * orthonormal right basis of that sweep, and Lam~ = Lam + sqrt(eps)
 * exp(-Lam / sqrt(eps)) (eq:reg2).  Canonicality is not re-imposed.
 * Limits: TDVP_FP64 contexts only, every bond dimension <= 64 (the
 * regularised inverse is a one-sided Jacobi SVD in one work-group);
 * TDVP_E_UNSUPPORTED otherwise.  The context workspace must hold
 * tdvp_mu_workspace_bytes (host-only computation). */
tdvp_status tdvp_mu_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                    size_t *bytes);
/* One evaluation of the right-hand side: out_site (host table of n device
 * pointers, c128, the shapes of the MPS sites, not aliasing them) receives
 * d(site i)/dt for the state mps.  eps > 0. */
tdvp_status tdvp_mu_rhs(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double eps,
                        void *const *out_site);
/* Integrate the MU equations from t = 0 to t_final (atomic time units) in
 * place, with the Dormand-Prince 5(4) pair: error per step measured as the
 * RMS of err / (atol + rtol max(|y|, |y_new|)) over every complex entry,
 * accepted when below 1, step factor 0.9 err^(-1/5) within [0.2, 10] (no
 * growth right after a rejection), first step from the two-evaluation
 * rule.  The host waits for the stream once per step (the accept/reject
 * decision).  stats (host int64[3], may be NULL): accepted steps, rejected
 * steps, right-hand-side evaluations.  TDVP_E_NUMERIC if the error becomes
 * non-finite, the step falls below the time resolution, or max_steps
 * steps (accepted + rejected) do not reach t_final; the state is then
 * left as it was at the start of the call. */
tdvp_status tdvp_mu_evolve(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double t_final,
                           double eps, double rtol, double atol, int max_steps, int64_t *stats);

/* TDVP-MU with the second-order constant-mean-field scheme (Sec. II.A.2,
 * the paragraph on VMF and CMF): one step of length tau > 0 in place.  The
 * mean fields of a site (its left and right environments, the bond matrix
 * D_i and the regularised inverse V Lam~^{-1} U^H) are taken at one state
 * and held; each site then obeys its own equation.  The fields of the
 * state at t carry every site to t + tau/2, the fields of that midpoint
 * state carry the state at t to t + tau.  The left-isometric sites follow
 *   dL_i/dt = -i (1 - L_i L_i^H) H[i](L_i D_i) V Lam~^{-1} U^H
 * with the frozen fields, integrated together on one packed vector by the
 * Dormand-Prince 5(4) pair of tdvp_mu_evolve (one step size for all
 * sites, error control over all of them; rtol, atol, max_steps per solve);
 * the centre follows its linear equation by the Lanczos propagator
 * exp(-i h H[n-1]) (Krylov dimension <= kmax, early stop at tol as in
 * tdvp_lanczos_expm).  Same limits as tdvp_mu_evolve; the workspace must
 * hold tdvp_mu_cmf_workspace_bytes for this kmax (1 <= kmax <= 32).  stats
 * (host int64[3], may be NULL): accepted and rejected Runge-Kutta steps
 * and site right-hand-side evaluations, summed over the two solves.
 * TDVP_E_NUMERIC as for tdvp_mu_evolve; the MPS then holds its start
 * state. */
tdvp_status tdvp_mu_cmf_workspace_bytes(const tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo,
                                        int kmax, size_t *bytes);
tdvp_status tdvp_mu_cmf_step(tdvp_ctx *ctx, const tdvp_mps *mps, const tdvp_mpo *mpo, double tau, double eps,
                             double rtol, double atol, int max_steps, int kmax, double tol, int64_t *stats);

/* Grouped form for an ensemble of UNEVEN bond dimensions (e.g. static-
 * disorder realisations whose bond dimensions are drawn from several
 * values): the nb = sum counts[q] chains are given group by group
 * (mps[0 .. counts[0]-1] form group 0, the next counts[1] group 1, ...;
 * 1 <= ngroups <= 4).  Inside a group the chains obey the rules of
 * tdvp_ps_step_batched (identical shapes, constant strides); across groups
 * the site count, physical dims and MPO channel dims must agree and the
 * MPS bond dims may differ (TDVP_E_SHAPE otherwise).  Every Krylov solve
 * of a sweep position is one launch sequence for all groups: per Krylov
 * step one fused-step launch covering the groups on the fused small-bond
 * path, one launch per contraction stage and one projection launch
 * covering the groups on the general path, and one orthogonalisation
 * launch covering every group (each launch reads a per-group argument
 * table); gauge shifts, environment updates and centre moves run per
 * group.  Groups whose bond dimensions all stay on the fused path and the
 * other groups form two lanes that run concurrently: the first on the
 * context stream, the second on an auxiliary stream of the context
 * (created on first use, default priority) forked from and joined to it
 * inside each call (parallel branches of the captured graph).  The GEMM tile of a grouped launch is the built-in choice of its
 * largest group (the autotuner is not consulted), so a group's results
 * agree with its own batched run to rounding order.  The workspace must
 * hold tdvp_workspace_bytes_grouped (groups laid out one after another);
 * the Krylov log is not written.  Graph mode as for tdvp_ps_step. */
tdvp_status tdvp_workspace_bytes_grouped(const tdvp_ctx *ctx, int ngroups, const int32_t *counts,
                                         const tdvp_mps *mps, const tdvp_mpo *mpo, int kmax,
                                         size_t *bytes);
tdvp_status tdvp_ps_step_grouped(tdvp_ctx *ctx, int ngroups, const int32_t *counts, const tdvp_mps *mps,
                                 const tdvp_mpo *mpo, const tdvp_envs *envs, double dt, int nsteps,
                                 int kmax, double tol);
/* Observables of every chain of a grouped ensemble, out_dev[r * (2 + n_el)]
 * in chain order r = 0 .. nb-1 (waits for the stream, as tdvp_observe). */
tdvp_status tdvp_observe_grouped(tdvp_ctx *ctx, int ngroups, const int32_t *counts, const tdvp_mps *mps,
                                 const tdvp_mpo *mpo, const tdvp_envs *envs, const int32_t *el_sites,
                                 int n_el, double *out_dev);

/* Frenkel-Holstein MPO (Sec. II.C, eq:holstein) written into HOST buffers.
 * Chain sites are given by kind[i] (0 = electronic two-level site, 1 = mode),
 * owner[i] (electronic index 0..n_e-1 the site belongs to) and phys[i].
 * eps[n_e] site energies and J[n_e*n_e] couplings, w[i] and g[i] the mode
 * frequency and dimensionless coupling of mode site i (ignored for electronic
 * sites), all in the energy unit of the caller.  The channel construction
 * uses complementary operators so that W_b = 2 + 2 min(k, n_e - k) + [inside
 * a mode block] with k electronic sites left of bond b.
 * Pass W_out = NULL to query: bond_out[n+1] and *total_elems (sum of site
 * tensor sizes in complex numbers) are filled.  Then call again with W_out
 * (host c128 of total_elems) to receive the tensors concatenated in site
 * order.  Host-only; no device needed. */
tdvp_status tdvp_holstein_mpo(int n, const int32_t *kind, const int32_t *owner, const int32_t *phys,
                              int n_e, const double *eps, const double *J, const double *w,
                              const double *g, int32_t *bond_out, int64_t *total_elems,
                              double *W_out);

#ifdef __cplusplus
}
#endif

#endif /* TDVP_H */
