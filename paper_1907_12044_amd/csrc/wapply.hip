// Stage 2 of the effective-Hamiltonian and environment contractions: the
// MPO site tensor W^{s' s}_{w w'} (eq:mpo) applied over the channel and
// physical indices,
//   out[wo][so][a][c] = sum_{wi, si} W(wo, so, si, wi) in[wi][si][a][c].
// An MPO of a sum of local terms is block sparse over (w, w'): for each
// output row (wo, so) the work-group first compacts the nonzero
// coefficients (in a fixed order, so results are deterministic), then every
// thread forms one (a, c) output from those few terms.  The pass is bound by
// HBM traffic (read in, write out); c is the fastest index on both sides.
#include "common.h"

namespace tdvp {

namespace {

constexpr int MAXNZ = 1024;
constexpr int WA_EPT = 8;   // outputs per thread and pass

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

template <typename T>
__device__ __forceinline__ void wapply_body(const WApplyArgs &p, const BlockXYZ &blk) {
  const int ri = blk.z;   // instance
  if (p.skip && p.skip[(int64_t)ri * p.inst.skip]) return;
  using V = typename Cplx<T>::type;
  __shared__ T cre[MAXNZ], cim[MAXNZ];
  __shared__ int cw[MAXNZ], cs[MAXNZ];
  __shared__ int nnz_s;
  const int d = p.d;
  const int wo = blk.y / d, so = blk.y % d;
  const int Win = p.w_in_right ? p.Wr : p.Wl;
  const double2 *W = reinterpret_cast<const double2 *>(p.W) + (int64_t)ri * p.inst.b;
  const int ncand = Win * d;
  // ordered compaction of nonzero coefficients by wave 0
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int base = 0;
    for (int c0 = 0; c0 < ncand; c0 += 64) {
      const int c = c0 + lane;
      double2 v = make_double2(0.0, 0.0);
      int wi = 0, si = 0;
      if (c < ncand) {
        wi = c / d;
        si = c % d;
        int64_t idx;
        if (p.w_in_right)   // W[wo][so][si][wi], shape (Wl, d, d, Wr)
          idx = (((int64_t)wo * d + so) * d + si) * p.Wr + wi;
        else                // W[wi][so][si][wo]
          idx = (((int64_t)wi * d + so) * d + si) * p.Wr + wo;
        v = W[idx];
      }
      const bool nz = (c < ncand) && (v.x != 0.0 || v.y != 0.0);
      const unsigned long long mask = __ballot(nz);
      const unsigned long long below = (lane == 0) ? 0ull : (mask & ((~0ull) >> (64 - lane)));
      const int pos = base + __popcll(below);
      if (nz && pos < MAXNZ) {
        cre[pos] = (T)v.x;
        cim[pos] = (T)v.y;
        cw[pos] = wi;
        cs[pos] = si;
      }
      base += __popcll(mask);
    }
    if (lane == 0) nnz_s = base < MAXNZ ? base : MAXNZ;
  }
  __syncthreads();
  const int nnz = nnz_s;
  const V *in = reinterpret_cast<const V *>(p.in) + (int64_t)ri * p.inst.a;
  V *out = reinterpret_cast<V *>(p.out) + (int64_t)ri * p.inst.c + (int64_t)wo * p.so_w + (int64_t)so * p.so_s;
  const int total = p.A * p.C;   // < 2^31 (checked by the launchers)
  // WA_EPT outputs per thread, 256 apart (coalesced): their input loads for
  // one nonzero are issued together, and the compaction above is shared by
  // 256 WA_EPT outputs.  Each output adds its terms in compaction order.
  for (int e0 = blk.x * (256 * WA_EPT) + threadIdx.x; e0 < total; e0 += blk.gx * (256 * WA_EPT)) {
    int64_t io[WA_EPT], oo[WA_EPT];
    bool ok[WA_EPT];
    T re[WA_EPT], im[WA_EPT];
#pragma unroll
    for (int u = 0; u < WA_EPT; ++u) {
      const int e = e0 + 256 * u;
      ok[u] = e < total;
      const int a = ok[u] ? e / p.C : 0, c = ok[u] ? e - a * p.C : 0;
      io[u] = (int64_t)a * p.si_a + (int64_t)c * p.si_c;
      oo[u] = (int64_t)a * p.so_a + (int64_t)c * p.so_c;
      re[u] = 0;
      im[u] = 0;
    }
    for (int t = 0; t < nnz; ++t) {
      const int64_t off = (int64_t)cw[t] * p.si_w + (int64_t)cs[t] * p.si_s;
      const T wr = cre[t], wi = cim[t];
      V v[WA_EPT];
#pragma unroll
      for (int u = 0; u < WA_EPT; ++u) {
        v[u].x = 0;
        v[u].y = 0;
        if (ok[u]) v[u] = in[io[u] + off];
      }
#pragma unroll
      for (int u = 0; u < WA_EPT; ++u) {
        re[u] += wr * v[u].x - wi * v[u].y;
        im[u] += wr * v[u].y + wi * v[u].x;
      }
    }
#pragma unroll
    for (int u = 0; u < WA_EPT; ++u) {
      if (ok[u]) {
        V o;
        o.x = re[u];
        o.y = im[u];
        out[oo[u]] = o;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void wapply_kernel(WApplyArgs p) {
  wapply_body<T>(p, native_block());
}
template <typename T>
__global__ __launch_bounds__(256) void wapply_grouped_kernel(Grp<WApplyArgs> g) {
  int k;
  const BlockXYZ b = g.locate(blockIdx.x, k);
  wapply_body<T>(g.a[k], b);
}

// grid of one argument set: x covers the (a, c) outputs (256 WA_EPT per
// work-group, at most 64 work-groups, grid-stride), y the output rows
// (wo, so), z the instances
bool wapply_grid(const WApplyArgs &a, dim3 &grid) {
  const int Wout = a.w_in_right ? a.Wl : a.Wr;
  const int64_t total = (int64_t)a.A * a.C;
  if (total <= 0 || Wout <= 0 || a.inst.count <= 0) return false;
  int gx = (int)((total + 256 * WA_EPT - 1) / (256 * WA_EPT));
  if (gx > 64) gx = 64;
  grid = dim3(gx, Wout * a.d, a.inst.count);
  return true;
}

}  // namespace

hipError_t wapply_grouped(DType t, const WApplyArgs *a, int ng, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  Grp<WApplyArgs> g;
  for (int k = 0; k < ng; ++k) {
    const int Win = a[k].w_in_right ? a[k].Wr : a[k].Wl;
    if (Win * a[k].d > MAXNZ || (int64_t)a[k].A * a[k].C >= (1ll << 31)) return hipErrorInvalidValue;
    dim3 gr;
    if (wapply_grid(a[k], gr)) g.add(a[k], gr.x, gr.y, gr.z);
  }
  if (g.ng == 0) return hipSuccess;
  if (t == F64)
    hipLaunchKernelGGL(wapply_grouped_kernel<double>, dim3(g.blocks()), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(wapply_grouped_kernel<float>, dim3(g.blocks()), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t wapply(DType t, const WApplyArgs &a, hipStream_t s) {
  const int Wout = a.w_in_right ? a.Wl : a.Wr;
  const int Win = a.w_in_right ? a.Wr : a.Wl;
  if (Win * a.d > MAXNZ || (int64_t)a.A * a.C >= (1ll << 31)) return hipErrorInvalidValue;
  (void)Wout;
  dim3 grid;
  if (!wapply_grid(a, grid)) return hipSuccess;
  if (t == F64)
    hipLaunchKernelGGL(wapply_kernel<double>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(wapply_kernel<float>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tdvp
