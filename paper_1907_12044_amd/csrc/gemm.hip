// Complex GEMM on CDNA4 matrix cores (MFMA), FP64 or FP32 arithmetic.
//
// Every dense contraction of the TDVP-PS step (stages 1 and 3 of H[i] x,
// the bond operator of eq:tdvp2_D, the environment update eq:tdvp1_h and the
// centre move C_{i+1} = D R_{i+1}) is a (batched) complex GEMM with
// arbitrary strides.  A complex product is three real MFMAs on split
// real/imaginary planes held in LDS (the three-multiplication form):
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi);
//   Cr = P1 - P2,  Ci = P3 - P1 - P2.
// Tiles: a 256-thread work-group (4 wave64) owns a BM x BN output tile, each
// wave a (BM/2) x (BN/2) quarter built from 16x16 MFMA blocks
// (v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32).  Operand lane layout of
// the 16x16x4 shapes: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k;
// result D[i][j] in lane j + 16 (i / 4), register i % 4 for f32, but in lane
// j + 16 (i % 4), register i / 4 for f64.
#include <type_traits>

#include "common.h"

namespace tdvp {

namespace {

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { using type = f64x4; };
template <> struct Acc<float> { using type = f32x4; };

__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Lanczos projection epilogue of a stage-3 GEMM (GemmArgs::lzU): the tile's
// results w (rounded to the output type TC, as a stored C would be) go to
// basis vector j + 1 in FP64, and the work-group's partials <u_i, w>
// (i <= j) and |w|^2 to its slot (tile index) of the partial arrays.  The
// basis elements of the tile are read four vectors at a time, each wave
// sums its lanes and wave 0 adds the four waves in order (fixed order: the
// partials do not depend on timing).
template <typename TC, typename TM, int BM, int BN, typename AccT>
__device__ __forceinline__ void lz_epilogue(const GemmArgs &g, const BlockXYZ &blk, int ri,
                                            const AccT (&p1)[BM / 32][BN / 32],
                                            const AccT (&p2)[BM / 32][BN / 32],
                                            const AccT (&p3)[BM / 32][BN / 32]) {
  constexpr int TI = BM / 32, TJ = BN / 32;
  constexpr bool IS_F64 = sizeof(TM) == 8;
  constexpr int NE = TI * TJ * 4;          // results per lane
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);
  const int M = g.M, N = g.N;
  const int64_t n = (int64_t)M * N;
  double2 *U = reinterpret_cast<double2 *>(reinterpret_cast<char *>(g.lzU) + (int64_t)ri * g.lzwss);
  LzPartials *pp = reinterpret_cast<LzPartials *>(reinterpret_cast<char *>(g.lzpp) + (int64_t)ri * g.lzwss);
  const int jj = g.lzj;
  const int slot = blk.y * blk.gx + blk.x;
  double wr[NE], wi[NE];
  int64_t ei[NE];
  bool ok[NE];
  double w2 = 0.0;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = (i * TJ + j) * 4 + r;
        const int rr = IS_F64 ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r);
        const int row = blk.y * BM + wm0 + i * 16 + rr;
        const int col = blk.x * BN + wn0 + j * 16 + (lane & 15);
        ok[q] = row < M && col < N;
        ei[q] = (int64_t)row * N + col;
        const TC re = (TC)(p1[i][j][r] - p2[i][j][r]), im = (TC)(p3[i][j][r] - p1[i][j][r] - p2[i][j][r]);
        wr[q] = ok[q] ? (double)re : 0.0;
        wi[q] = ok[q] ? (double)im : 0.0;
        if (ok[q]) U[(int64_t)(jj + 1) * n + ei[q]] = make_double2(wr[q], wi[q]);
        w2 += wr[q] * wr[q] + wi[q] * wi[q];
      }
  auto wsum = [](double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
  };
  for (int i0 = 0; i0 <= jj; i0 += 4) {
    double dr[4], di[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dr[t] = 0.0;
      di[t] = 0.0;
      const int i = i0 + t;
      if (i <= jj) {
        const double2 *ui = U + (int64_t)i * n;
        double2 u[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) u[q] = ok[q] ? ui[ei[q]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          dr[t] += u[q].x * wr[q] + u[q].y * wi[q];
          di[t] += u[q].x * wi[q] - u[q].y * wr[q];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dr[t] = wsum(dr[t]);
      di[t] = wsum(di[t]);
    }
    __syncthreads();   // (red is reused by the next group of four)
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        red[wave][2 * t] = dr[t];
        red[wave][2 * t + 1] = di[t];
      }
    }
    __syncthreads();
    if (threadIdx.x < 4 && i0 + (int)threadIdx.x <= jj) {
      const int t = threadIdx.x;
      double a = 0.0, b = 0.0;
      for (int w = 0; w < 4; ++w) {
        a += red[w][2 * t];
        b += red[w][2 * t + 1];
      }
      pp->dot[i0 + t][slot] = make_double2(a, b);
    }
  }
  w2 = wsum(w2);
  __syncthreads();
  if (lane == 0) red[wave][0] = w2;
  __syncthreads();
  if (threadIdx.x == 0) {
    pp->w2[slot] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    if (slot == 0) pp->ndot = blk.gx * blk.gy;
  }
}

// FP64 arithmetic: at least two waves per SIMD (registers capped at 256
// per lane, the accumulators then stay in the architectural registers; the
// uncapped 64x64 tile took ~390 and ran one wave per SIMD, 22 % slower).
template <typename TA, typename TB, typename TC, typename TM, int BM, int BN, int BK, bool LZ = false>
__device__ __forceinline__ void cgemm_tile(const GemmArgs &g, const BlockXYZ &blk) {
  const int bz = blk.z % g.batch;           // batch index
  const int ri = blk.z / g.batch;           // instance index
  if (g.skip && g.skip[(int64_t)ri * g.inst.skip]) return;
  using VA = typename Cplx<TA>::type;
  using VB = typename Cplx<TB>::type;
  using VC = typename Cplx<TC>::type;
  using AccT = typename Acc<TM>::type;
  constexpr int PAD = 1;
  constexpr bool IS_F64 = sizeof(TM) == 8;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TI = WM / 16, TJ = WN / 16;
  __shared__ TM As[2][BK][BM + PAD];
  __shared__ TM Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bm0 = blk.y * BM;
  const int bn0 = blk.x * BN;
  const VA *A = reinterpret_cast<const VA *>(g.A) + (int64_t)bz * g.bsa + (int64_t)ri * g.inst.a;
  const VB *B = reinterpret_cast<const VB *>(g.B) + (int64_t)bz * g.bsb + (int64_t)ri * g.inst.b;
  VC *C = reinterpret_cast<VC *>(g.C) + (int64_t)bz * g.bsc + (int64_t)ri * g.inst.c;
  const int M = g.M, N = g.N, K = g.K;
  const bool a_kfast = (g.sak == 1);
  const bool b_nfast = (g.sbn == 1) || (g.sbk != 1);
  const TM sa = g.conjA ? TM(-1) : TM(1);
  const TM sb = g.conjB ? TM(-1) : TM(1);
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  AccT p1[TI][TJ], p2[TI][TJ], p3[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      p1[i][j] = AccT{0, 0, 0, 0};
      p2[i][j] = AccT{0, 0, 0, 0};
      p3[i][j] = AccT{0, 0, 0, 0};
    }

  // Register-staged tiles: the global loads of tile k0 + BK are issued
  // before the MFMAs of tile k0, so their latency overlaps the arithmetic.
  constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
  VA ra[NA];
  VB rb[NB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      int mm, kk;
      if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      const int gm = bm0 + mm, gk = k0 + kk;
      ra[q].x = 0;
      ra[q].y = 0;
      if (gm < M && gk < K) ra[q] = A[(int64_t)gm * g.sam + (int64_t)gk * g.sak];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      int kk, nn;
      if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      const int gn = bn0 + nn, gk = k0 + kk;
      rb[q].x = 0;
      rb[q].y = 0;
      if (gn < N && gk < K) rb[q] = B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn];
    }
  };
  load_tiles(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      int mm, kk;
      if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      As[0][kk][mm] = (TM)ra[q].x;
      As[1][kk][mm] = sa * (TM)ra[q].y;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      int kk, nn;
      if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      Bs[0][kk][nn] = (TM)rb[q].x;
      Bs[1][kk][nn] = sb * (TM)rb[q].y;
    }
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      TM ar[TI], ai[TI], as[TI], br[TJ], bi[TJ], bs[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        ar[i] = As[0][kr][wm0 + i * 16 + (lane & 15)];
        ai[i] = As[1][kr][wm0 + i * 16 + (lane & 15)];
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        br[j] = Bs[0][kr][wn0 + j * 16 + (lane & 15)];
        bi[j] = Bs[1][kr][wn0 + j * 16 + (lane & 15)];
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          p1[i][j] = mfma16(ar[i], br[j], p1[i][j]);
          p2[i][j] = mfma16(ai[i], bi[j], p2[i][j]);
          p3[i][j] = mfma16(as[i], bs[j], p3[i][j]);
        }
    }
    __syncthreads();
  }

  if (LZ) {
    lz_epilogue<TC, TM, BM, BN>(g, blk, ri, p1, p2, p3);
    return;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // output row inside the 16x16 block: f64 MFMA puts row 4 r + lane/16 in
        // register r, f32 MFMA row 4 (lane/16) + r (measured lane layouts)
        const int rr = IS_F64 ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r);
        const int row = bm0 + wm0 + i * 16 + rr;
        const int col = bn0 + wn0 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          TM re = p1[i][j][r] - p2[i][j][r], im = p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
          VC &dst = C[(int64_t)row * g.scm + (int64_t)col * g.scn];
          if (g.mode == 1) {
            re = (TM)dst.x - re;
            im = (TM)dst.y - im;
          } else if (g.mode == 2) {
            re = -re;
            im = -im;
          }
          VC v;
          v.x = (TC)re;
          v.y = (TC)im;
          dst = v;
        }
      }
}

template <typename TA, typename TB, typename TC, typename TM, int BM, int BN, int BK>
__global__ __launch_bounds__(256, sizeof(TM) == 8 ? 2 : 1) void cgemm_kernel(GemmArgs g) {
  cgemm_tile<TA, TB, TC, TM, BM, BN, BK>(g, native_block());
}
// with the Lanczos projection epilogue
template <typename TA, typename TB, typename TC, typename TM, int BM, int BN, int BK>
__global__ __launch_bounds__(256, sizeof(TM) == 8 ? 2 : 1) void cgemm_lz_kernel(GemmArgs g) {
  cgemm_tile<TA, TB, TC, TM, BM, BN, BK, true>(g, native_block());
}
template <typename TA, typename TB, typename TC, typename TM, int BM, int BN, int BK>
__global__ __launch_bounds__(256, sizeof(TM) == 8 ? 2 : 1) void cgemm_grouped_kernel(Grp<GemmArgs> gg) {
  int k;
  const BlockXYZ b = gg.locate(blockIdx.x, k);
  cgemm_tile<TA, TB, TC, TM, BM, BN, BK>(gg.a[k], b);
}

// Split-BF16 variant (FP32 accumulation): every real operand x is stored as
// x_hi = bf16(x) and x_lo = bf16(x - x_hi), so x = x_hi + x_lo to about
// 2^-17 |x|, and a real product is x_hi y_hi + x_hi y_lo + x_lo y_hi (the
// x_lo y_lo term, ~2^-18 |x y|, is dropped).  The complex product uses the
// same three real products as above; each is three bf16 MFMAs
// (v_mfma_f32_16x16x32_bf16, 32 terms of k per instruction), nine per complex
// 16x16x32 block.  The planes in LDS are [row][k] with k fastest (a lane's
// eight k values are one 16-byte read) and a row pitch of 40 so that the
// sixteen rows of a fragment fall in distinct banks.
// Operand lane layout (checked on the device): A[i][k] in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; the result as
// for v_mfma_f32_16x16x4_f32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// Two waves per SIMD (at most 256 registers per lane): uncapped, the 64x64
// tile took 288 and ran one wave per SIMD, 15 % slower at M = 256.
template <typename TA, typename TB, typename TC, int BM, int BN>
__device__ __forceinline__ void cgemm_bf3_tile(const GemmArgs &g, const BlockXYZ &blk) {
  const int bz = blk.z % g.batch;
  const int ri = blk.z / g.batch;
  if (g.skip && g.skip[(int64_t)ri * g.inst.skip]) return;
  using VA = typename Cplx<TA>::type;
  using VB = typename Cplx<TB>::type;
  using VC = typename Cplx<TC>::type;
  constexpr int BK = 32, KP = 40;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TI = WM / 16, TJ = WN / 16;
  // planes: re hi, re lo, im hi, im lo, (re + im) hi, (re + im) lo
  __shared__ __attribute__((aligned(16))) __bf16 As[6][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[6][BN][KP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bm0 = blk.y * BM;
  const int bn0 = blk.x * BN;
  const VA *A = reinterpret_cast<const VA *>(g.A) + (int64_t)bz * g.bsa + (int64_t)ri * g.inst.a;
  const VB *B = reinterpret_cast<const VB *>(g.B) + (int64_t)bz * g.bsb + (int64_t)ri * g.inst.b;
  VC *C = reinterpret_cast<VC *>(g.C) + (int64_t)bz * g.bsc + (int64_t)ri * g.inst.c;
  const int M = g.M, N = g.N, K = g.K;
  const bool a_kfast = (g.sak == 1);
  const bool b_nfast = (g.sbn == 1) || (g.sbk != 1);
  const float sa = g.conjA ? -1.f : 1.f;
  const float sb = g.conjB ? -1.f : 1.f;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  f32x4 p1[TI][TJ], p2[TI][TJ], p3[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      p1[i][j] = f32x4{0, 0, 0, 0};
      p2[i][j] = f32x4{0, 0, 0, 0};
      p3[i][j] = f32x4{0, 0, 0, 0};
    }

  constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
  // Operands contiguous in k (rows of A with sak = 1, columns of B with
  // sbk = 1) are staged four consecutive k per thread when K is a multiple
  // of 4: each plane then gets one 8-byte LDS store per four values instead
  // of four 2-byte stores.  Otherwise one element per thread.  (The same
  // values land in LDS either way.)
  const bool a_vec = a_kfast && K % 4 == 0;
  const bool b_vec = !b_nfast && K % 4 == 0;
  VA ra[NA];
  VB rb[NB];
  auto load_tiles = [&](int k0) {
    if (a_vec) {
#pragma unroll
      for (int q = 0; q < NA / 4; ++q) {
        const int c = tid + 256 * q, mm = c / (BK / 4), kk = 4 * (c % (BK / 4));
        const int gm = bm0 + mm, gk = k0 + kk;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ra[4 * q + u].x = 0;
          ra[4 * q + u].y = 0;
        }
        if (gm < M && gk < K) {
          const VA *src = A + (int64_t)gm * g.sam + gk;
#pragma unroll
          for (int u = 0; u < 4; ++u) ra[4 * q + u] = src[u];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int e = tid + 256 * q;
        int mm, kk;
        if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
        const int gm = bm0 + mm, gk = k0 + kk;
        ra[q].x = 0;
        ra[q].y = 0;
        if (gm < M && gk < K) ra[q] = A[(int64_t)gm * g.sam + (int64_t)gk * g.sak];
      }
    }
    if (b_vec) {
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) {
        const int c = tid + 256 * q, nn = c / (BK / 4), kk = 4 * (c % (BK / 4));
        const int gn = bn0 + nn, gk = k0 + kk;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rb[4 * q + u].x = 0;
          rb[4 * q + u].y = 0;
        }
        if (gn < N && gk < K) {
          const VB *src = B + (int64_t)gn * g.sbn + gk;
#pragma unroll
          for (int u = 0; u < 4; ++u) rb[4 * q + u] = src[u];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int e = tid + 256 * q;
        int nn, kk;
        if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
        const int gn = bn0 + nn, gk = k0 + kk;
        rb[q].x = 0;
        rb[q].y = 0;
        if (gn < N && gk < K) rb[q] = B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn];
      }
    }
  };
  load_tiles(0);
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += BK) {
    if (a_vec) {
#pragma unroll
      for (int q = 0; q < NA / 4; ++q) {
        const int c = tid + 256 * q, mm = c / (BK / 4), kk = 4 * (c % (BK / 4));
        bf16x4 h[6];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float xr = (float)ra[4 * q + u].x, xi = sa * (float)ra[4 * q + u].y;
          __bf16 hi, lo;
          split_bf16(xr, hi, lo);
          h[0][u] = hi;
          h[1][u] = lo;
          split_bf16(xi, hi, lo);
          h[2][u] = hi;
          h[3][u] = lo;
          split_bf16(xr + xi, hi, lo);
          h[4][u] = hi;
          h[5][u] = lo;
        }
#pragma unroll
        for (int pl = 0; pl < 6; ++pl) *reinterpret_cast<bf16x4 *>(&As[pl][mm][kk]) = h[pl];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int e = tid + 256 * q;
        int mm, kk;
        if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
        const float xr = (float)ra[q].x, xi = sa * (float)ra[q].y;
        split_bf16(xr, As[0][mm][kk], As[1][mm][kk]);
        split_bf16(xi, As[2][mm][kk], As[3][mm][kk]);
        split_bf16(xr + xi, As[4][mm][kk], As[5][mm][kk]);
      }
    }
    if (b_vec) {
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) {
        const int c = tid + 256 * q, nn = c / (BK / 4), kk = 4 * (c % (BK / 4));
        bf16x4 h[6];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float yr = (float)rb[4 * q + u].x, yi = sb * (float)rb[4 * q + u].y;
          __bf16 hi, lo;
          split_bf16(yr, hi, lo);
          h[0][u] = hi;
          h[1][u] = lo;
          split_bf16(yi, hi, lo);
          h[2][u] = hi;
          h[3][u] = lo;
          split_bf16(yr + yi, hi, lo);
          h[4][u] = hi;
          h[5][u] = lo;
        }
#pragma unroll
        for (int pl = 0; pl < 6; ++pl) *reinterpret_cast<bf16x4 *>(&Bs[pl][nn][kk]) = h[pl];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int e = tid + 256 * q;
        int nn, kk;
        if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
        const float yr = (float)rb[q].x, yi = sb * (float)rb[q].y;
        split_bf16(yr, Bs[0][nn][kk], Bs[1][nn][kk]);
        split_bf16(yi, Bs[2][nn][kk], Bs[3][nn][kk]);
        split_bf16(yr + yi, Bs[4][nn][kk], Bs[5][nn][kk]);
      }
    }
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
    bf16x8 a[TI][6], b[TJ][6];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) a[i][pl] = *reinterpret_cast<const bf16x8 *>(&As[pl][wm0 + 16 * i + fr][fk]);
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) b[j][pl] = *reinterpret_cast<const bf16x8 *>(&Bs[pl][wn0 + 16 * j + fr][fk]);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], p1[i][j], 0, 0, 0);
        p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], p1[i][j], 0, 0, 0);
        p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], p1[i][j], 0, 0, 0);
        p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], b[j][2], p2[i][j], 0, 0, 0);
        p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][3], p2[i][j], 0, 0, 0);
        p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][2], p2[i][j], 0, 0, 0);
        p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][5], b[j][4], p3[i][j], 0, 0, 0);
        p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][4], b[j][5], p3[i][j], 0, 0, 0);
        p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][4], b[j][4], p3[i][j], 0, 0, 0);
      }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        const int col = bn0 + wn0 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          VC v;
          v.x = (TC)(p1[i][j][r] - p2[i][j][r]);
          v.y = (TC)(p3[i][j][r] - p1[i][j][r] - p2[i][j][r]);
          C[(int64_t)row * g.scm + (int64_t)col * g.scn] = v;
        }
      }
}

template <typename TA, typename TB, typename TC, int BM, int BN>
__global__ __launch_bounds__(256, 2) void cgemm_bf3_kernel(GemmArgs g) {
  cgemm_bf3_tile<TA, TB, TC, BM, BN>(g, native_block());
}
template <typename TA, typename TB, typename TC, int BM, int BN>
__global__ __launch_bounds__(256, 2) void cgemm_bf3_grouped_kernel(Grp<GemmArgs> gg) {
  int k;
  const BlockXYZ b = gg.locate(blockIdx.x, k);
  cgemm_bf3_tile<TA, TB, TC, BM, BN>(gg.a[k], b);
}

template <typename TA, typename TB, typename TC>
hipError_t launch_bf3(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.inst.count <= 0) return hipSuccess;
  const int nz = g.batch * g.inst.count;
  const int64_t tiles64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
  if (g.tile == 64 || (g.tile == 0 && tiles64 >= 240)) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz);
    hipLaunchKernelGGL((cgemm_bf3_kernel<TA, TB, TC, 64, 64>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, nz);
    hipLaunchKernelGGL((cgemm_bf3_kernel<TA, TB, TC, 32, 32>), grid, dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename TM>
hipError_t launch(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.inst.count <= 0) return hipSuccess;
  if (g.lzU) {
    // the projection epilogue: C = A B for one batch, row-major, at most
    // LZ_PARTS tiles of the smallest shape, same element types throughout
    constexpr bool same = std::is_same<TA, TB>::value && std::is_same<TB, TC>::value &&
                          std::is_same<TC, TM>::value;
    if (!same || g.mode != 0 || g.batch != 1 || g.scn != 1 || g.scm != g.N || !g.lzpp ||
        (int64_t)((g.M + 31) / 32) * ((g.N + 31) / 32) > LZ_PARTS || g.lzj < 0 || g.lzj >= KMAX)
      return hipErrorInvalidValue;
    // 32 x 32 tiles only (the epilogue holds a lane's four results and their
    // basis elements; the 64 x 64 tile would hold sixteen)
    if constexpr (same) {
      dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, g.inst.count);
      hipLaunchKernelGGL((cgemm_lz_kernel<TA, TB, TC, TM, 32, 32, 32>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
  }
  const int nz = g.batch * g.inst.count;
  // the tile shape depends on one instance's problem only, so a batched
  // launch computes every instance exactly as a single launch would.
  // tile 64: 64x64 with K steps of 16; 96 / 128: 64x64 with K steps of 32 /
  // 64 (FP32 arithmetic only: fewer, longer steps hide more load latency
  // when K is short); 32: 32x32 with K steps of 32.
#define GEMM_LAUNCH(BM_, BN_, BK_) \
  hipLaunchKernelGGL((cgemm_kernel<TA, TB, TC, TM, BM_, BN_, BK_>), grid, dim3(256), 0, s, g)
  const int64_t tiles64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
  constexpr bool F32M = sizeof(TM) == 4;
  int tile = g.tile;
  if (tile == 0) tile = tiles64 >= 240 ? 64 : 32;
  if (!F32M && tile > 64) tile = 64;
  if (F32M && tile == 96) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz);
    GEMM_LAUNCH(64, 64, F32M ? 32 : 16);
  } else if (F32M && tile == 128) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz);
    GEMM_LAUNCH(64, 64, F32M ? 64 : 16);
  } else if (tile == 64) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz);
    GEMM_LAUNCH(64, 64, 16);
  } else {
    // small problems: 32 x 32 tiles, K in steps of 32 (one LDS phase for K <= 32)
    dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, nz);
    GEMM_LAUNCH(32, 32, 32);
  }
#undef GEMM_LAUNCH
  return hipGetLastError();
}

// Tile of a grouped launch: the choice the largest group (by 64x64 tiles)
// would make alone, so that group computes exactly as its own launch.
int grouped_tile(const GemmArgs *g, int ng, bool f32m) {
  int64_t best = -1;
  int tile = 32;
  for (int k = 0; k < ng; ++k) {
    const int64_t t64 = (int64_t)((g[k].M + 63) / 64) * ((g[k].N + 63) / 64) * g[k].batch * g[k].inst.count;
    if (t64 > best) {
      best = t64;
      const int64_t one = (int64_t)((g[k].M + 63) / 64) * ((g[k].N + 63) / 64) * g[k].batch;
      tile = g[k].tile != 0 ? g[k].tile : (one >= 240 ? 64 : 32);
    }
  }
  if (!f32m && tile > 64) tile = 64;
  return tile;
}

template <typename TA, typename TB, typename TC, typename TM>
hipError_t launch_grouped(const GemmArgs *g, int ng, bool bf3, hipStream_t s) {
  constexpr bool F32M = sizeof(TM) == 4;
  const int tile = bf3 ? (grouped_tile(g, ng, false) == 64 ? 64 : 32) : grouped_tile(g, ng, F32M);
  const int bmn = tile == 32 ? 32 : 64;
  Grp<GemmArgs> gg;
  for (int k = 0; k < ng; ++k) {
    if (g[k].M <= 0 || g[k].N <= 0 || g[k].batch <= 0 || g[k].inst.count <= 0) continue;
    gg.add(g[k], (g[k].N + bmn - 1) / bmn, (g[k].M + bmn - 1) / bmn, g[k].batch * g[k].inst.count);
  }
  if (gg.ng == 0) return hipSuccess;
  const dim3 grid(gg.blocks()), blk(256);
  if (bf3) {
    if (tile == 64) hipLaunchKernelGGL((cgemm_bf3_grouped_kernel<TA, TB, TC, 64, 64>), grid, blk, 0, s, gg);
    else hipLaunchKernelGGL((cgemm_bf3_grouped_kernel<TA, TB, TC, 32, 32>), grid, blk, 0, s, gg);
  } else if (F32M && tile == 96) {
    hipLaunchKernelGGL((cgemm_grouped_kernel<TA, TB, TC, TM, 64, 64, F32M ? 32 : 16>), grid, blk, 0, s, gg);
  } else if (F32M && tile == 128) {
    hipLaunchKernelGGL((cgemm_grouped_kernel<TA, TB, TC, TM, 64, 64, F32M ? 64 : 16>), grid, blk, 0, s, gg);
  } else if (tile == 64) {
    hipLaunchKernelGGL((cgemm_grouped_kernel<TA, TB, TC, TM, 64, 64, 16>), grid, blk, 0, s, gg);
  } else {
    hipLaunchKernelGGL((cgemm_grouped_kernel<TA, TB, TC, TM, 32, 32, 32>), grid, blk, 0, s, gg);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t cgemm_grouped(DType ta, DType tb, DType tc, const GemmArgs *g, int ng, int bf3, hipStream_t s) {
  if (ng < 1 || ng > GMAX) return hipErrorInvalidValue;
  for (int k = 0; k < ng; ++k)
    if (g[k].lzU) return hipErrorInvalidValue;   // (no projection epilogue in grouped launches)
  if (bf3) {
    if (tc != F32) return hipErrorInvalidValue;
    for (int k = 0; k < ng; ++k)
      if (g[k].mode != 0) return hipErrorInvalidValue;
    if (ta == F64 && tb == F32) return launch_grouped<double, float, float, float>(g, ng, true, s);
    if (ta == F32 && tb == F64) return launch_grouped<float, double, float, float>(g, ng, true, s);
    if (ta == F32 && tb == F32) return launch_grouped<float, float, float, float>(g, ng, true, s);
    if (ta == F64 && tb == F64) return launch_grouped<double, double, float, float>(g, ng, true, s);
    return hipErrorInvalidValue;
  }
  if (ta == F64 && tb == F64 && tc == F64) return launch_grouped<double, double, double, double>(g, ng, false, s);
  if (ta == F64 && tb == F32 && tc == F32) return launch_grouped<double, float, float, float>(g, ng, false, s);
  if (ta == F32 && tb == F64 && tc == F32) return launch_grouped<float, double, float, float>(g, ng, false, s);
  if (ta == F32 && tb == F32 && tc == F32) return launch_grouped<float, float, float, float>(g, ng, false, s);
  if (ta == F64 && tb == F64 && tc == F32) return launch_grouped<double, double, float, float>(g, ng, false, s);
  return hipErrorInvalidValue;
}

hipError_t cgemm_bf3(DType ta, DType tb, DType tc, const GemmArgs &g, hipStream_t s) {
  if (tc != F32 || g.mode != 0 || g.lzU) return hipErrorInvalidValue;
  if (ta == F64 && tb == F32) return launch_bf3<double, float, float>(g, s);
  if (ta == F32 && tb == F64) return launch_bf3<float, double, float>(g, s);
  if (ta == F32 && tb == F32) return launch_bf3<float, float, float>(g, s);
  if (ta == F64 && tb == F64) return launch_bf3<double, double, float>(g, s);
  return hipErrorInvalidValue;
}

hipError_t cgemm(DType ta, DType tb, DType tc, const GemmArgs &g, hipStream_t s) {
  if (ta == F64 && tb == F64 && tc == F64) return launch<double, double, double, double>(g, s);
  if (ta == F64 && tb == F32 && tc == F32) return launch<double, float, float, float>(g, s);
  if (ta == F32 && tb == F64 && tc == F32) return launch<float, double, float, float>(g, s);
  if (ta == F32 && tb == F32 && tc == F32) return launch<float, float, float, float>(g, s);
  if (ta == F64 && tb == F64 && tc == F32) return launch<double, double, float, float>(g, s);
  return hipErrorInvalidValue;
}

}  // namespace tdvp
