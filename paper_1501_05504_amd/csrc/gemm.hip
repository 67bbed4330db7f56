// MFMA GEMMs for CDNA4 (gfx950): the dense contractions of the hot path.
//
// C[M x N] = alpha * A[M x K] * B[K x N] + beta * C   (row-major C, ldc)
//
// One kernel template serves FP64 (v_mfma_f64_16x16x4_f64), FP32
// (v_mfma_f32_16x16x4_f32) and BF16 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  Both operands are staged through LDS in an "outer-major"
// layout s[o][k]: every LDS row holds 128 bytes of K (16 doubles, 32 floats or
// 64 bf16) plus a 16-byte pad, so that the 16 lanes of a lane group, which
// read 16 different rows at the same column, hit 16 disjoint bank groups.
//
// MFMA k-slot permutation: an MFMA sums over its k slots, so any bijection
// between slots and actual k is valid as long as A and B use the same one.
// Lane group g = lane/16 takes the 32 contiguous bytes [32g, 32g+32) of the
// LDS row for the whole BK tile and feeds them to consecutive MFMA steps.
// Each lane therefore issues two 16-byte LDS reads per operand tile per BK.
//
// Output layout of the 16x16 MFMA blocks, lane l, accumulator r:
//   FP32 / BF16 variants: D[4*(l/16) + r][l % 16]
//   FP64 variant:         D[4*r + l/16][l % 16]   (one row per accumulator
//                          group, the four lane groups interleaved)
//
// Block-tile to workgroup mapping: consecutive workgroup ids are dispatched
// round-robin across the 8 XCDs, so the linear id is first remapped to give
// every XCD a contiguous range of tiles, then tiles are grouped 8 row-tiles
// at a time so that concurrently resident tiles share A rows and B columns
// in that XCD's L2.
#include "d3s_internal.h"

namespace d3s {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

union Frag {
  uint4 q[2];
  double d[4];
  float f[8];
  bf8v h[2];
};

template <typename S> struct Acc;
template <> struct Acc<double> { typedef double T; typedef d4v V; };
template <> struct Acc<float> { typedef float T; typedef f4v V; };
template <> struct Acc<bf16_t> { typedef float T; typedef f4v V; };

template <typename S>
__device__ __forceinline__ void mma_tile(typename Acc<S>::V& c, const Frag& a, const Frag& b) {
  if constexpr (sizeof(S) == 8) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.d[s], b.d[s], c, 0, 0, 0);
  } else if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[s], b.f[s], c, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h[s], b.h[s], c, 0, 0, 0);
  }
}

struct KParams {
  int M, N, K;
  const void* A; long lda; long sA;
  const void* B; long ldb; long sB;
  void* C; long ldc; long sC;
  double alpha, beta;
};

__device__ __forceinline__ void tile_coords(int nTm, int nTn, int& tm, int& tn) {
  const int nt = nTm * nTn;
  int bid = blockIdx.x;
  if ((nt & 7) == 0) bid = (bid & 7) * (nt >> 3) + (bid >> 3);
  constexpr int G = 8;
  const int per_group = G * nTn;
  const int group = bid / per_group;
  const int first = group * G;
  const int gs = min(nTm - first, G);
  const int in = bid - group * per_group;
  tm = first + in % gs;
  tn = in / gs;
}

// Stage one operand tile (O outer rows x BK k) from global into registers.
// KC: X[o*ld + k];  !KC: X[k*ld + o].
template <typename S, int O, int NT, bool KC>
struct Stager {
  static constexpr int BK = 128 / (int)sizeof(S);
  static constexpr int VE = 16 / (int)sizeof(S);
  static constexpr int LDK = BK + VE;              // LDS row: BK elements + 16-byte pad
  static constexpr int CHUNKS = O * BK / VE;       // 16-byte chunks per tile
  static constexpr int LPT = CHUNKS / NT;          // chunks per thread
  static_assert(CHUNKS % NT == 0, "tile not divisible among threads");
  uint4 r[LPT];

  __device__ __forceinline__ void load(const S* __restrict__ X, long ld, int o0, int Odim, int k0, int K) {
#pragma unroll
    for (int p = 0; p < LPT; ++p) {
      const int c = threadIdx.x + p * NT;
      int o, k;
      if constexpr (KC) { o = c / (BK / VE); k = (c % (BK / VE)) * VE; }
      else { k = c / (O / VE); o = (c % (O / VE)) * VE; }
      const int go = o0 + o, gk = k0 + k;
      union { uint4 q; S e[VE]; } u;
      if constexpr (KC) {
        const S* src = X + (long)go * ld + gk;
        if (go < Odim && gk + VE <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
          u.q = *reinterpret_cast<const uint4*>(src);
        } else {
#pragma unroll
          for (int v = 0; v < VE; ++v) u.e[v] = (go < Odim && gk + v < K) ? src[v] : S(0);
        }
      } else {
        const S* src = X + (long)gk * ld + go;
        if (gk < K && go + VE <= Odim && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
          u.q = *reinterpret_cast<const uint4*>(src);
        } else {
#pragma unroll
          for (int v = 0; v < VE; ++v) u.e[v] = (gk < K && go + v < Odim) ? src[v] : S(0);
        }
      }
      r[p] = u.q;
    }
  }

  __device__ __forceinline__ void store(S* __restrict__ s) const {
#pragma unroll
    for (int p = 0; p < LPT; ++p) {
      const int c = threadIdx.x + p * NT;
      if constexpr (KC) {
        const int o = c / (BK / VE), k = (c % (BK / VE)) * VE;
        *reinterpret_cast<uint4*>(s + o * LDK + k) = r[p];
      } else {
        const int k = c / (O / VE), o = (c % (O / VE)) * VE;
        union { uint4 q; S e[VE]; } u;
        u.q = r[p];
#pragma unroll
        for (int v = 0; v < VE; ++v) s[(o + v) * LDK + k] = u.e[v];
      }
    }
  }
};

template <typename S, int BM, int BN, int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_kernel(KParams p) {
  typedef typename Acc<S>::T AT;
  typedef typename Acc<S>::V AV;
  constexpr int NT = (BM / WM) * (BN / WN) * 64;
  constexpr int BK = 128 / (int)sizeof(S);
  constexpr int LDK = BK + 16 / (int)sizeof(S);
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int WGN = BN / WN;
  __shared__ __align__(16) S sA[2][BM * LDK];
  __shared__ __align__(16) S sB[2][BN * LDK];

  const int nTm = (p.M + BM - 1) / BM, nTn = (p.N + BN - 1) / BN;
  int tm, tn;
  tile_coords(nTm, nTn, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const long bz = blockIdx.y;
  const S* __restrict__ A = reinterpret_cast<const S*>(p.A) + bz * p.sA;
  const S* __restrict__ B = reinterpret_cast<const S*>(p.B) + bz * p.sB;
  AT* __restrict__ C = reinterpret_cast<AT*>(p.C) + bz * p.sC;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lrow = lane & 15, lgrp = lane >> 4;

  AV acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = AV{0, 0, 0, 0};

  Stager<S, BM, NT, AKC> ga;
  Stager<S, BN, NT, BKC> gb;
  const int nk = (p.K + BK - 1) / BK;
  if (nk > 0) {
    ga.load(A, p.lda, m0, p.M, 0, p.K);
    gb.load(B, p.ldb, n0, p.N, 0, p.K);
    ga.store(sA[0]);
    gb.store(sB[0]);
  }
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      ga.load(A, p.lda, m0, p.M, (kt + 1) * BK, p.K);
      gb.load(B, p.ldb, n0, p.N, (kt + 1) * BK, p.K);
    }
    Frag fa[TM], fb[TN];
    const int koff = lgrp * (32 / (int)sizeof(S));
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const S* src = sA[cur] + (wm * WM + i * 16 + lrow) * LDK + koff;
      fa[i].q[0] = *reinterpret_cast<const uint4*>(src);
      fa[i].q[1] = *reinterpret_cast<const uint4*>(src + 16 / sizeof(S));
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const S* src = sB[cur] + (wn * WN + j * 16 + lrow) * LDK + koff;
      fb[j].q[0] = *reinterpret_cast<const uint4*>(src);
      fb[j].q[1] = *reinterpret_cast<const uint4*>(src + 16 / sizeof(S));
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) mma_tile<S>(acc[i][j], fa[i], fb[j]);
    if (kt + 1 < nk) {
      ga.store(sA[cur ^ 1]);
      gb.store(sB[cur ^ 1]);
    }
    __syncthreads();
  }

  const AT alpha = (AT)p.alpha, beta = (AT)p.beta;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * WN + j * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(S) == 8) ? (r * 4 + lgrp) : (lgrp * 4 + r);
        const int row = m0 + wm * WM + i * 16 + rr;
        if (row < p.M && col < p.N) {
          AT* dst = C + (long)row * p.ldc + col;
          AT v = alpha * acc[i][j][r];
          if (p.beta != 0.0) v += beta * *dst;
          *dst = v;
        }
      }
    }
}

template <typename S, int BM, int BN, int WM, int WN>
void launch_cfg(Ctx* c, const GemmArgs& g) {
  KParams p{g.M, g.N, g.K, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta};
  const int nTm = (g.M + BM - 1) / BM, nTn = (g.N + BN - 1) / BN;
  dim3 grid((unsigned)(nTm * nTn), (unsigned)g.batch, 1);
  dim3 block((BM / WM) * (BN / WN) * 64, 1, 1);
  if (g.a_kc && g.b_kc)
    hipLaunchKernelGGL((gemm_kernel<S, BM, BN, WM, WN, true, true>), grid, block, 0, c->stream, p);
  else if (g.a_kc && !g.b_kc)
    hipLaunchKernelGGL((gemm_kernel<S, BM, BN, WM, WN, true, false>), grid, block, 0, c->stream, p);
  else if (!g.a_kc && g.b_kc)
    hipLaunchKernelGGL((gemm_kernel<S, BM, BN, WM, WN, false, true>), grid, block, 0, c->stream, p);
  else
    hipLaunchKernelGGL((gemm_kernel<S, BM, BN, WM, WN, false, false>), grid, block, 0, c->stream, p);
  D3S_HIP(hipGetLastError());
}

template <typename S>
void gemm_dispatch(Ctx* c, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  // The 128x128 tile needs at least ~1 tile per CU to fill the chip; smaller
  // problems use 64x64 tiles.
  const long big = (long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch;
  int cfg = c->tile_config;
  if (cfg < 0) cfg = (big >= 256) ? 0 : 1;
  if (cfg == 0)
    launch_cfg<S, 128, 128, 64, 64>(c, g);
  else
    launch_cfg<S, 64, 64, 32, 32>(c, g);
}

}  // namespace

void gemm_f64(Ctx* c, const GemmArgs& g) { gemm_dispatch<double>(c, g); }
void gemm_f32(Ctx* c, const GemmArgs& g) { gemm_dispatch<float>(c, g); }
void gemm_bf16(Ctx* c, const GemmArgs& g) { gemm_dispatch<bf16_t>(c, g); }

void gemm(Ctx* c, d3s_prec p, const GemmArgs& g) {
  if (p == D3S_F64) gemm_f64(c, g);
  else if (p == D3S_F32) gemm_f32(c, g);
  else gemm_bf16(c, g);
}

}  // namespace d3s
