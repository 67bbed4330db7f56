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
// LDS row for the whole BK tile and feeds them to consecutive MFMA steps,
// read as register groups of 8 bytes (FP64, FP32) or 16 bytes (BF16) so that
// each group can be refilled for the next tile as soon as its MFMAs issue
// (the K-loop pipeline below).
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
#include <algorithm>

#include "mfma_tile.h"

namespace d3s {
namespace {

using namespace tile;

struct KParams {
  int M, N, K;
  const void* A; long lda; long sA;
  const void* B; long ldb; long sB;
  void* C; long ldc; long sC;
  double alpha, beta;
  int kchunk;        // K range of one split (multiple of BK); == K when not split
  long sSplit;       // element stride between the partial products of two splits
};


template <typename S, int BM, int BN, int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, (kMinWaves<BM, BN>()))
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
  const int kbeg = blockIdx.z * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);
  const S* __restrict__ A = reinterpret_cast<const S*>(p.A) + bz * p.sA;
  const S* __restrict__ B = reinterpret_cast<const S*>(p.B) + bz * p.sB;
  AT* __restrict__ C = reinterpret_cast<AT*>(p.C) + bz * p.sC + (long)blockIdx.z * p.sSplit;

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
  const int nk = (kend - kbeg + BK - 1) / BK;
  // k-tiles [0, nfull) of an interior tile load without bounds tests
  int nfull = 0;
  if (nk > 0 && Stager<S, BM, NT, AKC>::full_ok(A, p.lda, m0, p.M, kbeg, kend) &&
      Stager<S, BN, NT, BKC>::full_ok(B, p.ldb, n0, p.N, kbeg, kend))
    nfull = (kend - kbeg) / BK;
  auto fetch = [&](int t) {
    const int k0 = kbeg + t * BK;
    if (t < nfull) {
      ga.load_full(A, p.lda, m0, k0);
      gb.load_full(B, p.ldb, n0, k0);
    } else {
      ga.load(A, p.lda, m0, p.M, k0, kend);
      gb.load(B, p.ldb, n0, p.N, k0, kend);
    }
  };

  // Pipeline over k-tiles, two LDS stages, one barrier per tile.  The
  // register groups of tile kt+1 are read between the MFMA steps of tile kt
  // (each group as soon as the MFMAs that used its registers are issued), and
  // tile kt+2 goes global -> registers -> LDS stage kt%2 during tile kt, so
  // after the barrier the MFMAs never wait for LDS.
  typedef Grp<S> G;
  constexpr int NG = G::NG;
  constexpr int GE = G::GB / (int)sizeof(S);       // elements per group
  typename G::U ra[NG][TM], rb[NG][TN];
  const int koff = lgrp * (32 / (int)sizeof(S));
  auto read_group = [&](int stage, int g) {
#pragma unroll
    for (int i = 0; i < TM; ++i) G::read(ra[g][i], sA[stage] + (wm * WM + i * 16 + lrow) * LDK + koff + g * GE);
#pragma unroll
    for (int j = 0; j < TN; ++j) G::read(rb[g][j], sB[stage] + (wn * WN + j * 16 + lrow) * LDK + koff + g * GE);
  };
  auto mma_group = [&](int g) {
#pragma unroll
    for (int st = 0; st < G::STEPS; ++st)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) G::mma(acc[i][j], ra[g][i], rb[g][j], st);
  };

  if (nk > 0) {
    fetch(0);
    ga.store(sA[0]);
    gb.store(sB[0]);
    if (nk > 1) {
      fetch(1);
      ga.store(sA[1]);
      gb.store(sB[1]);
    }
  }
  __syncthreads();
  if (nk > 0) {
#pragma unroll
    for (int g = 0; g < NG - 1; ++g) read_group(0, g);
  }
  // Steady state (every tile fetched here is interior): one branch-free
  // block per half, so the memory instructions can be spread between the
  // MFMAs.  The last register group of tile kt is read at the top of
  // iteration kt (its LDS stage is rewritten only after this iteration's
  // barrier), with the global loads of tile kt+2, during the MFMAs of group
  // 0; after the barrier each group of tile kt+1 is read during the MFMAs
  // of the next group of tile kt, and tile kt+2 is stored with the last one.
  constexpr int QM = G::STEPS * TM * TN;            // MFMAs per group
  int kt = 0;
  for (; kt + 2 < nfull; ++kt) {
    const int cur = kt & 1, nxt = cur ^ 1;
    ga.load_full(A, p.lda, m0, kbeg + (kt + 2) * BK);
    gb.load_full(B, p.ldb, n0, kbeg + (kt + 2) * BK);
    read_group(cur, NG - 1);
    mma_group(0);
    interleave<QM, TM + TN, 0, Stager<S, BM, NT, AKC>::LPT + Stager<S, BN, NT, BKC>::LPT>();
    __syncthreads();
#pragma unroll
    for (int g = 1; g < NG; ++g) {
      read_group(nxt, g - 1);
      if (g == NG - 1) {
        ga.store(sA[cur]);
        gb.store(sB[cur]);
      }
      mma_group(g);
      if (g == NG - 1) interleave<QM, TM + TN, 2 * (Stager<S, BM, NT, AKC>::LPT + Stager<S, BN, NT, BKC>::LPT), 0>();
      else interleave<QM, TM + TN, 0, 0>();
    }
  }
  if (kt < nk) read_group(kt & 1, NG - 1);
  for (; kt < nk; ++kt) {
    const bool has1 = kt + 1 < nk, has2 = kt + 2 < nk;
    const int nxt = (kt + 1) & 1;
    if (has2) fetch(kt + 2);
    mma_group(0);
    __syncthreads();
#pragma unroll
    for (int g = 1; g < NG; ++g) {
      if (has1) read_group(nxt, g - 1);
      mma_group(g);
      if (g == NG / 2 && has2) {
        ga.store(sA[kt & 1]);
        gb.store(sB[kt & 1]);
      }
    }
    if (has1) read_group(nxt, NG - 1);
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

// C = alpha * sum_z P[z] + beta * C, in a fixed order over the splits
template <typename AT>
__global__ void splitk_reduce_kernel(const AT* __restrict__ P, int S, long sSplit, int M, int N, AT* __restrict__ C,
                                     long ldc, double alpha, double beta) {
  const long total = (long)M * N;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long r = i / N, c = i - r * N;
    AT acc = 0;
    for (int z = 0; z < S; ++z) acc += P[z * sSplit + i];
    AT v = (AT)alpha * acc;
    AT* dst = C + r * ldc + c;
    if (beta != 0.0) v += (AT)beta * *dst;
    *dst = v;
  }
}

template <typename S, int BM, int BN, int WM, int WN>
void launch_cfg(Ctx* c, const GemmArgs& g, int splits) {
  typedef typename Acc<S>::T AT;
  constexpr int BK = 128 / (int)sizeof(S);
  const int nTm = (g.M + BM - 1) / BM, nTn = (g.N + BN - 1) / BN;
  KParams p{g.M, g.N, g.K, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta, g.K, 0};
  AT* part = nullptr;
  if (splits > 1 && g.part) {
    // the caller's buffer bounds the number of partial products
    const size_t per = sizeof(AT) * (size_t)g.M * g.N;
    splits = (int)std::min<size_t>((size_t)splits, g.part_cap / per);
    if (splits < 2) splits = 1;
  }
  if (splits > 1) {
    // chunk = ceil(K / splits) rounded up to BK; recompute the number of splits
    int chunk = (g.K + splits - 1) / splits;
    chunk = (chunk + BK - 1) / BK * BK;
    splits = (g.K + chunk - 1) / chunk;
    part = g.part ? (AT*)g.part : (AT*)ws_get(c, WS_SPLITK, sizeof(AT) * (size_t)splits * g.M * g.N);
    p.C = part;
    p.ldc = g.N;
    p.sC = 0;
    p.alpha = 1.0;
    p.beta = 0.0;
    p.kchunk = chunk;
    p.sSplit = (long)g.M * g.N;
  }
  dim3 grid((unsigned)(nTm * nTn), (unsigned)g.batch, (unsigned)splits);
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
  if (splits > 1) {
    long total = (long)g.M * g.N;
    long nb = std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((splitk_reduce_kernel<AT>), dim3((unsigned)nb), dim3(256), 0, c->stream, part, splits,
                       (long)g.M * g.N, g.M, g.N, (AT*)g.C, g.ldc, g.alpha, g.beta);
    D3S_HIP(hipGetLastError());
  }
}

// Tile configurations (block tile / wave tile / waves):
//   0: 128x128 / 64x64 / 4      1: 64x64 / 32x32 / 4
//   2: 256x128 / 64x64 / 8      3: 128x128 / 64x32 / 8
//   4: 256x128 / 128x64 / 4 (one wave per SIMD, accumulators in AGPRs;
//      FP32 and BF16 only, FP64 runs configuration 2)
template <typename S>
void gemm_dispatch(Ctx* c, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  constexpr int BK = 128 / (int)sizeof(S);
  int cfg = c->tile_config;
  const long t128 = (long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch;
  const long t256 = (long)((g.M + 255) / 256) * ((g.N + 127) / 128) * g.batch;
  // measured on MI355X (H_eff at m = 256..4096): the 8-wave 256x128 tile is
  // fastest once there are enough of them (split-K fills the rest); small
  // products use 64x64 tiles
  if (cfg < 0) cfg = (t256 >= 64 && g.M >= 512) ? 2 : 1;
  long tiles;
  switch (cfg) {
    case 0: case 3: tiles = t128; break;
    case 2: case 4: tiles = (long)((g.M + 255) / 256) * ((g.N + 127) / 128) * g.batch; break;
    default: tiles = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch; break;
  }
  // split K when the tiles cannot fill the 256 CUs and K is long enough for
  // every split to run several BK steps; only for unbatched products
  int splits = 1;
  if (g.batch == 1 && tiles < 256 && g.K >= 8 * BK) {
    splits = (int)std::min<long>((512 + tiles - 1) / tiles, g.K / (4 * BK));
    if (splits < 2) splits = 1;
  }
  if (c->splitk_off) splits = 1;
  switch (cfg) {
    case 0: launch_cfg<S, 128, 128, 64, 64>(c, g, splits); break;
    case 2: launch_cfg<S, 256, 128, 64, 64>(c, g, splits); break;
    case 3: launch_cfg<S, 128, 128, 64, 32>(c, g, splits); break;
    case 4:
      // FP64 accumulators of a 128x64 wave tile do not fit the register file
      if constexpr (sizeof(S) == 8) launch_cfg<S, 256, 128, 64, 64>(c, g, splits);
      else launch_cfg<S, 256, 128, 128, 64>(c, g, splits);
      break;
    default: launch_cfg<S, 64, 64, 32, 32>(c, g, splits); break;
  }
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
