// Grouped MFMA GEMM over a task table: one launch computes every
// symmetry-allowed block product of a block-sparse contraction.
//
// Each task owns an output block C[M x N] (at c_off, row stride ldc) and a
// list of K-segments; a segment is one product A_s[M x K_s] * B_s[K_s x N]
// (at a_off / b_off with its own leading dimensions).  The task's output is
// alpha * sum over its segments (+ beta * C when beta != 0), so contributions
// that land on the same
// output block (the sum over the right MPO bond of the last H_eff
// contraction, whose right-bond sectors differ from term to term) are
// accumulated in registers, without atomics and in a fixed order.
//
// The hardware hands consecutive workgroup ids to the eight XCDs in turn,
// each with its own L2.  Workgroup ids are therefore remapped so that runs of
// kChunk consecutive tiles (mostly tiles of one task, which share operand
// blocks) execute on the same XCD, the runs dealt to the XCDs round-robin for
// balance.  The task of a tile is read from a per-tile table (one load, where
// a search over the tasks' tile prefix sums would chain a dozen).  Tasks are
// sorted largest-first by the host so that long tiles start early.
//
// Block products are small (sector dimensions of tens to hundreds), so a
// tile's K loop is short and each K step carries little MFMA work.  With
// the small tiles (64x64 and 32x32, whose registers allow it) the operand
// loads of a K step are issued three steps ahead (two register buffers
// behind the two LDS stages), so that their latency overlaps two steps of
// MFMAs instead of one; the large tiles keep one register buffer.
#include <type_traits>

#include "mfma_tile.h"

namespace d3s {
namespace {

using namespace tile;

constexpr int kChunk = 8;   // consecutive tiles kept on one XCD
constexpr int kXcd = 8;

struct GParams {
  const GTask* tasks;
  const GSeg* segs;
  const int* tile_task;
  int ntasks;
  int total;                // tiles
  const void* A;
  const void* B;
  void* C;
  double alpha, beta;
};

template <typename S, int BM, int BN, int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, (kMinWaves<BM, BN>()))
void grouped_kernel(GParams p) {
  typedef typename Acc<S>::T AT;
  typedef typename Acc<S>::V AV;
  constexpr int NT = (BM / WM) * (BN / WN) * 64;
  constexpr int BK = 128 / (int)sizeof(S);
  constexpr int LDK = BK + 16 / (int)sizeof(S);
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int WGN = BN / WN;
  __shared__ __align__(16) S sA[2][BM * LDK];
  __shared__ __align__(16) S sB[2][BN * LDK];

  const int xcd = (int)blockIdx.x % kXcd, slot = (int)blockIdx.x / kXcd;
  const int bid = ((slot / kChunk) * kXcd + xcd) * kChunk + slot % kChunk;
  if (bid >= p.total) return;
  const GTask t = p.tasks[p.tile_task[bid]];
  const int local = bid - t.tile0;
  const int nTn = (t.N + BN - 1) / BN;
  const int m0 = (local / nTn) * BM, n0 = (local % nTn) * BN;

  const S* __restrict__ Ab = reinterpret_cast<const S*>(p.A);
  const S* __restrict__ Bb = reinterpret_cast<const S*>(p.B);
  AT* __restrict__ C = reinterpret_cast<AT*>(p.C) + t.c_off;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lrow = lane & 15, lgrp = lane >> 4;

  AV acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = AV{0, 0, 0, 0};

  // register buffers: two where the registers allow it (FP32 / BF16 tiles
  // up to 64x64, FP64 up to 32x32), else one
  constexpr int NB = (BM * BN <= 32 * 32 || (BM * BN <= 64 * 64 && sizeof(S) < 8)) ? 2 : 1;
  Stager<S, BM, NT, AKC> ga[NB];
  Stager<S, BN, NT, BKC> gb[NB];
  const int send = t.seg0 + t.nseg;
  int ntiles = 0;
  for (int q = t.seg0; q < send; ++q) {
    const int K = p.segs[q].K;
    if (K > 0) ntiles += (K + BK - 1) / BK;
  }
  // the K step to load next: segment fs (copied into cs), offset ck
  int fs = t.seg0, ck = 0;
  while (fs < send && p.segs[fs].K <= 0) ++fs;
  GSeg cs = (fs < send) ? p.segs[fs] : GSeg{0, 0, 0, 0, 0};
  // operand tiles of the next K step (in list order) into register buffer u.
  // Every fetch issues its loads, also past the end of the list (it then
  // reloads the last step, whose data is never used): with the same loads
  // on every path the compiler's wait counts stay exact, and the loads of
  // later steps stay in flight while earlier ones are consumed.
  auto fetch_next = [&](auto ub) {
    constexpr int u = decltype(ub)::value;
    ga[u].load_buf(Ab + cs.a_off, cs.lda, m0, t.M, ck, cs.K);
    gb[u].load_buf(Bb + cs.b_off, cs.ldb, n0, t.N, ck, cs.K);
    if (ck + BK < cs.K) {
      ck += BK;
    } else {
      int f = fs + 1;
      while (f < send && p.segs[f].K <= 0) ++f;
      if (f < send) {
        fs = f;
        cs = p.segs[f];
        ck = 0;
      }
    }
  };
  typedef Grp<S> G;
  constexpr int NG = G::NG;
  constexpr int GE = G::GB / (int)sizeof(S);
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
  // K step u lives in LDS stage u & 1 and, before that, in register buffer
  // u % NB.  Prologue: steps 0 and 1 into both stages (and, with two
  // buffers, step 2 into buffer 0).
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  if (ntiles > 0) {
    if constexpr (NB == 2) {
      fetch_next(B0());
      fetch_next(B1());
      ga[0].store(sA[0]);
      gb[0].store(sB[0]);
      ga[1].store(sA[1]);
      gb[1].store(sB[1]);
      fetch_next(B0());
    } else {
      fetch_next(B0());
      ga[0].store(sA[0]);
      gb[0].store(sB[0]);
      fetch_next(B0());
      ga[0].store(sA[1]);
      gb[0].store(sB[1]);
    }
  }
  __syncthreads();
  if (ntiles > 0) {
#pragma unroll
    for (int g = 0; g < NG - 1; ++g) read_group(0, g);
  }
  // As in the plain GEMM: the last register group of step kt is read at the
  // top of iteration kt, the groups of step kt+1 after the barrier during the
  // MFMAs of the next group of step kt, and step kt+2 is stored with the
  // last group; the loads of step kt+1+NB go out at the top (so step kt+2
  // was loaded during this iteration with one buffer, the previous one with
  // two).  Each iteration is branch-free: past the end of the list the
  // loads, reads and the store move data that is never used (the store's
  // stage holds a step that has been read in full).  The loop is unrolled
  // by two so that stage and buffer indices are constants.
  constexpr int QM = G::STEPS * TM * TN;
  constexpr int NW = 2 * (Stager<S, BM, NT, AKC>::LPT + Stager<S, BN, NT, BKC>::LPT);
  // (with one buffer the stage indices are run-time values and the loop is
  // not unrolled: fewer live registers for the large tiles)
  auto step = [&](auto parity, int kt) {
    constexpr int pc = decltype(parity)::value;
    const int cur = (NB == 2) ? pc : (kt & 1), nxt = cur ^ 1;
    constexpr int bload = (NB == 2) ? (pc ^ 1) : 0, bstore = (NB == 2) ? pc : 0;
    fetch_next(std::integral_constant<int, bload>());
    read_group(cur, NG - 1);
    mma_group(0);
    interleave<QM, TM + TN, 0, 0>();
    __syncthreads();
#pragma unroll
    for (int g = 1; g < NG; ++g) {
      read_group(nxt, g - 1);
      if (g == NG - 1) {
        ga[bstore].store(sA[cur]);
        gb[bstore].store(sB[cur]);
      }
      mma_group(g);
      if (g == NG - 1) interleave<QM, TM + TN, NW, 0>();
      else interleave<QM, TM + TN, 0, 0>();
    }
  };
  if constexpr (NB == 2) {
    for (int kt = 0; kt < ntiles; kt += 2) {
      step(B0(), kt);
      if (kt + 1 >= ntiles) break;
      step(B1(), kt + 1);
    }
  } else {
    for (int kt = 0; kt < ntiles; ++kt) step(B0(), kt);
  }

  const AT alpha = (AT)p.alpha, beta = (AT)p.beta;
  const bool accumulate = p.beta != 0.0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * WN + j * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(S) == 8) ? (r * 4 + lgrp) : (lgrp * 4 + r);
        const int row = m0 + wm * WM + i * 16 + rr;
        if (row < t.M && col < t.N) {
          AT* dst = C + (long)row * t.ldc + col;
          *dst = accumulate ? alpha * acc[i][j][r] + beta * *dst : alpha * acc[i][j][r];
        }
      }
    }
}

template <typename S, int BM, int BN, int WM, int WN>
void launch_grouped(Ctx* c, const GroupedPlan& g, const void* A, const void* B, void* C, double alpha,
                    double beta) {
  GParams p{g.d_tasks, g.d_segs, g.d_tile, g.ntasks, g.total_tiles, A, B, C, alpha, beta};
  const long span = (long)kXcd * kChunk;
  dim3 grid((unsigned)((g.total_tiles + span - 1) / span * span)), block((BM / WM) * (BN / WN) * 64);
  if (g.a_kc && g.b_kc)
    hipLaunchKernelGGL((grouped_kernel<S, BM, BN, WM, WN, true, true>), grid, block, 0, c->stream, p);
  else if (g.a_kc && !g.b_kc)
    hipLaunchKernelGGL((grouped_kernel<S, BM, BN, WM, WN, true, false>), grid, block, 0, c->stream, p);
  else if (!g.a_kc && g.b_kc)
    hipLaunchKernelGGL((grouped_kernel<S, BM, BN, WM, WN, false, true>), grid, block, 0, c->stream, p);
  else
    hipLaunchKernelGGL((grouped_kernel<S, BM, BN, WM, WN, false, false>), grid, block, 0, c->stream, p);
  D3S_HIP(hipGetLastError());
}

}  // namespace

// block tile per configuration (rows x columns, waves):
//   0: 128x128 (4 waves of 64x64)   1: 64x64 (4 of 32x32)    2: 96x96 (4 of 48x48)
//   3: 32x32 (4 of 16x16)           4: 128x128 (8 of 64x32)  5: 256x128 (8 of 64x64)
void grouped_tile_dims(int cfg, int& bm, int& bn) {
  switch (cfg) {
    case 0: bm = bn = 128; break;
    case 2: bm = bn = 96; break;
    case 3: bm = bn = 32; break;
    case 4: bm = bn = 128; break;
    case 5: bm = 256; bn = 128; break;
    default: bm = bn = 64; break;
  }
}

void grouped_gemm(Ctx* c, d3s_prec prec, const GroupedPlan& g, const void* A, const void* B, void* C,
                  double alpha, double beta) {
  if (g.ntasks <= 0 || g.total_tiles <= 0) return;
  if (prec != D3S_F64) {
    const bool ok = (prec == D3S_F32 ? g.chunked32 : g.chunked16) &&
                    (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
    if (!ok) throw Error{D3S_EINVAL, "grouped GEMM: FP32 / BF16 blocks must be whole 16-byte chunks"};
  }
  auto run = [&](auto tag) {
    typedef decltype(tag) S;
    switch (g.cfg) {
      case 0: launch_grouped<S, 128, 128, 64, 64>(c, g, A, B, C, alpha, beta); break;
      case 2: launch_grouped<S, 96, 96, 48, 48>(c, g, A, B, C, alpha, beta); break;
      case 3: launch_grouped<S, 32, 32, 16, 16>(c, g, A, B, C, alpha, beta); break;
      case 4: launch_grouped<S, 128, 128, 64, 32>(c, g, A, B, C, alpha, beta); break;
      case 5: launch_grouped<S, 256, 128, 64, 64>(c, g, A, B, C, alpha, beta); break;
      default: launch_grouped<S, 64, 64, 32, 32>(c, g, A, B, C, alpha, beta); break;
    }
  };
  if (prec == D3S_F64) run(double());
  else if (prec == D3S_F32) run(float());
  else run(bf16_t());
}

}  // namespace d3s
