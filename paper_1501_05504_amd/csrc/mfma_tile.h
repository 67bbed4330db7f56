// Building blocks shared by the MFMA GEMM kernels (plain and grouped):
// fragment type, MFMA step per precision, LDS staging of operand tiles and
// the XCD-aware tile order.  See gemm.hip for the design notes.
#pragma once

#include "d3s_internal.h"

namespace d3s {
namespace tile {

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
__device__ __forceinline__ void mma_step(typename Acc<S>::V& c, const Frag& a, const Frag& b, int s) {
  if constexpr (sizeof(S) == 8) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.d[s], b.d[s], c, 0, 0, 0);
  else if constexpr (sizeof(S) == 4) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[s], b.f[s], c, 0, 0, 0);
  else c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h[s], b.h[s], c, 0, 0, 0);
}

// MFMA steps per 32-byte fragment: 4 (FP64), 8 (FP32), 2 (BF16)
template <typename S> constexpr int kSteps() { return sizeof(S) == 8 ? 4 : (sizeof(S) == 4 ? 8 : 2); }

// Scheduling hint for one branch-free block: spread R LDS reads, W LDS
// writes and V global loads between Q MFMAs (one memory instruction after
// each MFMA, reads first, then writes, then global loads; the rest of the
// MFMAs after them), so that they issue while the matrix core is busy.
template <int Q, int R, int W, int V>
__device__ __forceinline__ void interleave() {
  constexpr int P = (R + W + V < Q) ? R + W + V : Q;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    if (i < R) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    else if (i < R + W) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    else __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
  }
  if constexpr (Q > P) __builtin_amdgcn_sched_group_barrier(0x008, Q - P, 0);
}

// Waves per SIMD a tile configuration is compiled for: the 4-wave 64x64 and
// smaller tiles need 16 KB-class LDS and run four workgroups per CU, so
// their registers are capped at 128; 96x96 tiles run two.
template <int BM, int BN> constexpr int kMinWaves() { return BM * BN <= 64 * 64 ? 4 : (BM == 96 ? 2 : 1); }

// A 32-byte fragment split into register groups that are read from LDS one
// at a time: 4 groups of 8 bytes (FP64: one MFMA step each; FP32: two) or 2
// groups of 16 bytes (BF16: one step each).  The group g of lane group lg
// holds bytes [32 lg + g*GB, 32 lg + (g+1)*GB) of an LDS row, the same
// k-slot assignment as the whole fragment.
template <typename S> struct Grp {
  static constexpr int NG = sizeof(S) == 2 ? 2 : 4;
  static constexpr int GB = 32 / NG;
  static constexpr int STEPS = kSteps<S>() / NG;
  union U {
    uint2 q2;
    uint4 q4;
    double d;
    float f[2];
    bf8v h;
  };
  __device__ __forceinline__ static void read(U& u, const S* src) {
    if constexpr (GB == 8) u.q2 = *reinterpret_cast<const uint2*>(src);
    else u.q4 = *reinterpret_cast<const uint4*>(src);
  }
  __device__ __forceinline__ static void mma(typename Acc<S>::V& c, const U& a, const U& b, int s) {
    if constexpr (sizeof(S) == 8) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.d, b.d, c, 0, 0, 0);
    else if constexpr (sizeof(S) == 4) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[s], b.f[s], c, 0, 0, 0);
    else c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
  }
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

  // Interior tiles: every chunk in bounds and 16-byte aligned (the caller
  // checks this once per tile with wave-uniform values), so the loads carry
  // no per-element tests and no divergent branches.
  __device__ __forceinline__ void load_full(const S* __restrict__ X, long ld, int o0, int k0) {
#pragma unroll
    for (int p = 0; p < LPT; ++p) {
      const int c = threadIdx.x + p * NT;
      int o, k;
      if constexpr (KC) { o = c / (BK / VE); k = (c % (BK / VE)) * VE; }
      else { k = c / (O / VE); o = (c % (O / VE)) * VE; }
      const S* src = KC ? X + (long)(o0 + o) * ld + (k0 + k) : X + (long)(k0 + k) * ld + (o0 + o);
      r[p] = *reinterpret_cast<const uint4*>(src);
    }
  }

  // Loads of the grouped kernel, through a buffer resource whose base is the
  // tile's first element (X at (o0, k0), always inside the block): each
  // chunk is a 32-bit byte offset from it, and a chunk outside the block
  // gets an offset beyond the resource's range, for which the hardware
  // returns zeros without touching memory.  Low precision: every block is
  // made of whole 16-byte chunks (offsets, leading dimensions and the
  // chunked extent multiples of VE, the base 16-byte aligned; the host
  // checks this), so a chunk is one 16-byte load.  FP64 makes no such
  // assumption: a chunk is two 8-byte elements.  No branches, no per-lane
  // 64-bit addresses, whole-register loads: the compiler keeps the loads of
  // later K steps in flight across the iterations.  Offsets stay below 2^31
  // when the host-checked bound ld * 256 * sizeof(S) < 2^31 - 2^20 holds.
  __device__ __forceinline__ void load_buf(const S* __restrict__ X, long ld, int o0, int Odim, int k0, int K) {
    const S* first = KC ? X + (long)o0 * ld + k0 : X + (long)k0 * ld + o0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(first), (short)0, 0x7fffffff, 0x00020000);
    constexpr unsigned kOut = 0x80000000u;          // beyond the range: reads as zero
    const int ldi = (int)ld;
#pragma unroll
    for (int p = 0; p < LPT; ++p) {
      const int c = threadIdx.x + p * NT;
      int o, k;
      if constexpr (KC) { o = c / (BK / VE); k = (c % (BK / VE)) * VE; }
      else { k = c / (O / VE); o = (c % (O / VE)) * VE; }
      const int go = o0 + o, gk = k0 + k;
      const unsigned off = (unsigned)((KC ? o * ldi + k : k * ldi + o) * (int)sizeof(S));
      if constexpr (sizeof(S) == 8) {
        const bool v0 = go < Odim && gk < K;
        const bool v1 = KC ? (go < Odim && gk + 1 < K) : (gk < K && go + 1 < Odim);
        typedef unsigned u2v __attribute__((ext_vector_type(2)));
        const u2v a = __builtin_amdgcn_raw_buffer_load_b64(rs, v0 ? off : kOut, 0, 0);
        const u2v b = __builtin_amdgcn_raw_buffer_load_b64(rs, v1 ? off + 8u : kOut, 0, 0);
        r[p] = make_uint4(a.x, a.y, b.x, b.y);
      } else {
        typedef unsigned u4v __attribute__((ext_vector_type(4)));
        const u4v q = __builtin_amdgcn_raw_buffer_load_b128(rs, (go < Odim && gk < K) ? off : kOut, 0, 0);
        r[p] = make_uint4(q.x, q.y, q.z, q.w);
      }
    }
  }

  // whether a tile starting at (o0, k0) may use load_full
  __device__ __forceinline__ static bool full_ok(const S* X, long ld, int o0, int Odim, int k0, int K) {
    const bool in = (o0 + O <= Odim) && (k0 + BK <= K);
    const bool al = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ld % VE == 0) &&
                    (KC ? (k0 % VE == 0) : (o0 % VE == 0));
    return in && al;
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

}  // namespace tile
}  // namespace d3s
