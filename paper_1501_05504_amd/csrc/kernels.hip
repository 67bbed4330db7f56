// Bandwidth-bound kernels of the hot path: the W-maps (step 2 of the H_eff
// ordering of Sec. 5), deterministic FP64 reductions and vector updates of
// the Lanczos solver, layout helpers of the truncation, casts of the
// mixed-precision path and the reduction of the W-adjoint.
#include <algorithm>

#include <type_traits>

#include "d3s_internal.h"

namespace d3s {
namespace {

constexpr int kThreads = 256;
constexpr int kRedBlocks = 1024;   // fixed partial count: reductions are order-deterministic

__device__ __forceinline__ float bf16_to_f32(bf16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
  return (bf16_t)(u >> 16);
}

template <typename T> struct Cvt;
template <> struct Cvt<double> {
  __device__ static double ld(double x) { return x; }
  __device__ static double st(double x) { return x; }
};
template <> struct Cvt<float> {
  __device__ static float ld(float x) { return x; }
  __device__ static float st(float x) { return x; }
};
template <> struct Cvt<bf16_t> {
  __device__ static float ld(bf16_t x) { return bf16_to_f32(x); }
  __device__ static bf16_t st(float x) { return f32_to_bf16(x); }
};

// ---------------------------------------------------------------- W-maps
// One thread per (a, y): it holds the K = wl*d values T1[a, :, :, y] in
// registers and produces the d*wr outputs; W (pre-scaled by alpha and laid
// out as [(s,v)][(w,t)]) sits in LDS and is read by broadcast.
template <typename Tin, typename Tout, typename Tc, int MAXK>
__global__ __launch_bounds__(kThreads)
void wmap_l2r_kernel(const Tin* __restrict__ T1, const Tc* __restrict__ Wg, Tout* __restrict__ out,
                     long ld_out, int ml, int d, int mr, int wl, int wr, Tc alpha) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Tc* sW = reinterpret_cast<Tc*>(smem_raw);
  const int K = wl * d;
  const int nOut = d * wr;
  // rows of MAXK entries, zero beyond K: the inner loop has no bounds test and
  // reads W with vector LDS loads
  for (int i = threadIdx.x; i < MAXK * nOut; i += blockDim.x) {
    const int o = i / MAXK, k = i - o * MAXK;  // o = s*wr + v, k = w*d + t
    const int s = o / wr, v = o - s * wr;
    const int w = k / d, t = k - w * d;
    sW[i] = (k < K) ? alpha * Wg[((w * wr + v) * d + s) * d + t] : Tc(0);
  }
  __syncthreads();
  const int a = blockIdx.y;
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= mr) return;
  Tc in[MAXK];
  const Tin* src = T1 + (long)a * K * mr + y;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) in[k] = (k < K) ? (Tc)Cvt<Tin>::ld(src[(long)k * mr]) : Tc(0);
  for (int o = 0; o < nOut; ++o) {
    const Tc* wrow = sW + o * MAXK;
    Tc acc = 0;
#pragma unroll
    for (int k = 0; k < MAXK; ++k) acc += wrow[k] * in[k];
    const int s = o / wr, v = o - s * wr;
    out[(long)(a * d + s) * ld_out + (long)v * mr + y] = Cvt<Tout>::st(acc);
  }
}

// One thread per (x, b): inputs Y[x, t, b, :] for all t (K = d*wr values),
// outputs Z[w, x, s, b] for all (w, s).
template <typename Tin, typename Tout, typename Tc, int MAXK>
__global__ __launch_bounds__(kThreads)
void wmap_r2l_kernel(const Tin* __restrict__ Y, const Tc* __restrict__ Wg, Tout* __restrict__ Z,
                     int ml, int d, int mr, int wl, int wr, Tc alpha) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Tc* sW = reinterpret_cast<Tc*>(smem_raw);
  const int K = d * wr;
  const int nOut = wl * d;
  for (int i = threadIdx.x; i < MAXK * nOut; i += blockDim.x) {
    const int o = i / MAXK, k = i - o * MAXK;  // o = w*d + s, k = t*wr + v
    const int w = o / d, s = o - w * d;
    const int t = k / wr, v = k - t * wr;
    sW[i] = (k < K) ? alpha * Wg[((w * wr + v) * d + s) * d + t] : Tc(0);
  }
  __syncthreads();
  const int x = blockIdx.y;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= mr) return;
  Tc in[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (k < K) {
      const int t = k / wr, v = k - t * wr;
      in[k] = (Tc)Cvt<Tin>::ld(Y[((long)(x * d + t) * mr + b) * wr + v]);
    } else {
      in[k] = Tc(0);
    }
  }
  for (int o = 0; o < nOut; ++o) {
    const Tc* wrow = sW + o * MAXK;
    Tc acc = 0;
#pragma unroll
    for (int k = 0; k < MAXK; ++k) acc += wrow[k] * in[k];
    const int w = o / d, s = o - w * d;
    Z[((long)(w * ml + x) * d + s) * mr + b] = Cvt<Tout>::st(acc);
  }
}

// W-maps for MPO bonds too wide for the register/LDS kernels above (the
// channel-pair MPO of H^2): one thread per output element, W read from
// global memory (every lane of a wave reads the same W entry, a broadcast).
template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(kThreads)
void wmap_l2r_wide_kernel(const Tin* __restrict__ T1, const Tc* __restrict__ Wg, Tout* __restrict__ out,
                          long ld_out, int ml, int d, int mr, int wl, int wr, Tc alpha) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)ml * d * wr * mr) return;
  const int y = (int)(e % mr);
  long r = e / mr;
  const int v = (int)(r % wr);
  r /= wr;
  const int s = (int)(r % d);
  const int a = (int)(r / d);
  Tc acc = 0;
  for (int w = 0; w < wl; ++w)
    for (int t = 0; t < d; ++t)
      acc += Wg[((w * wr + v) * d + s) * d + t] * (Tc)Cvt<Tin>::ld(T1[(((long)a * wl + w) * d + t) * mr + y]);
  out[((long)a * d + s) * ld_out + (long)v * mr + y] = Cvt<Tout>::st(alpha * acc);
}

template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(kThreads)
void wmap_r2l_wide_kernel(const Tin* __restrict__ Y, const Tc* __restrict__ Wg, Tout* __restrict__ Z, int ml,
                          int d, int mr, int wl, int wr, Tc alpha) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)wl * ml * d * mr) return;
  const int b = (int)(e % mr);
  long r = e / mr;
  const int s = (int)(r % d);
  r /= d;
  const int x = (int)(r % ml);
  const int w = (int)(r / ml);
  Tc acc = 0;
  for (int t = 0; t < d; ++t)
    for (int v = 0; v < wr; ++v)
      acc += Wg[((w * wr + v) * d + s) * d + t] * (Tc)Cvt<Tin>::ld(Y[(((long)x * d + t) * mr + b) * wr + v]);
  Z[e] = Cvt<Tout>::st(alpha * acc);
}

template <typename Tin, typename Tout, typename Tc>
void wmap_l2r_t(Ctx* c, const void* T1, const void* W, void* out, long ld_out, int ml, int d,
                int mr, int wl, int wr, double alpha) {
  const int K = wl * d;
  dim3 grid((mr + kThreads - 1) / kThreads, ml);
  auto args = [&](auto kern, int maxk) {
    const size_t sh = sizeof(Tc) * (size_t)maxk * d * wr;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), sh, c->stream, (const Tin*)T1, (const Tc*)W,
                       (Tout*)out, ld_out, ml, d, mr, wl, wr, (Tc)alpha);
  };
  const bool fits = d * wr <= 80;
  if (fits && K <= 8) args(wmap_l2r_kernel<Tin, Tout, Tc, 8>, 8);
  else if (fits && K <= 16) args(wmap_l2r_kernel<Tin, Tout, Tc, 16>, 16);
  else if (fits && K <= 24) args(wmap_l2r_kernel<Tin, Tout, Tc, 24>, 24);
  else if (fits && K <= 32) args(wmap_l2r_kernel<Tin, Tout, Tc, 32>, 32);
  else if (fits && K <= 48) args(wmap_l2r_kernel<Tin, Tout, Tc, 48>, 48);
  else if (fits && K <= 80) args(wmap_l2r_kernel<Tin, Tout, Tc, 80>, 80);
  else {
    const long n = (long)ml * d * wr * mr;
    hipLaunchKernelGGL((wmap_l2r_wide_kernel<Tin, Tout, Tc>), dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c->stream, (const Tin*)T1, (const Tc*)W, (Tout*)out, ld_out, ml, d, mr,
                       wl, wr, (Tc)alpha);
  }
  D3S_HIP(hipGetLastError());
}

template <typename Tin, typename Tout, typename Tc>
void wmap_r2l_t(Ctx* c, const void* Y, const void* W, void* Z, int ml, int d, int mr, int wl,
                int wr, double alpha) {
  const int K = d * wr;
  dim3 grid((mr + kThreads - 1) / kThreads, ml);
  auto args = [&](auto kern, int maxk) {
    const size_t sh = sizeof(Tc) * (size_t)maxk * d * wl;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), sh, c->stream, (const Tin*)Y, (const Tc*)W,
                       (Tout*)Z, ml, d, mr, wl, wr, (Tc)alpha);
  };
  const bool fits = d * wl <= 80;
  if (fits && K <= 8) args(wmap_r2l_kernel<Tin, Tout, Tc, 8>, 8);
  else if (fits && K <= 16) args(wmap_r2l_kernel<Tin, Tout, Tc, 16>, 16);
  else if (fits && K <= 24) args(wmap_r2l_kernel<Tin, Tout, Tc, 24>, 24);
  else if (fits && K <= 32) args(wmap_r2l_kernel<Tin, Tout, Tc, 32>, 32);
  else if (fits && K <= 48) args(wmap_r2l_kernel<Tin, Tout, Tc, 48>, 48);
  else if (fits && K <= 80) args(wmap_r2l_kernel<Tin, Tout, Tc, 80>, 80);
  else {
    const long n = (long)wl * ml * d * mr;
    hipLaunchKernelGGL((wmap_r2l_wide_kernel<Tin, Tout, Tc>), dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c->stream, (const Tin*)Y, (const Tc*)W, (Tout*)Z, ml, d, mr, wl, wr,
                       (Tc)alpha);
  }
  D3S_HIP(hipGetLastError());
}

// Block-sparse W-map over a table of tasks, one per (left sector i, right
// sector j) pair.  A task lists its allowed input channel pairs and output
// channel pairs as entries {offset within a row, partial W index}; for an
// element (a, y) of the D_i x D_j block
//   out[a*out_rs + e_out.off + y] = alpha * sum_k W[e_in[k].wp + e_out.wp] * in[a*in_rs + e_in[k].off + y]
// (the W index is the sum of the two partial indices).  Workgroups take
// chunks of kWmapChunk elements of a block (a per-chunk table names the
// task), four per thread, 256 apart so that loads and stores stay
// coalesced; the task's W sub-matrix sits in LDS.  Nothing outside the
// listed blocks is read or written.
template <typename Tin, typename Tout, typename Tc, int MAXK>
__global__ __launch_bounds__(kThreads)
void wmap_blocks_kernel(const Tin* __restrict__ in, const Tc* __restrict__ Wg, Tout* __restrict__ out,
                        const WmapTask* __restrict__ tasks, const int* __restrict__ ctask,
                        const WmapEnt* __restrict__ ents, long in_rs, long out_rs, Tc alpha) {
  constexpr int EPT = kWmapChunk / kThreads;
  __shared__ Tc sW[MAXK * MAXK];
  __shared__ long sInOff[MAXK], sOutOff[MAXK];
  __shared__ int sInW[MAXK], sOutW[MAXK];
  const WmapTask tk = tasks[ctask[blockIdx.x]];
  const int nin = tk.nin, nout = tk.nout;
  for (int i = threadIdx.x; i < nin; i += blockDim.x) {
    sInOff[i] = ents[tk.idx0 + i].off;
    sInW[i] = ents[tk.idx0 + i].wp;
  }
  for (int i = threadIdx.x; i < nout; i += blockDim.x) {
    sOutOff[i] = ents[tk.idx0 + nin + i].off;
    sOutW[i] = ents[tk.idx0 + nin + i].wp;
  }
  __syncthreads();
  // W rows zero-padded to MAXK; inputs past nin are zeros (the test is
  // uniform over the workgroup, so it costs no divergence and no loads)
  for (int i = threadIdx.x; i < nout * MAXK; i += blockDim.x) {
    const int o = i / MAXK, k = i - o * MAXK;
    sW[i] = (k < nin) ? alpha * Wg[sInW[k] + sOutW[o]] : Tc(0);
  }
  __syncthreads();
  const long n = (long)tk.di * tk.dj;
  const long e0 = (long)((int)blockIdx.x - tk.chunk0) * kWmapChunk + threadIdx.x;
  for (int r = 0; r < EPT; ++r) {
    const long e = e0 + (long)r * kThreads;
    if (e >= n) return;
    const long a = tk.i_off + e / tk.dj, y = tk.j_off + e % tk.dj;
    const Tin* src = in + a * in_rs + y;
    Tout* dst = out + a * out_rs + y;
    if (nin == 0) {
      for (int o = 0; o < nout; ++o) dst[sOutOff[o]] = Cvt<Tout>::st(Tc(0));
      continue;
    }
    Tc v[MAXK];
#pragma unroll
    for (int k = 0; k < MAXK; ++k) v[k] = (k < nin) ? (Tc)Cvt<Tin>::ld(src[sInOff[k]]) : Tc(0);
    for (int o = 0; o < nout; ++o) {
      Tc acc = 0;
#pragma unroll
      for (int k = 0; k < MAXK; ++k) acc += sW[o * MAXK + k] * v[k];
      dst[sOutOff[o]] = Cvt<Tout>::st(acc);
    }
  }
}

// Four consecutive elements of a block row per thread, moved with one
// vector load / store per channel pair: for tables whose offsets, row
// lengths and block widths are all multiples of 4 (so the four elements
// share a row and the vectors are aligned).  Same chunks and task table as
// wmap_blocks_kernel.
template <typename T> struct alignas(4 * sizeof(T)) Vec4 { T v[4]; };

template <typename Tin, typename Tout, typename Tc, int MAXK>
__global__ __launch_bounds__(kThreads)
void wmap_blocks_vec4_kernel(const Tin* __restrict__ in, const Tc* __restrict__ Wg, Tout* __restrict__ out,
                             const WmapTask* __restrict__ tasks, const int* __restrict__ ctask,
                             const WmapEnt* __restrict__ ents, long in_rs, long out_rs, Tc alpha) {
  static_assert(kWmapChunk == 4 * kThreads, "one vector of four elements per thread");
  __shared__ Tc sW[MAXK * MAXK];
  __shared__ long sInOff[MAXK], sOutOff[MAXK];
  __shared__ int sInW[MAXK], sOutW[MAXK];
  const WmapTask tk = tasks[ctask[blockIdx.x]];
  const int nin = tk.nin, nout = tk.nout;
  for (int i = threadIdx.x; i < nin; i += blockDim.x) {
    sInOff[i] = ents[tk.idx0 + i].off;
    sInW[i] = ents[tk.idx0 + i].wp;
  }
  for (int i = threadIdx.x; i < nout; i += blockDim.x) {
    sOutOff[i] = ents[tk.idx0 + nin + i].off;
    sOutW[i] = ents[tk.idx0 + nin + i].wp;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nout * MAXK; i += blockDim.x) {
    const int o = i / MAXK, k = i - o * MAXK;
    sW[i] = (k < nin) ? alpha * Wg[sInW[k] + sOutW[o]] : Tc(0);
  }
  __syncthreads();
  const long e = (long)((int)blockIdx.x - tk.chunk0) * kWmapChunk + 4L * threadIdx.x;
  if (e >= (long)tk.di * tk.dj) return;
  const long a = tk.i_off + e / tk.dj, y = tk.j_off + e % tk.dj;
  const Tin* src = in + a * in_rs + y;
  Tout* dst = out + a * out_rs + y;
  if (nin == 0) {
    Vec4<Tout> z;
#pragma unroll
    for (int j = 0; j < 4; ++j) z.v[j] = Cvt<Tout>::st(Tc(0));
    for (int o = 0; o < nout; ++o) *reinterpret_cast<Vec4<Tout>*>(dst + sOutOff[o]) = z;
    return;
  }
  Tc v[MAXK][4];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (k < nin) {
      const Vec4<Tin> q = *reinterpret_cast<const Vec4<Tin>*>(src + sInOff[k]);
#pragma unroll
      for (int j = 0; j < 4; ++j) v[k][j] = (Tc)Cvt<Tin>::ld(q.v[j]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[k][j] = Tc(0);
    }
  }
  for (int o = 0; o < nout; ++o) {
    Tc acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      const Tc wk = sW[o * MAXK + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += wk * v[k][j];
    }
    Vec4<Tout> r;
#pragma unroll
    for (int j = 0; j < 4; ++j) r.v[j] = Cvt<Tout>::st(acc[j]);
    *reinterpret_cast<Vec4<Tout>*>(dst + sOutOff[o]) = r;
  }
}

template <typename Tin, typename Tout, typename Tc>
void wmap_blocks_t(Ctx* c, const void* in, const void* W, void* out, const WmapPlan& w, double alpha) {
  dim3 grid((unsigned)w.chunks), block(kThreads);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, block, 0, c->stream, (const Tin*)in, (const Tc*)W, (Tout*)out, w.d_tasks,
                       w.d_ctask, w.d_ents, w.in_rs, w.out_rs, (Tc)alpha);
  };
  // the vector form: 4-byte (or smaller) elements, vector-aligned buffers
  if constexpr (sizeof(Tin) <= 4 && sizeof(Tout) <= 4) {
    const bool v4 = w.vec4 && w.maxk <= 24 && (reinterpret_cast<uintptr_t>(in) % (4 * sizeof(Tin)) == 0) &&
                    (reinterpret_cast<uintptr_t>(out) % (4 * sizeof(Tout)) == 0);
    if (v4) {
      if (w.maxk <= 8) go(wmap_blocks_vec4_kernel<Tin, Tout, Tc, 8>);
      else if (w.maxk <= 16) go(wmap_blocks_vec4_kernel<Tin, Tout, Tc, 16>);
      else go(wmap_blocks_vec4_kernel<Tin, Tout, Tc, 24>);
      D3S_HIP(hipGetLastError());
      return;
    }
  }
  if (w.maxk <= 8) go(wmap_blocks_kernel<Tin, Tout, Tc, 8>);
  else if (w.maxk <= 16) go(wmap_blocks_kernel<Tin, Tout, Tc, 16>);
  else if (w.maxk <= 24) go(wmap_blocks_kernel<Tin, Tout, Tc, 24>);
  else if (w.maxk <= 32) go(wmap_blocks_kernel<Tin, Tout, Tc, 32>);
  else if (w.maxk <= 48) go(wmap_blocks_kernel<Tin, Tout, Tc, 48>);
  else if (w.maxk <= 80) go(wmap_blocks_kernel<Tin, Tout, Tc, 80>);
  else throw Error{D3S_EINVAL, "block W-map: more than 80 channel pairs"};
  D3S_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kThreads)
void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, long n,
                        double* __restrict__ part) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// coef-partials for up to KMAX rows at once: each thread keeps one running
// sum per row over its grid-stride elements (w is read once), then every row
// is reduced over the block; part[j * gridDim.x + block].
// The row count of a Lanczos step is read from device memory, so the kernels
// below branch once, uniformly, to a body compiled for the next multiple of
// eight rows (rows past the last one are clamped to it and weighted by
// zero): every load of an element's rows is issued without a test, so a
// wave keeps many loads in flight.
template <int R>
__device__ __forceinline__ void mdot_rows(const double* __restrict__ Vj, long ldv, int kc,
                                          const double* __restrict__ w, long n, double* acc) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double wi = w[i];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] += Vj[(long)min(j, kc - 1) * ldv + i] * wi;
  }
}

template <int KMAX>
__global__ __launch_bounds__(kThreads, 2)
void mdot_partial_kernel(const double* __restrict__ V, long ldv, int k, const int* __restrict__ kdev, int j0,
                         const double* __restrict__ w, long n, double* __restrict__ part) {
  __shared__ double sh[kThreads / 64][KMAX];
  // rows of this launch: j0 .. j0 + kc - 1 of the k (or *kdev + 1) rows
  const int rows = kdev ? (*kdev + 1) : k;
  const int kc = min(rows - j0, KMAX);
  if (kc <= 0) return;
  const double* Vj = V + (long)j0 * ldv;
  double acc[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
  switch ((kc + 7) / 8) {
    case 1: mdot_rows<(KMAX < 8 ? KMAX : 8)>(Vj, ldv, kc, w, n, acc); break;
    case 2: if constexpr (KMAX >= 16) mdot_rows<16>(Vj, ldv, kc, w, n, acc); break;
    case 3: if constexpr (KMAX >= 24) mdot_rows<24>(Vj, ldv, kc, w, n, acc); break;
    case 4: if constexpr (KMAX >= 32) mdot_rows<32>(Vj, ldv, kc, w, n, acc); break;
    case 5: if constexpr (KMAX >= 40) mdot_rows<40>(Vj, ldv, kc, w, n, acc); break;
    case 6: if constexpr (KMAX >= 48) mdot_rows<48>(Vj, ldv, kc, w, n, acc); break;
    case 7: if constexpr (KMAX >= 56) mdot_rows<56>(Vj, ldv, kc, w, n, acc); break;
    default: if constexpr (KMAX >= 64) mdot_rows<64>(Vj, ldv, kc, w, n, acc); break;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < kc) {
      double v = acc[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) sh[wave][j] = v;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kc; j += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q][j];
    part[(long)(j0 + j) * gridDim.x + blockIdx.x] = t;
  }
}

// Second Gram-Schmidt pass fused with the first one's update: with
// c = -coef (the first pass's coefficients), w <- w + sum_j c_j V_j, and the
// partial sums of <V_j, w_new> for the second pass, reading every V_j once.
template <int R>
__device__ __forceinline__ void gs_update_dot_rows(const double* __restrict__ V, long ldv, int rows,
                                                   const double* sc, double* __restrict__ w, long n,
                                                   double* acc) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v[R];
    double x = w[i];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      v[j] = V[(long)min(j, rows - 1) * ldv + i];
      x += sc[j] * v[j];
    }
    w[i] = x;
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] += v[j] * x;
  }
}

template <int KMAX>
__global__ __launch_bounds__(kThreads, 2)
void gs_update_dot_kernel(const double* __restrict__ V, long ldv, int k, const int* __restrict__ kdev,
                          const double* __restrict__ coef, double* __restrict__ w, long n,
                          double* __restrict__ part) {
  __shared__ double sc[KMAX];
  __shared__ double sh[kThreads / 64][KMAX];
  const int rows = kdev ? (*kdev + 1) : k;
  for (int j = threadIdx.x; j < KMAX; j += blockDim.x) sc[j] = (j < rows) ? -coef[j] : 0.0;
  __syncthreads();
  double acc[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
  switch ((rows + 7) / 8) {
    case 1: gs_update_dot_rows<8>(V, ldv, rows, sc, w, n, acc); break;
    case 2: gs_update_dot_rows<16>(V, ldv, rows, sc, w, n, acc); break;
    case 3: if constexpr (KMAX >= 24) gs_update_dot_rows<24>(V, ldv, rows, sc, w, n, acc); break;
    case 4: if constexpr (KMAX >= 32) gs_update_dot_rows<32>(V, ldv, rows, sc, w, n, acc); break;
    case 5: if constexpr (KMAX >= 40) gs_update_dot_rows<40>(V, ldv, rows, sc, w, n, acc); break;
    case 6: if constexpr (KMAX >= 48) gs_update_dot_rows<48>(V, ldv, rows, sc, w, n, acc); break;
    case 7: if constexpr (KMAX >= 56) gs_update_dot_rows<56>(V, ldv, rows, sc, w, n, acc); break;
    default: if constexpr (KMAX >= 64) gs_update_dot_rows<64>(V, ldv, rows, sc, w, n, acc); break;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < rows) {
      double t = acc[j];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
      if (lane == 0) sh[wave][j] = t;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < rows; j += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q][j];
    part[(long)j * gridDim.x + blockIdx.x] = t;
  }
}

// Second pass update fused with the norm: w <- w - sum_j coef_j V_j and the
// per-block partial sums of |w_new|^2 (part[block]).
__global__ __launch_bounds__(kThreads, 2)
void gs_update_norm_kernel(const double* __restrict__ V, long ldv, int k, const int* __restrict__ kdev,
                           const double* __restrict__ coef, double* __restrict__ w, long n,
                           double* __restrict__ part) {
  __shared__ double sc[128];
  __shared__ double sh[kThreads / 64];
  const int rows = kdev ? (*kdev + 1) : k;
  for (int j = threadIdx.x; j < 128; j += blockDim.x) sc[j] = (j < rows) ? -coef[j] : 0.0;
  __syncthreads();
  double acc = 0.0;
  // rows in chunks of 8 (runtime count R/8): loads within a chunk are
  // issued together, and the register use stays bounded for any R
  auto pass = [&](auto rt) {
    constexpr int R = decltype(rt)::value;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
      double x = w[i];
#pragma unroll 2
      for (int jc = 0; jc < R; jc += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[(long)min(jc + u, rows - 1) * ldv + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) x += sc[jc + u] * v[u];
      }
      w[i] = x;
      acc += x * x;
    }
  };
  switch ((rows + 7) / 8) {
    case 1: pass(std::integral_constant<int, 8>()); break;
    case 2: pass(std::integral_constant<int, 16>()); break;
    case 3: pass(std::integral_constant<int, 24>()); break;
    case 4: pass(std::integral_constant<int, 32>()); break;
    case 5: pass(std::integral_constant<int, 40>()); break;
    case 6: pass(std::integral_constant<int, 48>()); break;
    case 7: pass(std::integral_constant<int, 56>()); break;
    case 8: pass(std::integral_constant<int, 64>()); break;
    default:
      for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double x = w[i];
        for (int j = 0; j < rows; ++j) x += sc[j] * V[(long)j * ldv + i];
        w[i] = x;
        acc += x * x;
      }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// End of a Lanczos step k (k from the host, or *kdev): V_{k+1} = w / beta
// with beta = sqrt(|w|^2) (zero when beta is not positive; skipped when
// k+1 = kk), and ab[2k] = alpha_k (the projections of both Gram-Schmidt
// passes on V_k), ab[2k+1] = beta.
__global__ __launch_bounds__(kThreads)
void lanczos_tail_kernel(const double* __restrict__ w, long n, const double* __restrict__ npart, int nnp,
                         const double* __restrict__ c1, const double* __restrict__ c2, int k,
                         const int* __restrict__ kdev, int kk, double* __restrict__ V, double* __restrict__ ab) {
  if (kdev) k = *kdev;
  // |w|^2 from the per-block partials, summed in a fixed order by every block
  __shared__ double sb;
  __shared__ double sh[kThreads / 64];
  double part = 0.0;
  for (int q = threadIdx.x; q < nnp; q += blockDim.x) part += npart[q];
  const double tot = block_sum(part, sh);
  if (threadIdx.x == 0) sb = tot;
  __syncthreads();
  const double b = sqrt(fmax(sb, 0.0));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ab[2 * k] = c1[k] + c2[k];
    ab[2 * k + 1] = b;
  }
  if (k + 1 >= kk) return;
  double* vnext = V + (long)(k + 1) * n;
  const double f = (b > 0.0) ? 1.0 / b : 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    vnext[i] = w[i] * f;
}

// dst = V_{*kdev}
__global__ __launch_bounds__(kThreads)
void copy_row_kernel(const double* __restrict__ V, long n, const int* __restrict__ kdev, double* __restrict__ dst) {
  const double* src = V + (long)(*kdev) * n;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// *p = v, or *p += v
__global__ void set_int_kernel(int* p, int v, int add) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = add ? (*p + v) : v;
}

// out[j] = sum_b part[j * nb + b] in a fixed order; one block per j
__global__ __launch_bounds__(kThreads)
void reduce_rows_kernel(const double* __restrict__ part, int nb, double* __restrict__ out,
                        const int* __restrict__ kdev) {
  __shared__ double sh[kThreads / 64];
  const int j = blockIdx.x;
  if (kdev && j >= *kdev + 1) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[(long)j * nb + b];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ __launch_bounds__(kThreads)
void maxpy_kernel(const double* __restrict__ V, long ldv, int k, const int* __restrict__ kdev,
                  const double* __restrict__ coef, double sign, double* __restrict__ w, long n) {
  __shared__ double sc[128];
  if (kdev) k = *kdev + 1;
  for (int j = threadIdx.x; j < k; j += blockDim.x) sc[j] = sign * coef[j];
  __syncthreads();
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double acc = w[i];
    for (int j = 0; j < k; ++j) acc += sc[j] * V[(long)j * ldv + i];
    w[i] = acc;
  }
}

__global__ void scale_kernel(double* __restrict__ x, long n, double s) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] *= s;
}

__global__ void scale_dev_kernel(double* __restrict__ x, long n, const double* __restrict__ s, int recip_sqrt) {
  const double f = recip_sqrt ? 1.0 / sqrt(*s) : *s;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] *= f;
}

// y = a x + b y; with b = 0 the old y is not read (it may hold anything,
// including NaN bit patterns of fresh workspace)
__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, long n) {
  if (b == 0.0) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
      y[i] = a * x[i];
    return;
  }
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void fill_kernel(double* __restrict__ x, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void zero_kernel(uint4* __restrict__ x, long n16, unsigned char* __restrict__ tail, int ntail) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long)gridDim.x * blockDim.x)
    x[i] = uint4{0, 0, 0, 0};
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// one workgroup per descriptor: a strided rows x cols block copy
__global__ void copy_desc_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                 const CopyDesc* __restrict__ desc) {
  const CopyDesc dd = desc[blockIdx.x];
  const long total = (long)dd.rows * dd.cols;
  for (long i = threadIdx.x; i < total; i += blockDim.x) {
    const long r = i / dd.cols, c = i - r * dd.cols;
    dst[dd.dst_off + r * dd.dst_rs + c * dd.dst_cs] = src[dd.src_off + r * dd.src_rs + c * dd.src_cs];
  }
}

// M[a,s,b] = 0 unless key(q_a) + key(q_s) = key(q_b) (linear charge keys)
__global__ void mask_site_kernel(double* __restrict__ M, int ml, int d, int mr, const int* __restrict__ ka,
                                 const int* __restrict__ ks, const int* __restrict__ kb) {
  const long total = (long)ml * d * mr;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long b = i % mr;
    const long as = i / mr;
    const int s = (int)(as % d), a = (int)(as / d);
    if (ka[a] + ks[s] != kb[b]) M[i] = 0.0;
  }
}

template <typename T>
__global__ void transpose_kernel(const T* __restrict__ in, long R, long C, T* __restrict__ out) {
  __shared__ T tile[32][33];
  const long r0 = (long)blockIdx.y * 32, c0 = (long)blockIdx.x * 32;
  for (int i = threadIdx.y; i < 32; i += blockDim.y) {
    const long r = r0 + i, cc = c0 + threadIdx.x;
    if (r < R && cc < C) tile[i][threadIdx.x] = in[r * C + cc];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += blockDim.y) {
    const long cc = c0 + i, r = r0 + threadIdx.x;
    if (r < R && cc < C) out[cc * R + r] = tile[threadIdx.x][i];
  }
}

template <typename Tin, typename Tout>
__device__ __forceinline__ Tout rl_convert(Tin v) {
  if constexpr (std::is_same<Tin, Tout>::value) return v;
  else if constexpr (std::is_same<Tout, bf16_t>::value) return f32_to_bf16((float)v);
  else return (Tout)v;
}

// One destination tile per workgroup (32 x 8 threads, rows along x).
template <typename Tin, typename Tout>
__global__ void relayout_tiles_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                      const RlTile* __restrict__ tiles) {
  const RlTile t = tiles[blockIdx.x];
  const int x = threadIdx.x;
  if (x >= t.pcols) return;
  for (int i = threadIdx.y; i < t.prows; i += blockDim.y) {
    Tout v = rl_convert<float, Tout>(0.0f);
    if (i < t.rows && x < t.cols) v = rl_convert<Tin, Tout>(in[t.src + (long)i * t.src_ld + x]);
    out[t.dst + (long)i * t.dst_ld + x] = v;
  }
}

// One 32 x 32 tile per workgroup, staged through LDS so that both the
// reads and the writes run along rows.
template <typename T>
__global__ void transpose_tiles_kernel(const T* __restrict__ in, T* __restrict__ out,
                                       const TrTile* __restrict__ tiles) {
  __shared__ T tile[32][33];
  const TrTile t = tiles[blockIdx.x];
  for (int i = threadIdx.y; i < t.rows; i += blockDim.y)
    if ((int)threadIdx.x < t.cols) tile[i][threadIdx.x] = in[t.src + (long)i * t.src_ld + threadIdx.x];
  __syncthreads();
  for (int i = threadIdx.y; i < t.cols; i += blockDim.y)
    if ((int)threadIdx.x < t.rows) out[t.dst + (long)i * t.dst_ld + threadIdx.x] = tile[threadIdx.x][i];
}

__global__ void copy2d_kernel(const double* __restrict__ src, long lds, double* __restrict__ dst, long ldd,
                              long rows, long cols) {
  const long total = rows * cols;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long r = i / cols, cc = i - r * cols;
    dst[r * ldd + cc] = src[r * lds + cc];
  }
}

template <typename Tout>
__global__ void cast_kernel(const double* __restrict__ x, Tout* __restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    if constexpr (sizeof(Tout) == 2) y[i] = f32_to_bf16((float)x[i]);
    else y[i] = (Tout)x[i];
  }
}

__global__ void cast_f32_f64_kernel(const float* __restrict__ x, double* __restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// Wbar[w, v, s, t] = sum_a part[a][(w,t)][(s,v)], fixed order over a
__global__ void adjoint_sum_kernel(const double* __restrict__ part, int ml, int d, int wl, int wr,
                                   double* __restrict__ Wbar) {
  const int n1 = wl * d, n2 = d * wr;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n1 * n2) return;
  const int r = idx / n2, cc = idx - r * n2;     // r = (w,t), cc = (s,v)
  double acc = 0.0;
  for (int a = 0; a < ml; ++a) acc += part[(long)a * n1 * n2 + idx];
  const int w = r / d, t = r - w * d;
  const int s = cc / wr, v = cc - s * wr;
  Wbar[((w * wr + v) * d + s) * d + t] = acc;
}

inline int grid_for(long n) {
  long g = (n + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

void wmap_l2r(Ctx* c, d3s_prec p, const void* T1, const void* W, void* out, long ld_out, int ml,
              int d, int mr, int wl, int wr, double alpha) {
  if (p == D3S_F64) wmap_l2r_t<double, double, double>(c, T1, W, out, ld_out, ml, d, mr, wl, wr, alpha);
  else if (p == D3S_F32) wmap_l2r_t<float, float, float>(c, T1, W, out, ld_out, ml, d, mr, wl, wr, alpha);
  else wmap_l2r_t<float, bf16_t, float>(c, T1, W, out, ld_out, ml, d, mr, wl, wr, alpha);
}

void wmap_r2l(Ctx* c, d3s_prec p, const void* Y, const void* W, void* Z, int ml, int d, int mr,
              int wl, int wr, double alpha) {
  if (p == D3S_F64) wmap_r2l_t<double, double, double>(c, Y, W, Z, ml, d, mr, wl, wr, alpha);
  else if (p == D3S_F32) wmap_r2l_t<float, float, float>(c, Y, W, Z, ml, d, mr, wl, wr, alpha);
  else wmap_r2l_t<float, bf16_t, float>(c, Y, W, Z, ml, d, mr, wl, wr, alpha);
}

void wmap_blocks(Ctx* c, d3s_prec p, const void* in, const void* W, void* out, const WmapPlan& w, double alpha) {
  if (w.tasks.empty() || w.chunks <= 0) return;
  if (p == D3S_F64) wmap_blocks_t<double, double, double>(c, in, W, out, w, alpha);
  else if (p == D3S_F32) wmap_blocks_t<float, float, float>(c, in, W, out, w, alpha);
  else wmap_blocks_t<float, bf16_t, float>(c, in, W, out, w, alpha);
}

void dot_f64(Ctx* c, const double* x, const double* y, long n, double* out_dev) {
  double* part = (double*)ws_get(c, WS_RED, sizeof(double) * kRedBlocks);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, x, y, n, part);
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kThreads), 0, c->stream, part, kRedBlocks, out_dev,
                     (const int*)nullptr);
  D3S_HIP(hipGetLastError());
}

void mdot_f64(Ctx* c, const double* V, long ldv, int k, const double* w, long n, double* coef_dev,
              const int* kdev) {
  if (k <= 0) return;
  if (k > 128) throw Error{D3S_EINVAL, "mdot: more than 128 vectors"};
  // partial count fixed by n (deterministic), at most kGsMaxBlocks
  const int nb = gs_blocks(n);
  double* part = (double*)ws_get(c, WS_RED, sizeof(double) * (size_t)nb * 128);
  for (int j0 = 0; j0 < k; j0 += 64) {
    const int kc = std::min(64, k - j0);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, c->stream, V, ldv, k, kdev, j0, w, n, part);
    };
    if (kc <= 8) go(mdot_partial_kernel<8>);
    else if (kc <= 16) go(mdot_partial_kernel<16>);
    else if (kc <= 32) go(mdot_partial_kernel<32>);
    else go(mdot_partial_kernel<64>);
  }
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(k), dim3(kThreads), 0, c->stream, part, nb, coef_dev, kdev);
  D3S_HIP(hipGetLastError());
}

int gs_blocks(long n) {
  return (int)std::max<long>(1, std::min<long>(kGsMaxBlocks, (n + 4L * kThreads - 1) / (4L * kThreads)));
}

void gs_second_pass(Ctx* c, const double* V, long ldv, int k, const int* kdev, const double* coef1, double* w,
                    long n, double* coef2) {
  if (k <= 0) return;
  if (k > 64) throw Error{D3S_EINVAL, "Gram-Schmidt: more than 64 vectors in the fused pass"};
  const int nb = gs_blocks(n);
  double* part = (double*)ws_get(c, WS_RED, sizeof(double) * (size_t)nb * 128);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, c->stream, V, ldv, k, kdev, coef1, w, n, part);
  };
  if (k <= 16) go(gs_update_dot_kernel<16>);
  else if (k <= 24) go(gs_update_dot_kernel<24>);
  else if (k <= 32) go(gs_update_dot_kernel<32>);
  else if (k <= 40) go(gs_update_dot_kernel<40>);
  else if (k <= 48) go(gs_update_dot_kernel<48>);
  else go(gs_update_dot_kernel<64>);
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(k), dim3(kThreads), 0, c->stream, part, nb, coef2, kdev);
  D3S_HIP(hipGetLastError());
}

void gs_update_norm(Ctx* c, const double* V, long ldv, int k, const int* kdev, const double* coef, double* w,
                    long n, double* npart) {
  if (k > 128) throw Error{D3S_EINVAL, "Gram-Schmidt: more than 128 vectors"};
  hipLaunchKernelGGL(gs_update_norm_kernel, dim3(gs_blocks(n)), dim3(kThreads), 0, c->stream, V, ldv, k, kdev,
                     coef, w, n, npart);
  D3S_HIP(hipGetLastError());
}

void lanczos_tail(Ctx* c, const double* w, long n, const double* npart, const double* c1, const double* c2, int k,
                  const int* kdev, int kk, double* V, double* ab) {
  hipLaunchKernelGGL(lanczos_tail_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, w, n, npart,
                     gs_blocks(n), c1, c2, k, kdev, kk, V, ab);
  D3S_HIP(hipGetLastError());
}

void copy_row_f64(Ctx* c, const double* V, long n, const int* kdev, double* dst) {
  hipLaunchKernelGGL(copy_row_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, V, n, kdev, dst);
  D3S_HIP(hipGetLastError());
}

void set_int_dev(Ctx* c, int* p, int v, bool add) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, p, v, add ? 1 : 0);
  D3S_HIP(hipGetLastError());
}

void maxpy_f64(Ctx* c, const double* V, long ldv, int k, const double* coef_dev, double sign, double* w,
               long n, const int* kdev) {
  if (k <= 0) return;
  if (k > 128) throw Error{D3S_EINVAL, "maxpy: more than 128 vectors"};
  hipLaunchKernelGGL(maxpy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, V, ldv, k, kdev, coef_dev,
                     sign, w, n);
  D3S_HIP(hipGetLastError());
}

void scale_f64(Ctx* c, double* x, long n, double s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, n, s);
  D3S_HIP(hipGetLastError());
}

void scale_by_dev_f64(Ctx* c, double* x, long n, const double* s_dev, bool reciprocal_sqrt) {
  hipLaunchKernelGGL(scale_dev_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, n, s_dev,
                     reciprocal_sqrt ? 1 : 0);
  D3S_HIP(hipGetLastError());
}

void axpby_f64(Ctx* c, double a, const double* x, double b, double* y, long n) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, a, x, b, y, n);
  D3S_HIP(hipGetLastError());
}

void copy_f64(Ctx* c, const double* x, double* y, long n) {
  if (n <= 0) return;
  D3S_HIP(hipMemcpyAsync(y, x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
}

void fill_f64(Ctx* c, double* x, long n, double v) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, n, v);
  D3S_HIP(hipGetLastError());
}

// Channel-pair MPO of H^2 between bra and ket copies of the state:
// W2[(w,c), (v,u), p, q] = sum_r W[w,v,r,p] W[c,u,r,q].
__global__ __launch_bounds__(kThreads)
void mpo_square_kernel(const double* __restrict__ W, double* __restrict__ W2, int wl, int wr, int d) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)wl * wl * wr * wr * d * d;
  if (e >= n) return;
  const int q = (int)(e % d);
  long r = e / d;
  const int p = (int)(r % d);
  r /= d;
  const int vu = (int)(r % ((long)wr * wr));
  const int wc = (int)(r / ((long)wr * wr));
  const int v = vu / wr, u = vu % wr, w = wc / wl, cc = wc % wl;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) acc += W[((w * wr + v) * d + k) * d + p] * W[((cc * wr + u) * d + k) * d + q];
  W2[e] = acc;
}

void mpo_square(Ctx* c, const double* W, double* W2, int wl, int wr, int d) {
  const long n = (long)wl * wl * wr * wr * d * d;
  hipLaunchKernelGGL(mpo_square_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     c->stream, W, W2, wl, wr, d);
  D3S_HIP(hipGetLastError());
}

// Metric of the residual's near-side vectors, ordered |S_y> (y < m), then
// H_v|S_y> at m + v*m + y:  G = [[1, E], [E^T, H2]] with E[y', (v,y)] =
// env[y', v, y] and H2[(v,y), (z,x)] = h2[y, v, z, x].
__global__ __launch_bounds__(kThreads)
void residual_metric_kernel(const double* __restrict__ env, const double* __restrict__ h2, int m, int w,
                            double* __restrict__ G) {
  const long n = (long)(1 + w) * m;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const long r = e / n, col = e % n;
  double val;
  if (r < m && col < m) {
    val = (r == col) ? 1.0 : 0.0;
  } else if (r < m) {
    val = env[r * w * m + (col - m)];
  } else if (col < m) {
    val = env[col * w * m + (r - m)];
  } else {
    const long rv = r - m, cz = col - m;
    const long v = rv / m, y = rv % m, z = cz / m, x = cz % m;
    val = h2[((y * w + v) * w + z) * m + x];
  }
  G[e] = val;
}

void residual_metric(Ctx* c, const double* env, const double* h2, int m, int w, double* G) {
  const long n = (long)(1 + w) * m;
  hipLaunchKernelGGL(residual_metric_kernel, dim3((unsigned)((n * n + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, c->stream, env, h2, m, w, G);
  D3S_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kThreads)
void scale2d_kernel(double* __restrict__ x, long ld, long rows, long cols, double f) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const long r = e / cols, col = e % cols;
  x[r * ld + col] *= f;
}

void scale2d_f64(Ctx* c, double* x, long ld, long rows, long cols, double f) {
  const long n = rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(scale2d_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     c->stream, x, ld, rows, cols, f);
  D3S_HIP(hipGetLastError());
}

// Enlarged environment of the centre-matrix formalism:
// Lt[(a,s), v, (x,t)] = sum_w L[a,w,x] W[w,v,s,t]; one thread per (a, x) with
// L[a, :, x] in registers and W in LDS.
template <int MAXW>
__global__ __launch_bounds__(kThreads)
void cwf_env_kernel(const double* __restrict__ L, const double* __restrict__ Wg, double* __restrict__ Lt, int ml,
                    int d, int wl, int wr) {
  extern __shared__ double sW[];
  const int nw = wl * wr * d * d;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) sW[i] = Wg[i];
  __syncthreads();
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)ml * ml) return;
  const int a = (int)(e / ml), x = (int)(e % ml);
  double l[MAXW];
#pragma unroll
  for (int w = 0; w < MAXW; ++w) l[w] = (w < wl) ? L[((long)a * wl + w) * ml + x] : 0.0;
  const long mlp = (long)ml * d;
  for (int sg = 0; sg < d; ++sg)
    for (int v = 0; v < wr; ++v) {
      double* dst = Lt + (((long)a * d + sg) * wr + v) * mlp + (long)x * d;
      for (int t = 0; t < d; ++t) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < MAXW; ++w)
          if (w < wl) acc += l[w] * sW[((w * wr + v) * d + sg) * d + t];
        dst[t] = acc;
      }
    }
}

void cwf_environment(Ctx* c, int ml, int d, int wl, int wr, const double* L, const double* W, double* Lt) {
  const long n = (long)ml * ml;
  const size_t sh = sizeof(double) * (size_t)wl * wr * d * d;
  if (sh > 64 * 1024) throw Error{D3S_EINVAL, "centre-matrix environment: MPO tensor too large for LDS"};
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  if (wl <= 8)
    hipLaunchKernelGGL(cwf_env_kernel<8>, grid, dim3(kThreads), sh, c->stream, L, W, Lt, ml, d, wl, wr);
  else if (wl <= 32)
    hipLaunchKernelGGL(cwf_env_kernel<32>, grid, dim3(kThreads), sh, c->stream, L, W, Lt, ml, d, wl, wr);
  else
    throw Error{D3S_EINVAL, "centre-matrix environment: w_l > 32"};
  D3S_HIP(hipGetLastError());
}

template <typename T>
__global__ __launch_bounds__(kThreads)
void sum_partials_kernel(const T* __restrict__ part, int parts, long n, T* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    T acc = part[i];
    for (int j = 1; j < parts; ++j) acc += part[(long)j * n + i];
    out[i] = acc;
  }
}

void sum_partials(Ctx* c, bool f64, const void* part, int parts, long n, void* out) {
  if (n <= 0) return;
  if (f64)
    hipLaunchKernelGGL(sum_partials_kernel<double>, dim3(grid_for(n)), dim3(kThreads), 0, c->stream,
                       (const double*)part, parts, n, (double*)out);
  else
    hipLaunchKernelGGL(sum_partials_kernel<float>, dim3(grid_for(n)), dim3(kThreads), 0, c->stream,
                       (const float*)part, parts, n, (float*)out);
  D3S_HIP(hipGetLastError());
}

void zero_bytes(Ctx* c, void* x, size_t bytes) {
  if (bytes == 0) return;
  if ((reinterpret_cast<uintptr_t>(x) & 15) != 0) throw Error{D3S_EINVAL, "zero_bytes: buffer not 16-byte aligned"};
  const long n16 = (long)(bytes / 16);
  const int ntail = (int)(bytes - (size_t)n16 * 16);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(std::max(n16, 1L))), dim3(kThreads), 0, c->stream, (uint4*)x, n16,
                     (unsigned char*)x + n16 * 16, ntail);
  D3S_HIP(hipGetLastError());
}

void copy_blocks(Ctx* c, const double* src, double* dst, const std::vector<CopyDesc>& desc_in) {
  if (desc_in.empty()) return;
  // one workgroup per descriptor: blocks of more than kPiece elements are
  // cut into row ranges (and long rows into column ranges) first
  constexpr long kPiece = 16384;
  std::vector<CopyDesc> desc;
  desc.reserve(desc_in.size());
  for (const CopyDesc& q : desc_in) {
    if ((long)q.rows * q.cols <= kPiece) {
      desc.push_back(q);
      continue;
    }
    const int cstep = (int)std::min<long>(q.cols, kPiece);
    const int rstep = (int)std::max<long>(1, kPiece / cstep);
    for (int r0 = 0; r0 < q.rows; r0 += rstep)
      for (int c0 = 0; c0 < q.cols; c0 += cstep) {
        CopyDesc p = q;
        p.src_off = q.src_off + (long)r0 * q.src_rs + (long)c0 * q.src_cs;
        p.dst_off = q.dst_off + (long)r0 * q.dst_rs + (long)c0 * q.dst_cs;
        p.rows = std::min(rstep, q.rows - r0);
        p.cols = std::min(cstep, q.cols - c0);
        desc.push_back(p);
      }
  }
  CopyDesc* d = (CopyDesc*)ws_get(c, WS_DESC, sizeof(CopyDesc) * desc.size());
  D3S_HIP(hipMemcpyAsync(d, desc.data(), sizeof(CopyDesc) * desc.size(), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(copy_desc_kernel, dim3((unsigned)desc.size()), dim3(kThreads), 0, c->stream, src, dst, d);
  D3S_HIP(hipGetLastError());
  // the descriptor upload reads pageable host memory: wait before it goes away
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void mask_site(Ctx* c, double* M, int ml, int d, int mr, const std::vector<int>& ka, const std::vector<int>& ks,
               const std::vector<int>& kb) {
  std::vector<int> all(ka);
  all.insert(all.end(), ks.begin(), ks.end());
  all.insert(all.end(), kb.begin(), kb.end());
  int* dk = (int*)ws_get(c, WS_DESC, sizeof(int) * all.size());
  D3S_HIP(hipMemcpyAsync(dk, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice, c->stream));
  const long n = (long)ml * d * mr;
  hipLaunchKernelGGL(mask_site_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, M, ml, d, mr, dk, dk + ml,
                     dk + ml + d);
  D3S_HIP(hipGetLastError());
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void transpose_f64(Ctx* c, const double* in, long R, long C, double* out) {
  transpose_any(c, 8, in, R, C, out);
}

void transpose_any(Ctx* c, int esz, const void* in, long R, long C, void* out) {
  if (R <= 0 || C <= 0) return;
  if ((R + 31) / 32 > 65535) throw Error{D3S_EINVAL, "transpose: too many rows"};
  dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
  if (esz == 8)
    hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(32, 8), 0, c->stream, (const double*)in, R, C,
                       (double*)out);
  else if (esz == 4)
    hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(32, 8), 0, c->stream, (const float*)in, R, C,
                       (float*)out);
  else
    hipLaunchKernelGGL(transpose_kernel<unsigned short>, grid, dim3(32, 8), 0, c->stream,
                       (const unsigned short*)in, R, C, (unsigned short*)out);
  D3S_HIP(hipGetLastError());
}

void transpose_tiles(Ctx* c, int esz, const void* in, void* out, const TrTile* tiles, int ntiles) {
  if (ntiles <= 0) return;
  if (esz == 8)
    hipLaunchKernelGGL(transpose_tiles_kernel<double>, dim3(ntiles), dim3(32, 8), 0, c->stream,
                       (const double*)in, (double*)out, tiles);
  else if (esz == 4)
    hipLaunchKernelGGL(transpose_tiles_kernel<float>, dim3(ntiles), dim3(32, 8), 0, c->stream,
                       (const float*)in, (float*)out, tiles);
  else
    hipLaunchKernelGGL(transpose_tiles_kernel<unsigned short>, dim3(ntiles), dim3(32, 8), 0, c->stream,
                       (const unsigned short*)in, (unsigned short*)out, tiles);
  D3S_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- small symmetric eigensolver
// Batched FP64 symmetric eigensolver for n <= kEigSmallMax, one workgroup
// per matrix with the whole matrix in LDS (rows of odd stride n+1, so column
// walks do not collide in the banks): Householder reduction to tridiagonal
// form with the orthogonal transformation accumulated in place, then the
// implicit QL iteration with shifts on the tridiagonal matrix (the classical
// tred2 / tql2 pair of Wilkinson and Reinsch's Handbook).  The scalar
// recurrence of each QL sweep runs on one thread, which stores the sweep's
// Givens rotations; all threads then apply them to the rows of the
// eigenvector matrix.  Nothing is launched per column, which is what makes
// the library solver slow on batches of small Gram matrices.
__device__ __forceinline__ double eig_allsum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();                       // red may still be read from the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
  return r;                              // the same sum, in the same order, on every thread
}

template <int NMAX>
__global__ __launch_bounds__(kThreads)
void eig_small_kernel(double* __restrict__ A, double* __restrict__ evals, int n, int* __restrict__ info) {
  constexpr int LD = NMAX + 1;
  __shared__ double a[NMAX * LD];
  __shared__ double d[NMAX], e[NMAX], cs[2 * NMAX], red[8];
  __shared__ int ctl[4], perm[NMAX];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ld = n + 1;
  double* Ab = A + (long)blockIdx.x * n * n;
  // symmetric: the column-major input read row by row is the same matrix
  for (int idx = tid; idx < n * n; idx += nt) a[(idx / n) * ld + idx % n] = Ab[idx];
  __syncthreads();
  // ---- Householder reduction (row i annihilated left of the subdiagonal)
  for (int i = n - 1; i > 0; --i) {
    const int l = i - 1;
    double h = 0.0;
    double* ai = a + i * ld;
    if (l > 0) {
      double part = 0.0;
      for (int k = tid; k <= l; k += nt) part += fabs(ai[k]);
      const double scale = eig_allsum(part, red);
      if (scale == 0.0) {
        if (tid == 0) e[i] = ai[l];
        __syncthreads();
      } else {
        part = 0.0;
        for (int k = tid; k <= l; k += nt) {
          const double v = ai[k] / scale;
          ai[k] = v;
          part += v * v;
        }
        h = eig_allsum(part, red);
        const double f = ai[l];
        const double g = (f >= 0.0) ? -sqrt(h) : sqrt(h);
        h -= f * g;
        __syncthreads();                 // every thread has read ai[l]
        if (tid == 0) {
          e[i] = scale * g;
          ai[l] = f - g;                 // u = row i, H = h
        }
        __syncthreads();
        // p = A u / H into e[0..l], u / H into column i
        part = 0.0;
        for (int j = tid; j <= l; j += nt) {
          a[j * ld + i] = ai[j] / h;
          double gg = 0.0;
          for (int k = 0; k <= j; ++k) gg += a[j * ld + k] * ai[k];
          for (int k = j + 1; k <= l; ++k) gg += a[k * ld + j] * ai[k];
          e[j] = gg / h;
          part += e[j] * ai[j];
        }
        const double hh = eig_allsum(part, red) / (h + h);
        for (int j = tid; j <= l; j += nt) e[j] -= hh * ai[j];      // q = p - K u
        __syncthreads();
        // A -= u q^T + q u^T on the lower triangle of the leading block
        for (int j = tid; j <= l; j += nt) {
          const double fj = ai[j], gj = e[j];
          for (int k = 0; k <= j; ++k) a[j * ld + k] -= fj * e[k] + gj * ai[k];
        }
        __syncthreads();
      }
    } else {
      if (tid == 0) e[i] = ai[l];
      __syncthreads();
    }
    if (tid == 0) d[i] = h;
    __syncthreads();
  }
  if (tid == 0) {
    d[0] = 0.0;
    e[0] = 0.0;
  }
  __syncthreads();
  // ---- accumulate the transformation: a becomes the orthogonal matrix
  for (int i = 0; i < n; ++i) {
    const int l = i - 1;
    const bool nz = (d[i] != 0.0);
    __syncthreads();                     // d[i] is rewritten below
    if (nz) {
      for (int j = tid; j <= l; j += nt) {
        double g = 0.0;
        for (int k = 0; k <= l; ++k) g += a[i * ld + k] * a[k * ld + j];
        for (int k = 0; k <= l; ++k) a[k * ld + j] -= g * a[k * ld + i];
      }
      __syncthreads();
    }
    if (tid == 0) {
      d[i] = a[i * ld + i];
      a[i * ld + i] = 1.0;
    }
    for (int j = tid; j <= l; j += nt) {
      a[j * ld + i] = 0.0;
      a[i * ld + j] = 0.0;
    }
    __syncthreads();
  }
  // ---- implicit QL on the tridiagonal (d, e), rotations applied to the rows of a
  if (tid == 0) {
    for (int i = 1; i < n; ++i) e[i - 1] = e[i];
    e[n - 1] = 0.0;
    ctl[2] = 0;
  }
  __syncthreads();
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      if (tid == 0) {
        int m = l;
        for (; m < n - 1; ++m) {
          const double dd = fabs(d[m]) + fabs(d[m + 1]);
          if (fabs(e[m]) + dd == dd) break;
        }
        int ilo = m - 1;                 // no rotation
        if (m != l) {
          if (iter++ >= 60) {
            ctl[2] = 1;                  // no convergence: stop this eigenvalue
            m = l;
          } else {
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double sn = 1.0, cn = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
              const double f = sn * e[i], b = cn * e[i];
              r = hypot(f, g);
              e[i + 1] = r;
              if (r == 0.0) {
                d[i + 1] -= p;
                e[m] = 0.0;
                break;
              }
              sn = f / r;
              cn = g / r;
              g = d[i + 1] - p;
              r = (d[i] - g) * sn + 2.0 * cn * b;
              p = sn * r;
              d[i + 1] = g + p;
              g = cn * r - b;
              cs[2 * i] = cn;
              cs[2 * i + 1] = sn;
            }
            ilo = i;                     // rotations ilo+1 .. m-1 were formed
            if (!(r == 0.0 && i >= l)) {
              d[l] -= p;
              e[l] = g;
              e[m] = 0.0;
            }
          }
        }
        ctl[0] = m;
        ctl[1] = ilo;
      }
      __syncthreads();
      const int m = ctl[0], ilo = ctl[1];
      __syncthreads();                   // ctl is rewritten in the next pass
      if (m == l) break;
      for (int k = tid; k < n; k += nt) {
        double* zk = a + k * ld;
        for (int i = m - 1; i > ilo; --i) {
          const double cn = cs[2 * i], sn = cs[2 * i + 1];
          const double f = zk[i + 1];
          zk[i + 1] = sn * zk[i] + cn * f;
          zk[i] = cn * zk[i] - sn * f;
        }
      }
      __syncthreads();
    }
  }
  // ---- ascending order; eigenvector r = column perm[r] of a
  if (tid == 0) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (d[perm[j]] < d[perm[best]]) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
    info[blockIdx.x] = ctl[2];
  }
  __syncthreads();
  double* wb = evals + (long)blockIdx.x * n;
  for (int r = tid; r < n; r += nt) wb[r] = d[perm[r]];
  for (int idx = tid; idx < n * n; idx += nt) {
    const int r = idx / n, k = idx % n;
    Ab[idx] = a[k * ld + perm[r]];
  }
}

void relayout_tiles(Ctx* c, int in_kind, int out_kind, const void* in, void* out, const RlTile* tiles,
                    int ntiles) {
  if (ntiles <= 0) return;
  const dim3 g(ntiles), b(32, 8);
  if (in_kind == RL_F64 && out_kind == RL_BF16)
    hipLaunchKernelGGL((relayout_tiles_kernel<double, bf16_t>), g, b, 0, c->stream, (const double*)in, (bf16_t*)out,
                       tiles);
  else if (in_kind == RL_F64 && out_kind == RL_F32)
    hipLaunchKernelGGL((relayout_tiles_kernel<double, float>), g, b, 0, c->stream, (const double*)in, (float*)out,
                       tiles);
  else if (in_kind == RL_F32 && out_kind == RL_F64)
    hipLaunchKernelGGL((relayout_tiles_kernel<float, double>), g, b, 0, c->stream, (const float*)in, (double*)out,
                       tiles);
  else if (in_kind == RL_F32 && out_kind == RL_F32)
    hipLaunchKernelGGL((relayout_tiles_kernel<float, float>), g, b, 0, c->stream, (const float*)in, (float*)out,
                       tiles);
  else if (in_kind == RL_BF16 && out_kind == RL_BF16)
    hipLaunchKernelGGL((relayout_tiles_kernel<bf16_t, bf16_t>), g, b, 0, c->stream, (const bf16_t*)in,
                       (bf16_t*)out, tiles);
  else
    throw Error{D3S_EINVAL, "relayout: unsupported element types"};
  D3S_HIP(hipGetLastError());
}

// Batched symmetric eigensolver (eigenvalues ascending, eigenvectors as the
// columns of the column-major matrices): the LDS solver above for
// n <= kEigSmallMax when chosen (d3s_set_eigensolver kind 3), rocSOLVER
// otherwise.  Measured on MI355X the LDS solver takes about 0.11 / 0.8 /
// 2.6 / 6.1 ms for n = 8 / 32 / 64 / 96 whatever the batch (up to 256
// matrices side by side): the Householder and accumulation phases have
// about n threads each walking O(n) dependent LDS operations, so it beats
// rocSOLVER only on batches of small matrices.
bool eig_small_used(const Ctx* c, int n) { return c->eig_kind == 3 && n >= 1 && n <= kEigSmallMax; }

void eig_batched_f64(Ctx* c, int n, int batch, double* A, double* evals) {
  if (batch <= 0) return;
  if (!eig_small_used(c, n)) {
    syevd_batched_f64(c, n, batch, A, evals);
    return;
  }
  int* info = (int*)ws_get(c, WS_INFO, sizeof(int) * (size_t)batch);
  const dim3 g((unsigned)batch), b(kThreads);
  if (n <= 32) hipLaunchKernelGGL(eig_small_kernel<32>, g, b, 0, c->stream, A, evals, n, info);
  else if (n <= 64) hipLaunchKernelGGL(eig_small_kernel<64>, g, b, 0, c->stream, A, evals, n, info);
  else if (n <= 96) hipLaunchKernelGGL(eig_small_kernel<96>, g, b, 0, c->stream, A, evals, n, info);
  else hipLaunchKernelGGL(eig_small_kernel<kEigSmallMax>, g, b, 0, c->stream, A, evals, n, info);
  D3S_HIP(hipGetLastError());
  std::vector<int> h(batch);
  D3S_HIP(hipMemcpyAsync(h.data(), info, sizeof(int) * batch, hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  for (int q = 0; q < batch; ++q)
    if (h[q] != 0) throw Error{D3S_EDEVICE, "small eigensolver: the QL iteration did not converge"};
}

void copy2d_f64(Ctx* c, const double* src, long lds, double* dst, long ldd, long rows, long cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(rows * cols)), dim3(kThreads), 0, c->stream, src, lds,
                     dst, ldd, rows, cols);
  D3S_HIP(hipGetLastError());
}

void cast_f64_to_f32(Ctx* c, const double* x, float* y, long n) {
  hipLaunchKernelGGL(cast_kernel<float>, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, y, n);
  D3S_HIP(hipGetLastError());
}

void cast_f64_to_bf16(Ctx* c, const double* x, bf16_t* y, long n) {
  hipLaunchKernelGGL(cast_kernel<bf16_t>, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, y, n);
  D3S_HIP(hipGetLastError());
}

void cast_f32_to_f64(Ctx* c, const float* x, double* y, long n) {
  hipLaunchKernelGGL(cast_f32_f64_kernel, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, x, y, n);
  D3S_HIP(hipGetLastError());
}

void adjoint_reduce_f64(Ctx* c, const double* T1, const double* U, double* Wbar, int ml, int d, int mr,
                        int wl, int wr) {
  const int n1 = wl * d, n2 = d * wr;
  double* part = (double*)ws_get(c, WS_MISC, sizeof(double) * (size_t)ml * n1 * n2);
  // part[a] = T1[a] (n1 x mr) * U[a]^T (mr x n2), batched over a
  GemmArgs g{n1, n2, mr, T1, mr, true, (long)n1 * mr, U, mr, true, (long)n2 * mr, part, n2,
             (long)n1 * n2, 1.0, 0.0, ml};
  gemm_f64(c, g);
  const int tot = n1 * n2;
  hipLaunchKernelGGL(adjoint_sum_kernel, dim3((tot + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     c->stream, part, ml, d, wl, wr, Wbar);
  D3S_HIP(hipGetLastError());
}

}  // namespace d3s
