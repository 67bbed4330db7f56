// Internal declarations of libdmrg3s (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg3s.h"

namespace d3s {

typedef uint16_t bf16_t;   // raw bfloat16 bits (round-to-nearest-even on conversion)

// ---------------------------------------------------------------- errors
struct Error {
  d3s_status code;
  std::string msg;
};

#define D3S_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::d3s::Error{D3S_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define D3S_REQUIRE(cond, text)                                                \
  do {                                                                         \
    if (!(cond)) throw ::d3s::Error{D3S_EINVAL, std::string(text)};           \
  } while (0)

// ---------------------------------------------------------------- context
enum WsSlot {
  WS_T1 = 0, WS_T2, WS_LZ_V, WS_LZ_W, WS_LZ_COEF, WS_RED, WS_GRAM, WS_EIGVAL,
  WS_EIGTMP, WS_UKT, WS_X, WS_MT, WS_CAST_L, WS_CAST_R, WS_CAST_X, WS_CAST_Y,
  WS_CAST_W, WS_REF, WS_PSI, WS_INFO, WS_NBR, WS_MISC, WS_SPLITK, WS_DESC, WS_BLK_X, WS_XPACK, WS_GPACK, WS_GVAL, WS_TUNE, WS_PK, WS_LZ_K, WS_GS_NORM, WS_JD_V, WS_JD_W, WS_JD_Z, WS_JD_COEF, WS_G2_PART, WS_W2, WS_RMET, WS_RZ, WS_RT, WS_RGRAM, WS_H2, WS_PSIT, WS_LP_L, WS_LP_R, WS_LP_X, WS_LP_Y,
  WS_TR_G, WS_TR_V, WS_TR_W0, WS_TR_W1, WS_TR_T2, WS_TR_T3, WS_TR_T4, WS_TR_P, WS_TR_TAB, WS_TR_AUX, WS_TR_XT,
  WS_EIG_PAR,
  WS_NSLOTS
};

struct EigPool;   // worker threads of the concurrent eigensolves (eigpool.hip)
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  d3s_allocator alloc{};
  bool has_alloc = false;
  void* ws_ptr[WS_NSLOTS] = {};
  size_t ws_cap[WS_NSLOTS] = {};
  void* solver = nullptr;            // rocblas_handle, created lazily
  double* host_red = nullptr;        // pinned host staging for scalars (512 doubles)
  void* lz_ev[2] = {nullptr, nullptr};   // Lanczos step events
  std::string last_error;
  int tile_config = -1;              // GEMM tile configuration (-1 = heuristic)
  int grouped_cfg = -1;              // grouped GEMM tile configuration (-1 = model / autotuner)
  double block_split_gflop = 1.0;    // split the block GEMM-2 from this many GFLOP on (< 0: never)
  bool splitk_off = false;           // disable split-K (tests compare both paths)
  bool autotune = false;             // time tile configurations on first use of a shape
  d3s_prec tune_prec = D3S_F64;      // precision the grouped plans being built will run in
  int eig_kind = 0;                  // batched eigensolver: 0 auto, 1 divide and conquer, 2 Jacobi, 3 LDS solver
  int eig_jacobi_max = 0;            // auto: Jacobi up to this size
  // concurrent shares of a truncation's divide-and-conquer solves, the
  // calling thread's on the context's stream (1: one at a time).  Four:
  // with the concurrency-aware grouping four beat three on large sectors
  // and tie on small ones; five or more were slower (measured on MI355X)
  int eig_workers = 4;
  double refine_eta = 0.1;           // mixed-precision refinement: inner CG target relative to the outer residual
  int refine_inner = 20;             // ... and its step cap
  double refine_low_tol = 0.0;       // low-precision Lanczos stop (<= 0: per-precision default)
  EigPool* eig_pool = nullptr;       // created on first concurrent use
  // truncation statistics, accumulated until the caller resets them: wall
  // seconds of the batched eigensolves and the Gram passes run
  double stat_eig_s = 0.0;
  int stat_passes = 0;
  std::unordered_map<std::string, int> tune_cache;
  std::string tune_path;
  // per-kernel profiling of H_eff: events around GEMM-1, W-map, GEMM-2
  bool prof = false;
  int prof_cap = 0, prof_n = 0;
  std::vector<hipEvent_t> prof_ev;   // 4 per recorded application
};

void* ws_get(Ctx* c, int slot, size_t bytes);
void ws_release_all(Ctx* c);
// Device memory the library keeps outside the workspace (the tables of block
// plans): from the context's allocator when one was given, else hipMalloc.
// A null context in dev_free means hipFree.  D3S_ENOMEM on failure.
void* dev_alloc(Ctx* c, size_t bytes);
void dev_free(Ctx* c, void* p);

// ---------------------------------------------------------------- GEMM
// C[M x N] = alpha * A[M x K] * B[K x N] + beta * C, row-major C with ldc.
// A is "K-contiguous" (A[m*lda + k]) when a_kc, else "M-contiguous" (A[k*lda + m]).
// B is "K-contiguous" (B[n*ldb + k]) when b_kc, else "N-contiguous" (B[k*ldb + n]).
// Batched over `batch` with element strides sA, sB, sC.
// part / part_cap: a caller buffer for the split-K partial products (the
// split count is then limited to what fits); null = the context workspace.
struct GemmArgs {
  int M, N, K;
  const void* A; long lda; bool a_kc; long sA;
  const void* B; long ldb; bool b_kc; long sB;
  void* C; long ldc; long sC;
  double alpha, beta;
  int batch;
  void* part = nullptr;
  size_t part_cap = 0;
};
void gemm_f64(Ctx* c, const GemmArgs& g);
void gemm_f32(Ctx* c, const GemmArgs& g);
void gemm_bf16(Ctx* c, const GemmArgs& g);   // bf16 operands, fp32 C
void gemm(Ctx* c, d3s_prec p, const GemmArgs& g);

// ---------------------------------------------------------------- grouped GEMM
// One output block per task, sum over the task's K-segments (see grouped.hip).
struct GTask { int M, N, seg0, nseg, tile0; long c_off, ldc; };
struct GSeg { int K; long a_off, lda, b_off, ldb; };
struct GroupedPlan {
  std::vector<GTask> tasks;
  std::vector<GSeg> segs;
  GTask* d_tasks = nullptr;     // device copies (owned by the plan; one allocation from d_tasks on)
  GSeg* d_segs = nullptr;
  int* d_tile = nullptr;        // task of every tile of the current configuration
  int ntasks = 0, total_tiles = 0;
  long tile_cap = 0;            // entries of d_tile (the most tiles of any configuration)
  bool chunked32 = false;       // every block made of whole 16-byte chunks with 4-byte elements
  bool chunked16 = false;       // ... with 2-byte elements (FP32 / BF16 launches require it)
  bool a_kc = true, b_kc = true;
  int cfg = 1;                  // tile configuration (grouped_tile_dims)
  double flops = 0.0;
  int table_slot = -1;          // >= 0: the device tables live in this workspace slot (not owned)
  Ctx* owner = nullptr;         // context whose allocator holds the tables
  size_t tune_n[3] = {0, 0, 0}; // extents (in doubles) of A, B, C for timing its tile configurations
};
void grouped_tile_dims(int cfg, int& bm, int& bn);   // block tile of a grouped configuration
// the tile configuration of a plan's launches in precision p (the rule; or
// the context's fixed configuration)
int grouped_pick_cfg(const Ctx* c, const GroupedPlan& g, d3s_prec p);
// sort tasks largest-first, pick the tile size, compute tile prefix sums and
// upload the tables (synchronises the stream)
void grouped_finalize(Ctx* c, GroupedPlan& g);
// recompute the tile prefix sums for g.cfg and upload the task table again
void grouped_retile(Ctx* c, GroupedPlan& g);
// autotuner (autotune.hip)
void autotune_load(Ctx* c);
void tuned_gemm(Ctx* c, d3s_prec p, const GemmArgs& g);
void tune_grouped(Ctx* c, GroupedPlan& g, const void* A, const void* B, void* C);
void grouped_release(GroupedPlan& g);
void grouped_gemm(Ctx* c, d3s_prec p, const GroupedPlan& g, const void* A, const void* B, void* C,
                  double alpha, double beta = 0.0);

// ---------------------------------------------------------------- kernels
// W-map of a left-to-right contraction:
//   T2[a, s, v, y] = alpha * sum_{w,t} W[w, v, s, t] * T1[a, w, t, y]
// T1 contiguous (ml, wl, d, mr); output row (a, s) at out + (a*d + s)*ld_out, inner (v, y).
void wmap_l2r(Ctx* c, d3s_prec p, const void* T1, const void* W, void* out, long ld_out,
              int ml, int d, int mr, int wl, int wr, double alpha);
// W-map of a right-to-left contraction:
//   Z[w, x, s, b] = alpha * sum_{v,t} W[w, v, s, t] * Y[x, t, b, v]
// Y contiguous (ml, d, mr, wr); Z contiguous (wl, ml, d, mr).
void wmap_r2l(Ctx* c, d3s_prec p, const void* Y, const void* W, void* Z,
              int ml, int d, int mr, int wl, int wr, double alpha);

// Block-sparse W-map (see kernels.hip): tasks over (left sector, right sector)
// pairs; ents[idx0 .. idx0+nin) are the input entries, the next nout the
// output entries; chunk0 = first kWmapChunk-element chunk of the task.
struct WmapTask { int i_off, di, j_off, dj, nin, nout, idx0, chunk0; };
struct WmapEnt { long off; int wp, pad_; };
// elements of a block W-map chunk (one workgroup of 256 threads, four
// elements per thread)
constexpr int kWmapChunk = 1024;
struct WmapPlan {
  std::vector<WmapTask> tasks;
  std::vector<WmapEnt> ents;
  WmapTask* d_tasks = nullptr;
  WmapEnt* d_ents = nullptr;
  int* d_ctask = nullptr;       // task of each chunk
  bool vec4 = false;            // every offset, row length and block width a multiple of 4
  int chunks = 0, maxk = 1;
  long in_rs = 0, out_rs = 0;
  Ctx* owner = nullptr;         // context whose allocator holds the tables
};
// append a task (skipped when it has no outputs); upload() copies the tables
void wmap_add(WmapPlan& w, int i_off, int di, int j_off, int dj, const std::vector<WmapEnt>& ins,
              const std::vector<WmapEnt>& outs);
void wmap_upload(Ctx* c, WmapPlan& w);
void wmap_release(WmapPlan& w);
void wmap_blocks(Ctx* c, d3s_prec p, const void* in, const void* W, void* out, const WmapPlan& w, double alpha);

// deterministic reductions (FP64)
void dot_f64(Ctx* c, const double* x, const double* y, long n, double* out_dev);
// coef[j] = <V_j, w> for j < k, V rows of length n with stride ldv.  With
// kdev the row count is *kdev + 1 (read on the device; k is then the
// largest possible count), so one captured launch serves every step.
void mdot_f64(Ctx* c, const double* V, long ldv, int k, const double* w, long n, double* coef_dev,
              const int* kdev = nullptr);
// partial-sum count of the Gram-Schmidt kernels for vectors of length n (fixed by n)
// partial sums per Gram-Schmidt pass: one per workgroup, at most kGsMaxBlocks
constexpr int kGsMaxBlocks = 1024;
int gs_blocks(long n);
// fused second pass: w -= sum_j coef1_j V_j, then coef2 = V^T w (rows k or *kdev + 1, <= 64)
void gs_second_pass(Ctx* c, const double* V, long ldv, int k, const int* kdev, const double* coef1, double* w,
                    long n, double* coef2);
// w -= sum_j coef_j V_j with the per-block partials of |w|^2 in npart (gs_blocks(n) entries)
void gs_update_norm(Ctx* c, const double* V, long ldv, int k, const int* kdev, const double* coef, double* w,
                    long n, double* npart);
// Lanczos step end (k from the host, or *kdev): beta = sqrt(sum of npart), V_{k+1} = w / beta
// unless k+1 = kk; ab[2k] = c1[k] + c2[k], ab[2k+1] = beta
void lanczos_tail(Ctx* c, const double* w, long n, const double* npart, const double* c1, const double* c2, int k,
                  const int* kdev, int kk, double* V, double* ab);
void copy_row_f64(Ctx* c, const double* V, long n, const int* kdev, double* dst);   // dst = V_{*kdev}
void set_int_dev(Ctx* c, int* p, int v, bool add);                                   // *p = v or *p += v
// w += sign * sum_j coef[j] V_j  (coef on device; row count k or *kdev + 1)
void maxpy_f64(Ctx* c, const double* V, long ldv, int k, const double* coef_dev, double sign,
               double* w, long n, const int* kdev = nullptr);
void scale_f64(Ctx* c, double* x, long n, double s_host);
void scale_by_dev_f64(Ctx* c, double* x, long n, const double* s_dev, bool reciprocal);
void axpby_f64(Ctx* c, double a, const double* x, double b, double* y, long n);
void copy_f64(Ctx* c, const double* x, double* y, long n);
void fill_f64(Ctx* c, double* x, long n, double v);
void zero_bytes(Ctx* c, void* x, size_t bytes);   // kernel fill (safe inside graph capture)
// out[i] = sum_{j < parts} part[j*n + i] in a fixed order (FP64, or FP32 when !f64)
void sum_partials(Ctx* c, bool f64, const void* part, int parts, long n, void* out);
// strided 2D block copies: dst[dst_off + r*dst_rs + c*dst_cs] = src[src_off + r*src_rs + c*src_cs]
struct CopyDesc { long src_off, src_rs, src_cs, dst_off, dst_rs, dst_cs; int rows, cols; };
void copy_blocks(Ctx* c, const double* src, double* dst, const std::vector<CopyDesc>& desc);
// zero the entries of a site tensor that violate q_a + q_s = q_b (linear charge keys per state)
void mask_site(Ctx* c, double* M, int ml, int d, int mr, const std::vector<int>& ka, const std::vector<int>& ks,
               const std::vector<int>& kb);
// out[r][col] = in[col][r] for an R x C input (row-major), i.e. out is C x R
void transpose_f64(Ctx* c, const double* in, long R, long C, double* out);
// out[C][R] = in[R][C] for 8-, 4- or 2-byte elements (esz)
void transpose_any(Ctx* c, int esz, const void* in, long R, long C, void* out);
// copy a rows x cols block with leading dimensions
void copy2d_f64(Ctx* c, const double* src, long lds, double* dst, long ldd, long rows, long cols);
// casts for the mixed-precision path
void cast_f64_to_f32(Ctx* c, const double* x, float* y, long n);
void cast_f64_to_bf16(Ctx* c, const double* x, bf16_t* y, long n);
void cast_f32_to_f64(Ctx* c, const float* x, double* y, long n);
// Wbar reduction of the adjoint: G[(w,t),(s,v)] = sum_{a,y} T1[a,w,t,y] * U[a,s,v,y]
void adjoint_reduce_f64(Ctx* c, const double* T1, const double* U, double* G,
                        int ml, int d, int mr, int wl, int wr);

// ---------------------------------------------------------------- host-side ops
void op_apply_heff(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr,
                   const void* L, const void* W, const void* R, const void* psi, void* out);
// the same product on caller buffers T1 (ml wl d mr), T2 (ml d wr mr), psiT
// (ml d mr) and split-K space `part`; plain: no autotuning, no profiling
// events, no context workspace
void heff_product(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const void* L, const void* W,
                  const void* R, const void* psi, void* out, void* T1, void* T2, void* psiT, void* part,
                  size_t part_cap, bool plain);
// allocation-free H_eff (noalloc.hip): bytes of scratch a product needs, the
// per-device scratch set-up (d3s_create) and the product itself
size_t noalloc_bytes(d3s_prec p, int ml, int d, int mr, int wl, int wr);
size_t noalloc_capacity();
void noalloc_init(int device);
void op_apply_heff_noalloc(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const void* L,
                           const void* W, const void* R, const void* psi, void* out);
void op_apply_heff_two_site(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wc, int wr, const void* L,
                            const void* W1, const void* W2, const void* R, const void* psi2, void* out);
void op_apply_cwf(Ctx* c, d3s_prec p, int mlp, int mr, int wr, const void* Lt, const void* R, const void* C,
                  void* out);
void cwf_environment(Ctx* c, int ml, int d, int wl, int wr, const double* L, const double* W, double* Lt);
void mpo_square(Ctx* c, const double* W, double* W2, int wl, int wr, int d);
void residual_metric(Ctx* c, const double* env, const double* h2, int m, int w, double* G);
void scale2d_f64(Ctx* c, double* x, long ld, long rows, long cols, double f);
void op_update_env_h2(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* env_in,
                      const double* W, const double* site, double* env_out);
void op_residual_gram(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                      const double* R, const double* h2, const double* W, const double* psi, double energy,
                      double alpha, double* gram);
void op_expand(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
               const double* env, const double* W, const double* psi, double alpha, double* Mt);
void op_update_env(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                   const double* env_in, const double* W, const double* site, double* env_out);
// ---------------------------------------------------------------- truncation engine (trunc.hip)
// Batches of the eigensolver: per matrix its padded size and the offsets of
// its (column-major) matrix and eigenvalues; matrices of a bucket share a size.
// one batched solve: `batch` matrices of size n stored consecutively from G
// + goff (column-major n x n each), eigenvalues from V + voff
struct EigCall { int n, batch; long goff, voff; };
struct EigPlan {
  std::vector<int> npad;
  std::vector<long> goff, voff;
  std::vector<int> bucket_n;
  std::vector<std::vector<int>> members;
  std::vector<long> bucket_goff, bucket_voff;
  long gtot = 0, vtot = 0;
  // the solves and, when they run concurrently, the worker of each
  std::vector<EigCall> calls;
  std::vector<int> worker;
  int workers = 1;
};
// the calls on `workers` threads at once (divide and conquer); returns when
// all have completed; D3S_EDEVICE on a failed or unconverged solve
void eig_calls_parallel(Ctx* c, const std::vector<EigCall>& calls, const std::vector<int>& worker, int workers,
                        double* G, double* V);
void eig_pool_destroy(Ctx* c);
EigPlan plan_eig(Ctx* c, const std::vector<int>& n);          // n[q] <= 0: matrix q not in the plan
// normalise every matrix (largest diagonal entry 1, padded diagonal -1) and
// solve; scale[q] multiplies matrix q's eigenvalues back
void eig_run(Ctx* c, const EigPlan& ep, const std::vector<int>& n, double* G, double* V,
             std::vector<double>& scale);
// A set of matrices truncated together: X_q (nr[q] x nc[q], row-major, row
// stride nc[q]) at X + xoff[q]; the singular vectors sought are the left ones.
struct TruncMats {
  const double* X = nullptr;
  std::vector<long> xoff;
  std::vector<int> nr, nc;
};
// `count` unit vectors of length nr: vector j at base + start + j*step, elements contiguous
struct TruncVecSeg { const double* base; long start, step; int count; };
struct TruncSel {
  std::vector<std::vector<double>> s;            // per matrix: accepted singular values, descending
  std::vector<std::vector<TruncVecSeg>> vecs;    // per matrix: their left singular vectors, same order
  std::vector<std::vector<double>> rest;         // per matrix: estimates of the values left unresolved
  std::vector<int> keep;                         // per matrix: kept states (a prefix of s)
  int k = 0;
  double total = 0.0, kept = 0.0;                // sum of all / of the kept squared singular values
};
// Singular values and left singular vectors of every matrix, resolved by
// deflated passes down to what the cut needs, and the global choice of the
// kept states (at most kmax, only s > eps * s_0).  The vectors live in the
// context's workspace until the next truncation.  Synchronises.
void trunc_solve(Ctx* c, const TruncMats& tm, int kmax, double eps, TruncSel& out);
// copies of elements [e0, e0 + ne) of the kept vectors of matrix q:
// dst[dst_off + j*dst_js + (e - e0)*dst_es] = vector_j[e], grouped by source buffer
void kept_copies(const TruncSel& sel, int q, int e0, int ne, long dst_off, long dst_js, long dst_es,
                 std::map<const double*, std::vector<CopyDesc>>& out);
void run_copies(Ctx* c, const std::map<const double*, std::vector<CopyDesc>>& cp, double* dst);
// X[r*ld + col] *= f[r] for r < rows, col < cols (f on the host)
void scale_rows_f64(Ctx* c, double* X, long ld, int rows, int cols, const std::vector<double>& f);

struct TruncResult { int k; double discarded; double total; };
TruncResult op_truncate(Ctx* c, d3s_dir dir, int ml, int d, int mr, long width,
                        const double* Mt, const double* psi, int kmax, double eps,
                        const double* nbr, long nbr_other, double* site_out, double* nbr_out,
                        double* s_host, bool renormalize);
// The exact-residual expanded tensor on an orthonormal basis of its far-side
// vectors: L2R [psi | alpha Zc F] ((ml d) x (mr + r)), R2L [psi ; alpha F^T Zc]
// ((ml + r) x (d mr)), G = F F^T the metric; returns the width (L2R) or row
// count (R2L) mr + r / ml + r.
long op_residual_expand(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                        const double* R, const double* h2, const double* W, const double* psi, double energy,
                        double alpha, double* Mt);
struct LanczosResult { double theta; int matvecs; bool converged; int restarts; int f64_matvecs = 0; };
LanczosResult op_lanczos(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr,
                         const double* L, const double* W, const double* R, double* psi,
                         double tol, int kmax, int max_matvecs);
double op_energy(Ctx* c, int ml, int d, int mr, int wl, int wr, const double* L,
                 const double* W, const double* R, const double* psi);
void op_heff_grad_W(Ctx* c, int ml, int d, int mr, int wl, int wr, const double* L,
                    const double* R, const double* psi, const double* ybar, double* Wbar);

double op_prepare(Ctx* c, d3s_state* s, double eps);
void op_sweep(Ctx* c, d3s_state* s, d3s_sweep_params* p, d3s_sweep_stats* st);
void op_gradients(Ctx* c, d3s_state* s, double** grads);

// ---------------------------------------------------------------- symmetry blocks
// Charge sectors of one bond, states ordered by sector.
struct Sectors {
  int nq = 1, n = 0, total = 0;
  std::vector<int> q, dim, off;
  std::unordered_map<long, int> index;
  Sectors() = default;
  Sectors(int nq, int n, const int* q, const int* dim);
  int find(const int* charge) const;   // -1 if the charge has no sector
};

// Packed layout of an environment on a bond with w channels: the allowed
// blocks (i, c) (partner sector of q_i - Delta_c), each dim_i x dim_partner
// row-major, one after the other.
struct EnvPack {
  std::vector<long> off;   // at i*w + c, -1 if forbidden
  long total = 0;
};
EnvPack build_envpack(const Sectors& s, const int* wq, int w);

// One tile (at most 32 x 32) of a block relayout: the destination tile
// (prows x pcols at dst, row stride dst_ld) receives the source entries
// (rows x cols at src, row stride src_ld) converted to its element type and
// zeros in the rest.
struct RlTile { long src, dst; int src_ld, dst_ld, rows, cols, prows, pcols; };
enum { RL_F64 = 0, RL_F32 = 1, RL_BF16 = 2 };
void relayout_tiles(Ctx* c, int in_kind, int out_kind, const void* in, void* out, const RlTile* tiles, int ntiles);
struct LowpTwin;

// One tile (at most 32 x 32) of a batched block transpose:
// out[dst + c*dst_ld + r] = in[src + r*src_ld + c] for r < rows, c < cols.
struct TrTile { long src, dst; int src_ld, dst_ld, rows, cols; };
void transpose_tiles(Ctx* c, int esz, const void* in, void* out, const TrTile* tiles, int ntiles);

// Grouped-GEMM plans of one block-sparse H_eff (and its captured graph).
struct BlockHeff {
  Ctx* owner = nullptr;                  // context whose allocator holds the device tables
  int ml = 0, mr = 0, d = 0, wl = 0, wr = 0;
  Sectors left, right;                   // the bonds the plan was built for
  std::vector<int> pq, wql, wqr;         // charges: physical (d*nq), MPO bonds (wl*nq, wr*nq)
  // psi / out layout of the H_eff products: dense (ml, d, mr), or packed:
  // the allowed blocks (i, s) one after the other, each dim_i x dim_j row-major
  bool packed = false;
  std::vector<long> poff;                // packed offset of block (i, s) at i*d + s, -1 if forbidden
  long npacked = 0;
  // environment layout: dense (m, w, m), or packed (L and new R on the left
  // bond: epl; R and new L on the right bond: epr)
  bool penv = false;
  EnvPack epl, epr;
  GroupedPlan g1, g2;                    // H_eff: GEMM-1 and GEMM-2
  // GEMM-1 on the block-transposed psi (K-contiguous B operand: block (i, t)
  // stored dim_j x dim_i at poff), used for FP32 / BF16 products (built for
  // the padded twins, which run them); the tiles of the block transpose
  // (device table)
  GroupedPlan g1t;
  TrTile* d_trt = nullptr;
  int ntrt = 0;
  // FP32 / BF16 products run on a twin plan whose sector dimensions are
  // rounded up to multiples of 8 (every block offset and row length a
  // multiple of 16 bytes, so the GEMM operand loads are whole 16-byte
  // vectors); built on first use; `padded` marks a twin
  LowpTwin* lp = nullptr;
  bool padded = false;
  int g2_split = 1;                      // GEMM-2 split-K factor (packed outputs)
  WmapPlan wm;                           // H_eff: T1 -> T2
  // built on first use:
  WmapPlan wm_x;                         // L2R expansion: T1 -> P columns of [psi | P]
  GroupedPlan g_el;                      // L2R environment: site^T * T2
  GroupedPlan g_y;                       // R2L: Y = psi * R^T
  WmapPlan wm_yx;                        // R2L expansion: Y -> P rows of [psi ; P]
  WmapPlan wm_yz;                        // R2L environment: Y -> Z
  GroupedPlan g_er;                      // R2L environment: site * Z^T
  double flops = 0.0;
  void* graph = nullptr;
  void* graph_exec = nullptr;
  void* cap_stream = nullptr;
  void* ev_in = nullptr;
  void* ev_out = nullptr;
  const void* graph_key[9] = {};
  int graph_prec = -1;
};
// The padded twin of a plan and the relayout tables between the plan's
// layouts (dense or packed) and the twin's packed ones: L and R into the
// twin's packed environments, psi into its packed blocks, and the product
// back into the plan's psi layout.
struct LowpTwin {
  BlockHeff h;
  RlTile *d_L = nullptr, *d_R = nullptr, *d_X = nullptr, *d_Y = nullptr;
  int nL = 0, nR = 0, nX = 0, nY = 0;
  // an operator bound by op_block_bind: L, R in the twin's layouts and the
  // product's element type, W in FP32 (owned, from the plan owner's allocator)
  void *bL = nullptr, *bR = nullptr, *bW = nullptr;
  d3s_prec bprec = D3S_F64;                 // D3S_F64: nothing bound
  d3s_prec prec = D3S_F32;                  // precision its tile sizes were chosen for
};
// built on the first FP32 / BF16 product; its grouped launches are tuned
// (autotuning on) in that product's precision
LowpTwin& ensure_lowp(Ctx* c, BlockHeff& h, d3s_prec p);
void build_block_heff(Ctx* c, BlockHeff& h, const Sectors& left, const Sectors& right, int d, int wl, int wr,
                      const int* phys_q, const int* wq_left, const int* wq_right, bool packed = false,
                      bool with_g2 = true, bool packed_env = false, bool with_psit = false);
// elements of the L / R operands of a plan (packed or dense)
inline long plan_nl(const BlockHeff& h) { return h.penv ? h.epl.total : (long)h.ml * h.wl * h.ml; }
inline long plan_nr(const BlockHeff& h) { return h.penv ? h.epr.total : (long)h.mr * h.wr * h.mr; }
// dense (ml, d, mr) site tensor <-> packed blocks of a packed plan; unpack
// clears the rest of the dense tensor; `rowlen` is the length of a dense
// (a, s) row (mr for a site tensor, (1+wr)*mr for [psi | P]).
void pack_psi(Ctx* c, const BlockHeff& h, const double* dense, double* packed);
void unpack_psi(Ctx* c, const BlockHeff& h, const double* packed, double* dense, long rowlen, bool clear);
void release_block_heff(BlockHeff& h);
// y = H x (FP64 vectors in the plan's layout) with an FP32 / BF16 product on
// the twin: x moved into the twin's layout and precision (xin), the product
// into yout (FP32), moved back into y (whose forbidden entries are cleared
// for a dense layout)
void lowp_product(Ctx* c, BlockHeff& h, LowpTwin& tw, d3s_prec p, const void* Lc, const void* Wc, const void* Rc,
                  const double* x, double* y, void* xin, float* yout, bool use_graph);
// bind an operator (FP64 L, W, R in the plan's layouts) for FP32 / BF16
// products, and apply it
void op_block_bind(Ctx* c, BlockHeff& h, d3s_prec p, const double* L, const double* W, const double* R);
void op_apply_heff_blocks_bound(Ctx* c, BlockHeff& h, const double* psi, double* out, bool use_graph);
void op_apply_heff_blocks(Ctx* c, BlockHeff& h, d3s_prec p, const void* L, const void* W, const void* R,
                          const void* psi, void* out, bool use_graph);
// Block-sparse expansion (FP64): writes the allowed blocks of Mt = [psi | P]
// (L2R, env = L, row length (1+wr)*mr) or [psi ; P] (R2L, env = R, row length
// d*mr) and zeroes the rest.
void op_expand_blocks(Ctx* c, BlockHeff& h, d3s_dir dir, const double* env, const double* W, const double* psi,
                      double alpha, double* Mt);
// Block-sparse environment update (FP64) for a site tensor on the plan's bonds.
void op_update_env_blocks(Ctx* c, BlockHeff& h, d3s_dir dir, const double* env_in, const double* W,
                          const double* site, double* env_out);
// <psi|H_eff|psi> / <psi|psi> with the block H_eff (FP64)
double op_energy_blocks(Ctx* c, BlockHeff& h, const double* L, const double* W, const double* R,
                        const double* psi);

// Charges of one symmetric chain (host copies of the caller's d3s_symmetry).
struct SymChain {
  int nq = 1;
  long env_cap = 0;                      // elements per environment buffer
  std::vector<int> phys;                 // d*nq
  std::vector<std::vector<int>> wq;      // per MPO bond b: w[b]*nq
  std::vector<Sectors> bonds;            // per MPS bond b = 0..l
};
int charge_lkey(const int* q, int nq);   // linear key: key(q1 + q2) = key(q1) + key(q2)

struct TruncBlocksResult {
  int k = 0;
  double discarded = 0.0, total = 0.0;
  std::vector<int> q, dim;               // sectors of the new bond
};
// Block-diagonal truncation (per charge sector of the truncated bond) of the
// expanded tensor; the neighbour update is the dense product on the
// structured layout.  `wq_exp`: channel charges of the expanded MPO bond
// (nullptr / wexp = 0 when Mt holds psi only).
TruncBlocksResult op_truncate_blocks(Ctx* c, d3s_dir dir, const Sectors& left, const Sectors& right, int d,
                                     const int* pq, const int* wq_exp, int wexp, long width, const double* Mt,
                                     const double* psi, int kmax, double eps, const double* nbr, long nbr_other,
                                     double* site_out, double* nbr_out, bool renormalize);
double op_prepare_blocks(Ctx* c, d3s_state* s, SymChain& sym, double eps);
void op_sweep_blocks(Ctx* c, d3s_state* s, SymChain& sym, d3s_sweep_params* p, d3s_sweep_stats* st,
                     bool use_graph);
// Lanczos with block-sparse products on a dense site tensor psi.  With a
// packed plan the Krylov vectors hold only the allowed blocks (length
// plan.npacked); the Ritz vector is written back to psi (dense, forbidden
// entries zero) and, when `packed_out` is given, also kept there packed.
LanczosResult op_lanczos_blocks(Ctx* c, d3s_prec p, BlockHeff& plan, const double* L, const double* W,
                                const double* R, double* psi, double tol, int kmax, int max_matvecs,
                                bool use_graph, double* packed_out = nullptr);
void syevd_batched_f64(Ctx* c, int n, int batch, double* A, double* evals);
// the batched eigensolver of the truncations: an LDS-resident solver for
// n <= kEigSmallMax (eigensolver kind 3), rocSOLVER otherwise
constexpr int kEigSmallMax = 128;
bool eig_small_used(const Ctx* c, int n);
void eig_batched_f64(Ctx* c, int n, int batch, double* A, double* evals);

// lowest eigenpair of a symmetric tridiagonal matrix (bisection + inverse iteration)
bool tridiag_lowest(int n, const double* a, const double* b, double* theta, double* y);
// host symmetric eigensolver (cyclic Jacobi) for small tridiagonal projections
void jacobi_eigh(int n, std::vector<double>& A, std::vector<double>& evals,
                 std::vector<double>& evecs);


double read_scalar(Ctx* c, const double* dev);

}  // namespace d3s
