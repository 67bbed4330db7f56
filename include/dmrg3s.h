/*
 * dmrg3s.h -- C-ABI of the MI355X hot path of strictly single-site DMRG with
 * subspace expansion (DMRG3S; Hubig, McCulloch, Schollwoeck, Wolf).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All tensors are real, dense and row-major.  Tensor pointers are DEVICE
 *    pointers owned by the caller unless a comment says "host".  The library
 *    never frees caller memory; it owns only its workspace (Sec. "Ownership").
 *  - Index names follow the paper's notation:
 *      L[a, w, x]    (m_l, w_l, m_l)   left environment L_{i-1}; a bra, x ket
 *      W[w, v, s, t] (w_l, w_r, d, d)  MPO tensor W_i; s out (bra), t in (ket)
 *                                      (the paper's (d, d, w, w), permuted)
 *      psi[x, t, y]  (m_l, d, m_r)     site tensor M_i (paper: (d, m, m), permuted)
 *      R[b, v, y]    (m_r, w_r, m_r)   right environment R_{i+1}; b bra, y ket
 *  - Dimensions are ints >= 1.  Every call checks shapes, nulls and enums
 *    before any launch and returns D3S_EINVAL with a message (d3s_last_error)
 *    when they are wrong.  HIP / rocSOLVER failures return D3S_EDEVICE.
 *  - Calls are stream-ordered on the context's stream and asynchronous unless
 *    they return host values (truncate, energy, lanczos, sweep, prepare),
 *    which synchronise the stream.
 *  - No exception and no abort crosses this boundary.
 *
 * Ownership
 * ---------
 *  The context owns a grow-only workspace (intermediates T1/T2, Krylov basis,
 *  Gram matrix, eigen-workspace).  It is allocated with the optional
 *  allocator callbacks (stream-ordered) or with hipMalloc, and released by
 *  d3s_destroy.  rocSOLVER, used for the FP64 symmetric eigensolve of the
 *  truncation, allocates its own internal workspace.
 */
#ifndef DMRG3S_H
#define DMRG3S_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  D3S_OK = 0,
  D3S_ENOCONV = 1,   /* warning: the eigensolver hit its limit; the output is the best Ritz pair */
  D3S_EINVAL = -1,   /* bad argument (shape, null pointer, enum) -- nothing was launched */
  D3S_ENOMEM = -2,   /* workspace allocation failed */
  D3S_EDEVICE = -3,  /* HIP or rocSOLVER error */
  D3S_ENUMERIC = -4  /* non-finite energy or norm */
} d3s_status;

/* Arithmetic of the contractions.  Element types of the tensor pointers:
 *  D3S_F64 : every tensor double.
 *  D3S_F32 : every tensor float (FP32 MFMA, FP32 accumulation).
 *  D3S_BF16: L, R, psi bfloat16 (uint16 bits), W float, out float
 *            (BF16 MFMA with FP32 accumulation). */
typedef enum { D3S_F64 = 0, D3S_F32 = 1, D3S_BF16 = 2 } d3s_prec;

/* Sweep direction of a site update: left-to-right expands the right bond
 * of the site, right-to-left its left bond (Sec. 4.1). */
typedef enum { D3S_L2R = 0, D3S_R2L = 1 } d3s_dir;

typedef struct d3s_ctx_s* d3s_ctx;

/* Optional stream-ordered allocator for the workspace; NULL = hipMalloc. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} d3s_allocator;

/* Create a context on `device` issuing work on `stream` (a hipStream_t;
 * NULL = the null stream).  `alloc` may be NULL.  *ctx is set on success. */
d3s_status d3s_create(d3s_ctx* ctx, int device, void* stream, const d3s_allocator* alloc);
/* Release the workspace and the context.  NULL is ignored. */
void d3s_destroy(d3s_ctx ctx);
/* Message of the last non-OK status on this context ("" if none).  Owned by
 * the context, valid until the next call on it. */
const char* d3s_last_error(d3s_ctx ctx);
/* Change the stream of a context. */
d3s_status d3s_set_stream(d3s_ctx ctx, void* stream);
/* Wait for all work issued on the context's stream. */
d3s_status d3s_synchronize(d3s_ctx ctx);
/* Library version string (host, static). */
const char* d3s_version(void);
/* GEMM tile configuration: -1 = size heuristic (default), 0 = 128x128
 * block tiles (4 waves of 64x64), 1 = 64x64 (4 waves of 32x32), 2 = 256x128
 * (8 waves of 64x64), 3 = 128x128 (8 waves of 64x32), 4 = 256x128 (4 waves
 * of 128x64; FP32 and BF16, FP64 runs 2). */
d3s_status d3s_set_tile_config(d3s_ctx ctx, int cfg);
/* Tile configuration of the grouped block-sparse launches of plans built
 * afterwards: -1 = chosen per launch by a work model (or by timing, with
 * autotuning on; default), 0 = 128x128 tiles, 1 = 64x64, 2 = 96x96,
 * 3 = 32x32 (four waves each), 4 = 128x128 (eight waves), 5 = 256x128
 * (eight waves). */
d3s_status d3s_set_grouped_tile(d3s_ctx ctx, int cfg);
/* Split-K of the second grouped GEMM in the block sweeps' H_eff (packed
 * vectors): from min_gflop GFLOP of that product on (default 1.0; < 0 never),
 * when its output blocks give too few tiles to fill the device, each
 * block's channel segments are dealt to up to four partial outputs that are
 * summed afterwards in a fixed order (results stay deterministic). */
d3s_status d3s_set_block_split(d3s_ctx ctx, double min_gflop);
/* Autotuning of tile configurations (default off: a size heuristic picks
 * them).  When on, the first dense GEMM of every shape class (precision,
 * layouts, M, N, K) is timed in all tile configurations with HIP events and
 * the fastest is kept, and block plans time both tile sizes of their grouped
 * launches when they are created.  cache_path (may be NULL) names a text file
 * of "key config" lines read now and appended to on every new decision.
 * Tuning never happens during graph capture or for accumulating products. */
d3s_status d3s_set_autotune(d3s_ctx ctx, int enable, const char* cache_path);
/* Batched eigensolver of the per-sector Gram matrices in the block-sparse
 * truncation (FP64): kind 1 = rocSOLVER divide and conquer (syevd), 2 =
 * rocSOLVER Jacobi (syevj), 0 = Jacobi for sizes <= jacobi_max_n and divide
 * and conquer above (the default: kind 0, jacobi_max_n 0, i.e. syevd),
 * 3 = the library's own solver for n <= 128 (one workgroup per matrix with
 * the matrix in LDS: Householder tridiagonalisation and implicit QL; faster
 * than rocSOLVER only on batches of matrices of a few tens of rows) and
 * divide and conquer above.  All give the eigenpairs to FP64 accuracy
 * (eigenvectors of repeated eigenvalues may differ by a rotation within
 * their eigenspace); only the speed differs.  D3S_EINVAL outside 0..3. */
d3s_status d3s_set_eigensolver(d3s_ctx ctx, int kind, int jacobi_max_n);
/* Concurrency of the truncations' divide-and-conquer solves (Sec. 5 step 4
 * on a GPU): rocSOLVER's solver is bound by its per-column launch sequence,
 * so the batched calls of one truncation (groups of sector matrices) are
 * split into `workers` shares that run at once: one on the calling thread
 * and the context's stream, the others on host threads with their own
 * streams and rocBLAS handles (default 4; 1 = one call after the other).  A
 * call of several matrices may be halved to balance the shares.  The
 * results are those of the one-at-a-time solves up to rounding (the
 * grouping into calls may differ).  D3S_EINVAL outside 1..8. */
d3s_status d3s_set_eig_workers(d3s_ctx ctx, int workers);
/* The mixed-precision eigensolver's two phases (FP32 / BF16 products, see
 * d3s_lanczos): Lanczos on the low-precision operator stops at relative
 * residual `low_tol` (<= 0: 1e-6 for FP32, 3e-3 for BF16, the defaults);
 * each FP64 refinement step then solves its correction equation with at
 * most `inner_max` low-precision conjugate-gradient steps, until the inner
 * residual is below `eta` times the outer one (defaults 0.1 and 20).  A
 * smaller eta spends more low-precision products per FP64 product.  The
 * converged eigenpair meets the same FP64 residual tolerance whatever the
 * setting.  D3S_EINVAL unless 0 < eta < 1, 1 <= inner_max <= 1000 and
 * low_tol < 1. */
d3s_status d3s_set_refinement(d3s_ctx ctx, double eta, int inner_max, double low_tol);
/* The batched FP64 symmetric eigensolver of the truncations (a6): `batch`
 * matrices of size n, column-major, stored one after the other in A
 * (device, n*n*batch), are replaced by their eigenvectors (columns) and W
 * (device, n*batch) receives the eigenvalues in ascending order; the solver
 * is the one chosen by d3s_set_eigensolver.  Each matrix is divided by its
 * largest diagonal entry before the solve and its eigenvalues scaled back
 * (rocSOLVER's divide and conquer loses accuracy in proportion to a small
 * matrix norm).  Synchronises; D3S_EDEVICE if an eigensolve did not converge. */
d3s_status d3s_eig_batched(d3s_ctx ctx, int n, int batch, double* A, double* W);
/* Split-K of GEMMs whose tiles cannot fill the device (default on; the
 * partial products are summed in a fixed order, so results stay
 * deterministic).  enable = 0 turns it off. */
d3s_status d3s_set_splitk(d3s_ctx ctx, int enable);

/*
 * H_eff * psi  (eq. es-iter, Sec. 5):
 *   out[a,s,b] = sum_{w,v,x,t,y} L[a,w,x] W[w,v,s,t] psi[x,t,y] R[b,v,y]
 * contracted in the order (((L psi) W) R) of Sec. 5: a GEMM over the left
 * MPS bond (M = m_l w_l, K = m_l, N = d m_r), the W-map over (w, t), and a
 * GEMM over (v, y) (M = m_l d, K = w_r m_r, N = m_r).
 * Element types follow `prec` (see d3s_prec).  `out` must not alias an input.
 * Asynchronous.
 */
d3s_status d3s_apply_heff(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr,
                          const void* L, const void* W, const void* R, const void* psi, void* out);

/*
 * H_eff * psi with no device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same product as d3s_apply_heff (same arguments, element
 * types and results up to rounding), but its intermediates -- T1 (ml wl d mr
 * elements: double for D3S_F64, float otherwise), T2 and the K-contiguous
 * copy of psi (ml d wr mr and ml d mr elements of the operand type) -- and
 * the split-K partial products live in a 64 MiB array of device memory that
 * the library holds per GPU until the process ends (set up by d3s_create;
 * no autotuning, no profiling events).  A product whose intermediates need
 * more than 64 MiB (each rounded up to 256 bytes) returns D3S_EINVAL before
 * any launch; e.g. d = 4, w = 6 in FP64 fits up to m_l = m_r = 400.  Every
 * call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (other streams, other contexts) race.  Asynchronous on the context's stream.
 */
d3s_status d3s_apply_heff_noalloc(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr,
                                  const void* L, const void* W, const void* R, const void* psi, void* out);

/* Per-kernel timing of d3s_apply_heff: while enabled, HIP events are
 * recorded on the context's stream around each of its three launches (GEMM
 * over the left bond, W-map, GEMM over (v, y)) for up to `capacity` calls.
 * d3s_profile_end synchronises, writes the summed milliseconds of the three
 * kernels to total_ms[0..2] (host) and the number of timed calls to *count,
 * and disables the recording. */
d3s_status d3s_profile_begin(d3s_ctx ctx, int capacity);
d3s_status d3s_profile_end(d3s_ctx ctx, double* total_ms, int* count);

/*
 * Subspace expansion (Sec. 4.1) with the expansion term of eq. subexp-ourt
 * (Sec. 4.2), FP64:
 *   L2R: P[a,s,v,y] = alpha sum L[a,w,x] W[w,v,s,t] psi[x,t,y]
 *        Mtilde = [psi | P], an (m_l d) x (m_r + w_r m_r) row-major matrix:
 *        row (a,s), columns y (psi) then (v,y) (P).  `env` is L (m_l, w_l, m_l).
 *   R2L: P[w,a,s,b] = alpha sum W[w,v,s,t] psi[a,t,y] R[b,v,y]
 *        Mtilde = [psi ; P], an (m_l + w_l m_l) x (d m_r) row-major matrix:
 *        rows a (psi) then (w,a) (P), column (s,b).  `env` is R (m_r, w_r, m_r).
 * The zero block of the neighbour (Sec. 4.1) is never materialised.
 * Asynchronous.
 */
d3s_status d3s_expand_subspace(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                               const double* env, const double* W, const double* psi,
                               double alpha, double* Mtilde);

/*
 * Truncation of the expanded bond and absorption into the neighbour
 * (steps 4-5 of the site update, Sec. 5; cost discussion in Sec. 4.2), FP64.
 *   L2R: Mtilde is (m_l d) x width.  Its top-k left singular vectors U_k give
 *        site_out = U_k as (m_l, d, k).  The neighbour B (m_r x nbr_other,
 *        i.e. (m_r, d', m') flattened) becomes nbr_out = (U_k^T psi_mat) B,
 *        k x nbr_other: only the first m_r columns of S V^T meet the nonzero
 *        rows of the zero-padded neighbour.
 *   R2L: Mtilde is width x (d m_r).  Its top-k right singular vectors give
 *        site_out = V_k^T as (k, d, m_r).  The neighbour A (nbr_other x m_l)
 *        becomes nbr_out = A (psi_mat V_k), nbr_other x k.
 * k = min(kmax, #{ j : s_j > rel_cutoff * s_0 }).  Singular values come from
 * the FP64 Gram matrix of Mtilde on the site side (an MFMA GEMM) and its
 * eigen-decomposition, refined by deflated passes wherever a single Gram
 * matrix cannot resolve a value that the cut may keep (one pass resolves
 * s_j down to about sqrt(n u) s_0), so the cut is the SVD's down to the
 * FP64 rounding of the singular values (about n u s_0).
 * nbr_in may be NULL, with nbr_other = m_r (L2R) or m_l (R2L): then nbr_out
 * is U_k^T psi_mat = S_k V_k^T (k x m_r), or psi_mat V_k = U_k S_k (m_l x k),
 * the truncated SVD split of a two-site tensor (Mtilde = psi = the two-site
 * tensor as (m_l d) x (d' m_r'), passed with m_r = d' m_r').
 * `renormalize` != 0 scales nbr_out to unit Frobenius norm.
 * s_host (host, may be NULL) receives n = m_l d (L2R) or d m_r (R2L)
 * singular values, descending (zeros beyond the rank; values below the
 * resolution the cut needed are estimates).  *k_out (host) and
 * *discarded (host, sum of the dropped s_j^2) are set.  Synchronises.
 */
d3s_status d3s_truncate(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, long width,
                        const double* Mtilde, const double* psi, int kmax, double rel_cutoff,
                        const double* nbr_in, long nbr_other, double* site_out, double* nbr_out,
                        int renormalize, double* s_host, int* k_out, double* discarded);

/*
 * Two-site H_eff * psi2 (the local problem of two-site DMRG, the comparison
 * method of the numerical examples, Sec. 7.2; its eigenproblem is d times
 * larger than the single-site one):
 *   out[a,s1,s2,b] = sum L[a,w,x] W1[w,v,s1,t1] W2[v,u,s2,t2] psi2[x,t1,t2,y] R[b,u,y]
 * L (ml, wl, ml), W1 (wl, wc, d, d), W2 (wc, wr, d, d), R (mr, wr, mr),
 * psi2 and out (ml, d, d, mr), all dense row-major device arrays.  The same
 * order as the single-site product: GEMM over the left MPS bond, one W-map
 * per site, GEMM over (u, y).  prec D3S_F64 (double everywhere) or D3S_F32
 * (float everywhere).  wl*d, wc*d <= 80.  out must not alias psi2.
 * Asynchronous.
 */
d3s_status d3s_apply_heff_two_site(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wc, int wr,
                                   const void* L, const void* W1, const void* W2, const void* R,
                                   const void* psi2, void* out);

/*
 * Centre-matrix (CWF) form of the H application (Sec. 3.3; its cost
 * O(w (d^2 + d) m^3) is compared with the single-site order in Sec. 5):
 *   Lt[(a,s), v, (x,t)] = sum_w L[a,w,x] W[w,v,s,t]        (d3s_cwf_environment, FP64)
 *   out[(a,s), b] = sum Lt[(a,s),v,(x,t)] C[(x,t),y] R[b,v,y]   (d3s_apply_cwf)
 * Lt is (ml d, wr, ml d); C and out are (mlp, mr) with mlp = ml d.  The
 * application is two GEMMs: over (x,t), then over (v,y).  d3s_apply_cwf
 * takes prec D3S_F64 or D3S_F32 (Lt, R, C and out in that type).  For
 * d3s_cwf_environment w_l <= 32 and W must fit 64 KiB.  Device pointers,
 * caller-owned.  Asynchronous.
 */
d3s_status d3s_cwf_environment(d3s_ctx ctx, int ml, int d, int wl, int wr, const double* L, const double* W,
                               double* Lt);
d3s_status d3s_apply_cwf(d3s_ctx ctx, d3s_prec prec, int mlp, int mr, int wr, const void* Lt, const void* R,
                         const void* C, void* out);

/*
 * Exact-residual expansion (the residual Z = H Psi - E Psi of the Sec. 4
 * opening, used in place of the term of eq. subexp-ourt).  At a site of a
 * left-to-right sweep the residual is taken with its left part projected
 * onto the state's left basis and its right part exact; its coefficients
 * then sit on the right-side vectors |B_y> (from -E Psi) and H_v|B_y> (the
 * right-part MPO operator of channel v applied to them, from H Psi), which
 * are not orthonormal.  Their metric needs the ordinary right environment
 * and the H^2 environment <H_v B_y | H_z B_x>.  Right-to-left mirrors this.
 *
 * d3s_update_env_h2: the H^2 environment update, FP64.  Layouts: L2R env_in
 *   (ml, wl*wl, ml) [a, (w,w'), x], env_out (mr, wr*wr, mr); R2L env_in
 *   (mr, wr*wr, mr), env_out (ml, wl*wl, ml); the channel pair (w,w') at
 *   w*wl + w' (bra channel first).  Boundary environments are 1x1x1 ones.
 *   It is d3s_update_env with the channel-pair MPO
 *   W2[(w,w'),(v,v'),p,q] = sum_r W[w,v,r,p] W[w',v',r,q].  Asynchronous.
 * d3s_residual_gram: the Gram matrix of the expanded tensor on the site
 *   side, gram (n x n): L2R n = ml*d, gram = M M^T + alpha^2 <z|z> with
 *   h2 = the right H^2 environment of the site (mr, wr*wr, mr); R2L
 *   n = d*mr, gram = M^T M + alpha^2 <z|z> with h2 = the left one
 *   (ml, wl*wl, ml).  L, R: the site's ordinary environments; energy: E
 *   (the eigenvalue of the site's local problem).  Costs O((w m)^2 d m) and
 *   a metric of (1+w) m squared: meant for m of a few hundred.  Asynchronous.
 * d3s_residual_expand: the same expanded tensor written out on an
 *   orthonormal basis of the far-side vectors, so that d3s_truncate applies
 *   the same cut as for the expansion term of eq. subexp-ourt.  The metric Q
 *   of those vectors ((1+w) m square) is factored as F F^T through its
 *   eigen-decomposition; its eigenvalues at or below n_Q u lambda_max are
 *   exact linear dependences (the far-side operator of the completed MPO
 *   channel is the identity) and are dropped, leaving r columns of F.
 *   L2R: Mtilde = [M | alpha Zc F], (ml*d) x (mr + r), *extent = mr + r
 *   (the row length); R2L: Mtilde = [M ; alpha F^T Zc], (ml + r) x (d*mr),
 *   *extent = ml + r (the row count).  Mtilde needs room for
 *   (ml*d) x ((2+wr)*mr) (L2R) or ((2+wl)*ml) x (d*mr) (R2L) doubles.
 *   Mtilde Mtilde^T (Mtilde^T Mtilde) equals d3s_residual_gram's matrix.
 *   Synchronises (the rank r is read back).
 */
d3s_status d3s_update_env_h2(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                             const double* env_in, const double* W, const double* site, double* env_out);
d3s_status d3s_residual_gram(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                             const double* R, const double* h2, const double* W, const double* psi, double energy,
                             double alpha, double* gram);
d3s_status d3s_residual_expand(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                               const double* R, const double* h2, const double* W, const double* psi, double energy,
                               double alpha, double* Mtilde, long* extent);

/*
 * Environment update (Sec. 2: L_i = L_{i-1} A_i^+ W_i A_i, R_i = R_{i+1} B_i^+ W_i B_i;
 * step 6 of Sec. 5), FP64.
 *   L2R: env_in = L (m_l, w_l, m_l), site = A (m_l, d, m_r)
 *        -> env_out[b,v,y] = sum L[a,w,x] A[a,s,b] W[w,v,s,t] A[x,t,y], (m_r, w_r, m_r)
 *   R2L: env_in = R (m_r, w_r, m_r), site = B (m_l, d, m_r)
 *        -> env_out[a,w,x] = sum B[a,s,b] W[w,v,s,t] B[x,t,y] R[b,v,y], (m_l, w_l, m_l)
 * Asynchronous.
 */
d3s_status d3s_update_env(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                          const double* env_in, const double* W, const double* site,
                          double* env_out);

/*
 * Smallest eigenpair of H_eff (step 1 of Sec. 5: "an eigensolver targeting
 * the smallest eigenvalue"): Lanczos with full FP64 re-orthogonalisation,
 * warm-started from psi, at most kmax (2..64) Krylov vectors per restart, stopping at
 * residual <= tol * max(1, |theta|) or after max_matvecs products.  psi (FP64,
 * in/out) receives the normalised Ritz vector, *theta (host) the Ritz value,
 * *matvecs (host, may be NULL) the number of H_eff products.
 * `prec` selects the arithmetic of the products: D3S_F64 is the plain path;
 * D3S_F32 / D3S_BF16 run the products on FP32 / BF16 MFMA from cast copies of
 * L, R and recover FP64 accuracy by FP64 residual refinement of the Ritz
 * vector (the Krylov vectors, re-orthogonalisation and tridiagonal problem
 * stay FP64).  Returns D3S_ENOCONV (a warning) when the limit was hit.
 * Synchronises.
 */
/* Host helper of the eigensolver (no GPU involved): the lowest eigenpair of
 * the symmetric tridiagonal matrix with diagonal alpha[0..n) and
 * off-diagonal beta[0..n-1) (the Lanczos projection of Sec. 5 step 1), the
 * eigenvalue by Sturm-sequence bisection, the unit eigenvector y[0..n) by
 * inverse iteration (sign: largest component positive).  Host arrays.
 * D3S_EINVAL for bad arguments, D3S_ENUMERIC when no finite vector results. */
d3s_status d3s_tridiag_lowest(int n, const double* alpha, const double* beta, double* theta, double* y);

d3s_status d3s_lanczos(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr,
                       const double* L, const double* W, const double* R, double* psi,
                       double tol, int kmax, int max_matvecs, double* theta, int* matvecs);

/* <psi|H_eff|psi> / <psi|psi> in FP64 (host result).  Synchronises. */
d3s_status d3s_energy(d3s_ctx ctx, int ml, int d, int mr, int wl, int wr, const double* L,
                      const double* W, const double* R, const double* psi, double* energy);

/*
 * Adjoint of H_eff with respect to W (FP64): for y = H_eff(W) psi and a
 * cotangent ybar (m_l, d, m_r),
 *   Wbar[w,v,s,t] = sum_{a,b,x,y} ybar[a,s,b] L[a,w,x] psi[x,t,y] R[b,v,y],
 * shape (w_l, w_r, d, d).  With ybar = psi this is dE/dW of <psi|H_eff|psi>.
 * (The paper is silent on derivatives; this is the exact vector-Jacobian
 * product of the linear map W -> H_eff(W) psi.)  Asynchronous.
 */
d3s_status d3s_heff_grad_W(d3s_ctx ctx, int ml, int d, int mr, int wl, int wr, const double* L,
                           const double* R, const double* psi, const double* ybar, double* Wbar);

/* ---------------------------------------------------------------- symmetry blocks */

/* Charge sectors of one bond (host arrays): sector i holds dim[i] consecutive
 * basis states of charge q[i*nq .. i*nq+nq-1]; the bond dimension is the sum
 * of the dims.  nq = 1 for U(1) (2Sz), 2 for U(1)xU(1) (N, 2Sz). */
typedef struct {
  int nsec;
  const int* q;
  const int* dim;
} d3s_sectors;

typedef struct d3s_block_plan_s* d3s_block_plan;

/* Layouts of the tensors of a block plan.
 * D3S_LAYOUT_DENSE: the dense layouts above (psi (m_l, d, m_r), L (m_l, w_l,
 *   m_l), R (m_r, w_r, m_r)), bond states ordered by sector, zero outside the
 *   allowed blocks.
 * D3S_LAYOUT_PACKED (the block sweeps' layout): only the allowed blocks,
 *   one after the other, each row-major.  psi / out: blocks (i, s) in the
 *   order of the left sector i, then the physical state s, block (i, s)
 *   being dim_i x dim_j with q_j = q_i + q_s (row a, column b).  L: blocks
 *   (i, w) in the order of i, then the channel w, block (i, w) being
 *   dim_i x dim_i' with q_i - q_i' = Delta_w (row a, column x); R likewise on
 *   the right bond.  Missing sectors contribute no block.  Element counts:
 *   d3s_block_plan_sizes. */
typedef enum { D3S_LAYOUT_DENSE = 0, D3S_LAYOUT_PACKED = 1 } d3s_layout;

/* Plan the block-sparse H_eff of one site (the paper uses U(1) symmetries
 * throughout Sec. 7 without describing the blocks; the block rules are the
 * charge-conservation conditions stated here).  Tensors keep the dense layouts above with bond
 * states ordered by sector; psi must vanish outside q_a + q_s = q_b, L outside
 * q_a - q_x = Delta_w and R outside q_b - q_y = Delta_v, where phys_q (d*nq)
 * are the physical charges and wq_left (w_l*nq) / wq_right (w_r*nq) the MPO
 * channel charges Delta.  The plan holds the task tables of the grouped
 * MFMA launches of the two GEMMs of the Sec. 5 ordering and of the block
 * W-map between them.
 * *flops (host, may be NULL) receives the flop count of the allowed block
 * products, *ntasks (may be NULL) the number of block tasks.  Synchronises. */
d3s_status d3s_block_plan_create(d3s_ctx ctx, int nq, int d, int wl, int wr, const d3s_sectors* left,
                                 const d3s_sectors* right, const int* phys_q, const int* wq_left,
                                 const int* wq_right, d3s_block_plan* plan, double* flops, int* ntasks);
/* The same plan for tensors of the given layout (d3s_layout); a plan of the
 * packed layout serves d3s_apply_heff_blocks, d3s_block_plan_bind and
 * d3s_apply_heff_blocks_bound (the expansion, truncation and environment
 * entries below take dense-layout plans: D3S_EINVAL otherwise).
 * d3s_block_plan_create is this call with D3S_LAYOUT_DENSE. */
d3s_status d3s_block_plan_create_layout(d3s_ctx ctx, int nq, int d, int wl, int wr, const d3s_sectors* left,
                                        const d3s_sectors* right, const int* phys_q, const int* wq_left,
                                        const int* wq_right, int layout, d3s_block_plan* plan, double* flops,
                                        int* ntasks);
/* Element counts (host) of L, R and psi / out in the plan's layout.
 * D3S_EINVAL on a null argument. */
d3s_status d3s_block_plan_sizes(d3s_block_plan plan, long* nl, long* nr, long* npsi);
void d3s_block_plan_destroy(d3s_ctx ctx, d3s_block_plan plan);

/* Block-sparse H_eff * psi with a plan: the same result as d3s_apply_heff on
 * symmetric inputs, computing only the allowed blocks; `out` is zero outside
 * the allowed blocks.  use_graph != 0 captures the launches into a hipGraph
 * on first use with these buffers and replays it afterwards (ordered after /
 * before the context's stream by events).  FP32 / BF16 products copy L, R
 * and psi into internal buffers laid out over the sectors with their
 * dimensions rounded up to multiples of 8 (zero-filled, so every block is
 * 16-byte aligned), multiply there and copy the product back; the plan
 * builds the tables of that padded layout on the first such call, which
 * therefore synchronises.  Asynchronous otherwise. */
d3s_status d3s_apply_heff_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_prec prec, const void* L,
                                 const void* W, const void* R, const void* psi, void* out, int use_graph);

/* The low-precision product of the eigensolver (Sec. 5 step 1 with FP32 /
 * BF16 MFMA products; FP64 vectors in and out), with the operator bound once:
 * d3s_block_plan_bind converts FP64 L, W, R (device, the plan's layout) into
 * copies the plan owns (allocated through the context's allocator, released
 * with the plan or by the next bind): L and R in `prec` (D3S_F32 or
 * D3S_BF16; D3S_EINVAL otherwise) in the padded layout of
 * d3s_apply_heff_blocks' low-precision path, W in FP32; the caller's
 * tensors may be freed afterwards.  Synchronises on its first call on a
 * plan (the padded layout's tables are built then).
 * d3s_apply_heff_blocks_bound computes out = H_eff psi with the bound
 * operator: psi (FP64, the plan's layout) is rounded to `prec`, multiplied
 * (FP32 accumulation, T2 in `prec`), and the product is written to out
 * (FP64, the plan's layout; zero outside the allowed blocks).  D3S_EINVAL
 * if nothing is bound or out aliases psi.  use_graph as for
 * d3s_apply_heff_blocks (the graph holds the multiplication; the two
 * conversions are launched around it).  Asynchronous. */
d3s_status d3s_block_plan_bind(d3s_ctx ctx, d3s_block_plan plan, d3s_prec prec, const double* L, const double* W,
                               const double* R);
d3s_status d3s_apply_heff_blocks_bound(d3s_ctx ctx, d3s_block_plan plan, const double* psi, double* out,
                                       int use_graph);

/* Block-sparse expansion of a site on the plan's bonds (Sec. 4.1-4.2, the
 * expansion term of eq. subexp-ourt): the same FP64 result as
 * d3s_expand_subspace on symmetric inputs.  L2R: env = L, Mt = [psi | alpha P]
 * of shape (ml*d) x ((1+wr)*mr); R2L: env = R, Mt = [psi ; alpha P] of shape
 * ((1+wl)*ml) x (d*mr).  Only the allowed blocks are computed (the first GEMM
 * of the Sec. 5 ordering as a grouped launch, then a block W-map writing P
 * straight into Mt); every other entry of Mt is written as zero.  Device
 * pointers, caller-owned.  Asynchronous. */
d3s_status d3s_expand_subspace_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* env,
                                      const double* W, const double* psi, double alpha, double* Mt);
/* Block-diagonal truncation of an expanded tensor on the plan's bonds (steps
 * 4-5 of the site update, Sec. 5; the paper uses U(1) symmetries in Sec. 7):
 * Mt is [psi | alpha P] (L2R, (ml*d) x ((1+wr)*mr)) or [psi ; alpha P] (R2L,
 * ((1+wl)*ml) x (d*mr)) as written by d3s_expand_subspace_blocks.  Every
 * charge Q of the new bond has its own block of Mt (the rows (a,s) with
 * q_a + q_s = Q and the columns of charge Q, or the mirror); each is
 * truncated as in d3s_truncate (same cut: k = min(kmax, #{s_j > rel_cutoff *
 * s_0}) over all sectors together, s_0 the largest of all), and the kept
 * states are ordered by sector.  site_out: L2R (ml*d) x k, R2L k x (d*mr);
 * nbr_out as in d3s_truncate with the neighbour nbr_in (L2R: mr x nbr_other,
 * R2L: nbr_other x ml).  new_q / new_dim (host, room for maxsec sectors of
 * nq charges) receive the sectors of the new bond, *new_nsec their number;
 * D3S_EINVAL if there are more than maxsec.  Synchronises. */
d3s_status d3s_truncate_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* Mt, const double* psi,
                               int kmax, double rel_cutoff, const double* nbr_in, long nbr_other, double* site_out,
                               double* nbr_out, int renormalize, int maxsec, int* new_nsec, int* new_q,
                               int* new_dim, int* k_out, double* discarded);
/* Block-sparse environment update with the site tensor on the plan's bonds
 * (Sec. 2 definitions of L_i and R_i): the same FP64 result as
 * d3s_update_env on symmetric inputs.  L2R: env_in = L (ml, wl, ml),
 * env_out (mr, wr, mr); R2L: env_in = R (mr, wr, mr), env_out (ml, wl, ml).
 * Three grouped launches (first GEMM, block W-map, closing GEMM over the
 * allowed (sector, channel) pairs); env_out is zero outside its allowed
 * blocks.  Asynchronous. */
d3s_status d3s_update_env_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* env_in,
                                 const double* W, const double* site, double* env_out);

/* Charges of a symmetric chain for the block-sparse sweep (host arrays,
 * owned by the caller).  Bond b (0..l) currently has nsec[b] sectors with
 * charges sec_q[b][0..nsec[b]*nq) and dimensions sec_dim[b][0..nsec[b]),
 * states ordered by sector; the arrays hold up to maxsec sectors and are
 * updated in place by d3s_prepare_blocks / d3s_sweep_blocks.  The sum of the
 * dims of bond b must equal the state's m[b].  mpo_q[b] holds the w[b]*nq
 * channel charges of MPO bond b (e.g. from d3s_mpo_fermion_charges; the
 * boundary bonds have one channel of charge 0).  Bond l carries the target
 * charge (the total quantum number of the state). */
typedef struct {
  int nq;
  const int* phys_q;
  const int* const* mpo_q;
  int maxsec;
  int* nsec;
  int* const* sec_q;
  int* const* sec_dim;
  long env_cap;   /* elements of every lenv/renv buffer of the state; 0 = mmax*wmax*mmax.
                     The block calls store environments packed: the allowed blocks (i, c)
                     of a bond (partner sector of q_i - Delta_c), each dim_i x dim_partner
                     row-major, in sector-major then channel order.  A packed environment
                     that would not fit is an error (D3S_EINVAL), never an overflow. */
} d3s_symmetry;

/* ---------------------------------------------------------------- sweeps */

/* A finite MPS with its MPO and environments, all FP64 device buffers owned
 * by the caller (Sec. 2 notation, sites numbered 0..l-1 here):
 *   site[i]  M_i, (m[i], d, m[i+1]), capacity >= mmax*d*mmax doubles
 *   mpo[i]   W_i, (w[i], w[i+1], d, d)
 *   lenv[i]  environment of sites 0..i-1, (m[i], w[i], m[i]),   capacity >= mmax*wmax*mmax
 *   renv[i]  environment of sites i+1..l-1, (m[i+1], w[i+1], m[i+1]), same capacity
 * m (host, l+1 entries, m[0] = m[l] = 1) holds the current bond dimensions and
 * is updated in place; w (host, l+1 entries, w[0] = w[l] = 1).  The
 * orthogonality centre is tracked in `center`. */
typedef struct {
  int l;
  int d;
  int mmax;
  int* m;
  const int* w;
  double** site;
  double* const* mpo;
  double** lenv;
  double** renv;
  int center;
} d3s_state;

typedef struct {
  double alpha;          /* in/out: mixing factor of the expansion term (Sec. 6) */
  int adaptive_alpha;    /* 1: adapt alpha after every site update (Sec. 6); 0: keep it */
  double eps;            /* singular values s_j <= eps * s_0 are dropped (1e-14) */
  double lanczos_tol;    /* residual tolerance of the eigensolver (1e-12) */
  int lanczos_kmax;      /* Krylov vectors per restart (40; 2..64) */
  int lanczos_max_matvecs; /* products per site update (2000) */
  d3s_prec prec;         /* arithmetic of the eigensolver's H_eff products (see d3s_lanczos) */
  double e_before;       /* in/out: energy of the state entering the next site update */
  int m_limit;           /* bond dimension limit of this sweep (<= 0 or > mmax: the state's mmax);
                            lets a run grow m from sweep to sweep in one allocation */
  double mixed_min_gflop; /* with prec = D3S_F32 / D3S_BF16: sites whose H_eff product costs
                             fewer GFLOP (allowed blocks only for block sweeps) use FP64
                             products, since there the products are launch-bound and low
                             precision saves nothing; 0 = every site mixed */
  int expansion;         /* 0: the expansion term P of eq. subexp-ourt (Sec. 4.2);
                            1: the exact residual H Psi - E Psi (Sec. 4 opening), see
                            d3s_residual_gram; dense sweeps only.  The library then keeps
                            the H^2 environments of every bond in its own workspace,
                            sum over bonds of m_b^2 w_b^2 doubles per side */
} d3s_sweep_params;

/* One record per site update (steps 1-8 of Sec. 5). */
typedef struct {
  int site, dir, k, matvecs, f64_matvecs;   /* matvecs: all H_eff products; f64_matvecs: the FP64 ones */
  double e_before, lambda, e_f, alpha, discarded;
  double t_eig, t_expand, t_trunc, t_env, t_energy;  /* seconds */
  double t_trunc_eig;        /* seconds of t_trunc in the batched eigensolves */
  int trunc_passes;          /* Gram passes of the truncation */
  int reserved_;
} d3s_site_record;

typedef struct {
  int capacity;              /* entries available in `records` (>= 2 (l-1)) */
  int count;                 /* out */
  d3s_site_record* records;  /* host array */
  double energy;             /* out: last lambda* of the sweep */
  double seconds;            /* out: wall time of the sweep */
  int nonconverged;          /* out: eigensolves that hit their limit */
} d3s_sweep_stats;

/* Bring a state with Gaussian (or any) site tensors into left-canonical form
 * with its centre on the last site (QR-like gauge through the truncation
 * machinery without expansion), normalise it, set lenv[0] = renv[l-1] = 1,
 * build lenv[1..l-1] and return <Psi|H|Psi> in *energy (host).  Bond
 * dimensions in m are capped at min(mmax, d^b, d^(l-b)).  Synchronises. */
d3s_status d3s_prepare(d3s_ctx ctx, d3s_state* state, double* energy);

/* One full sweep: right-to-left over sites l-1..1, then left-to-right over
 * sites 0..l-2, every site update being steps 1-8 of Sec. 5 with the
 * alpha rule of Sec. 6 when adaptive_alpha is set.
 * Requires the centre on site l-1 (as left by d3s_prepare or a previous
 * sweep).  Synchronises. */
d3s_status d3s_sweep(d3s_ctx ctx, d3s_state* state, d3s_sweep_params* params,
                     d3s_sweep_stats* stats);

/* dE/dW_i of E = <Psi|H|Psi> for every site (FP64): grads[i] (device, host
 * array of l pointers) receives a (w[i], w[i+1], d, d) tensor, the adjoint
 * d3s_heff_grad_W with ybar = psi in the gauge centred on site i.  Summing
 * <grads[i], dW_i/dJ> over sites gives dE/dJ for any MPO parameter J
 * (product rule; equal to <Psi|dH/dJ|Psi>).  Requires the centre on site
 * l-1 (as after d3s_prepare or a sweep); walks the centre to site 0 by uncut
 * truncations, which leave the state unchanged, and rebuilds renv on the way.
 * Synchronises. */
d3s_status d3s_energy_gradients(d3s_ctx ctx, d3s_state* state, double** grads);

/* Block-sparse (U(1) / U(1)xU(1)) twins of d3s_prepare / d3s_sweep.  The
 * site tensors are first projected onto the symmetric subspace defined by
 * the bond sectors in `sym` (entries violating q_a + q_s = q_b are zeroed),
 * then treated exactly as by the dense calls, except that (i) the Lanczos
 * products are block-sparse grouped launches (d3s_apply_heff_blocks),
 * replayed from a hipGraph per site when use_graph != 0, and (ii) the
 * truncation is block-diagonal: one FP64 Gram matrix and one batched
 * rocSOLVER eigensolve per charge sector of the truncated bond, the kept
 * states chosen globally by singular value.  The bond sectors are updated
 * in `sym` after every truncation.  Environments are kept in the packed
 * layout described at d3s_symmetry (so a state swept by these calls needs
 * d3s_prepare before dense calls such as d3s_sweep or d3s_energy_gradients
 * use its environments).  Synchronise. */
d3s_status d3s_prepare_blocks(d3s_ctx ctx, d3s_state* state, d3s_symmetry* sym, double* energy);
d3s_status d3s_sweep_blocks(d3s_ctx ctx, d3s_state* state, d3s_symmetry* sym, d3s_sweep_params* params,
                            d3s_sweep_stats* stats, int use_graph);

/* ---------------------------------------------------------------- models */
/* MPO builders (host arrays, FP64, layout W[w,v,s,t], one block per site,
 * concatenated; offsets[i] = start of site i, dims[i] = w_i for i = 0..l).
 * `out` may be NULL to query the total number of doubles in *total. */
/* Spin-1/2 exchange: H = sum_{i<j<=i+range} J_ij S_i.S_j; J given as an
 * l x range table, J[i*range + r-1] = J_{i,i+r}. */
d3s_status d3s_mpo_spin_exchange(int l, int range, const double* J, double* out, long* offsets,
                                 int* dims, long* total);
/* Spinful fermions: H = -sum t_ij (c+_is c_js + h.c.) + U sum n_up n_dn - sum mu_i n_i,
 * t given as an l x range table like J; Jordan-Wigner strings between partners;
 * site basis (|0>, |up>, |dn>, |updn>). */
d3s_status d3s_mpo_fermion_hopping(int l, int range, const double* t, double U, const double* mu,
                                   double* out, long* offsets, int* dims, long* total);

/* Charges Delta of the MPO channels of the builders above, in their channel
 * order: spins 2 + 3*range channels of 2Sz (nq = 1; S+ / S- / Sz kinds carry
 * +2 / -2 / 0), fermions 2 + 4*range channels of (N, 2Sz) (nq = 2; c+_up F,
 * c+_dn F, F c_up, F c_dn carry (1,1), (1,-1), (-1,-1), (-1,1)); identity
 * and completion channels carry 0.  out: host array of w*nq ints. */
d3s_status d3s_mpo_spin_charges(int range, int* out);
d3s_status d3s_mpo_fermion_charges(int range, int* out);

#ifdef __cplusplus
}
#endif
#endif /* DMRG3S_H */
