// Host-side composition of the kernels into the operations of the site
// update (Sec. 5): H_eff*psi, expansion, truncation, environment update,
// the Lanczos eigensolver and the energy.  Everything here is stream-ordered
// on the context's stream; host values are read back only where the
// algorithm needs them (Ritz values, singular values, norms).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <functional>
#include <map>

#include "d3s_internal.h"

namespace d3s {

// ---------------------------------------------------------------- workspace
void* ws_get(Ctx* c, int slot, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c->ws_cap[slot] >= bytes) return c->ws_ptr[slot];
  size_t cap = std::max(bytes, c->ws_cap[slot] + c->ws_cap[slot] / 4);
  cap = (cap + 255) & ~(size_t)255;
  if (c->ws_ptr[slot]) {
    if (c->has_alloc) c->alloc.free(c->ws_ptr[slot], c->stream, c->alloc.user);
    else {
      D3S_HIP(hipStreamSynchronize(c->stream));
      D3S_HIP(hipFree(c->ws_ptr[slot]));
    }
    c->ws_ptr[slot] = nullptr;
    c->ws_cap[slot] = 0;
  }
  void* p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(cap, c->stream, c->alloc.user);
  } else if (hipMalloc(&p, cap) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (!p) throw Error{D3S_ENOMEM, "workspace allocation of " + std::to_string(cap) + " bytes failed"};
  c->ws_ptr[slot] = p;
  c->ws_cap[slot] = cap;
  return p;
}

void ws_release_all(Ctx* c) {
  for (int s = 0; s < WS_NSLOTS; ++s) {
    if (!c->ws_ptr[s]) continue;
    if (c->has_alloc) c->alloc.free(c->ws_ptr[s], c->stream, c->alloc.user);
    else (void)hipFree(c->ws_ptr[s]);
    c->ws_ptr[s] = nullptr;
    c->ws_cap[s] = 0;
  }
}

void* dev_alloc(Ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(bytes, c->stream, c->alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (!p) throw Error{D3S_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  return p;
}

void dev_free(Ctx* c, void* p) {
  if (!p) return;
  if (c && c->has_alloc) c->alloc.free(p, c->stream, c->alloc.user);
  else (void)hipFree(p);
}

double read_scalar(Ctx* c, const double* dev) {
  D3S_HIP(hipMemcpyAsync(c->host_red, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  return c->host_red[0];
}

static void read_many(Ctx* c, double* host, const double* dev, size_t n) {
  D3S_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
}

static void write_many(Ctx* c, double* dev, const double* host, size_t n) {
  D3S_HIP(hipMemcpyAsync(dev, host, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
}

// ---------------------------------------------------------------- H_eff psi
// (((L psi) W) R), Sec. 5: GEMM over the left MPS bond, W-map, GEMM over (v, y).
void op_apply_heff(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const void* L,
                   const void* W, const void* R, const void* psi, void* out) {
  const size_t tsz = (p == D3S_F64) ? 8 : 4;       // T1 element size (fp32 for BF16 too)
  const size_t t2sz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  const size_t esz = t2sz;
  void* T1 = ws_get(c, WS_T1, tsz * (size_t)ml * wl * d * mr);
  void* T2 = ws_get(c, WS_T2, t2sz * (size_t)ml * d * wr * mr);
  void* psiT = ws_get(c, WS_PSIT, esz * (size_t)ml * d * mr);
  heff_product(c, p, ml, d, mr, wl, wr, L, W, R, psi, out, T1, T2, psiT, nullptr, 0, false);
}

void heff_product(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const void* L, const void* W,
                  const void* R, const void* psi, void* out, void* T1, void* T2, void* psiT, void* part,
                  size_t part_cap, bool plain) {
  hipEvent_t* ev = nullptr;
  if (!plain && c->prof && c->prof_n < c->prof_cap) ev = &c->prof_ev[4 * (size_t)c->prof_n++];
  if (ev) D3S_HIP(hipEventRecord(ev[0], c->stream));
  // GEMM-1's B operand psi[x][(t,y)] runs along N; a copy psi^T[(t,y)][x]
  // runs along K, which keeps the LDS staging of B in 16-byte vector stores
  // (the transposing stores cost most in BF16).  Counted in GEMM-1's time.
  const size_t esz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  transpose_any(c, (int)esz, psi, ml, (long)d * mr, psiT);
  GemmArgs g1{ml * wl, d * mr, ml, L, ml, true, 0, psiT, ml, true, 0, T1, (long)d * mr, 0, 1.0, 0.0, 1};
  g1.part = part;
  g1.part_cap = part_cap;
  if (plain) gemm(c, p, g1);
  else tuned_gemm(c, p, g1);
  if (ev) D3S_HIP(hipEventRecord(ev[1], c->stream));
  wmap_l2r(c, p, T1, W, T2, (long)wr * mr, ml, d, mr, wl, wr, 1.0);
  if (ev) D3S_HIP(hipEventRecord(ev[2], c->stream));
  GemmArgs g2{ml * d, mr, wr * mr, T2, (long)wr * mr, true, 0, R, (long)wr * mr, true, 0, out, mr, 0,
              1.0, 0.0, 1};
  g2.part = part;
  g2.part_cap = part_cap;
  if (plain) gemm(c, p, g2);
  else tuned_gemm(c, p, g2);
  if (ev) D3S_HIP(hipEventRecord(ev[3], c->stream));
}

// ---------------------------------------------------------------- comparison methods
// Two-site H_eff (the two-site DMRG local problem): GEMM over the left MPS
// bond, a W-map per site MPO, GEMM over the right MPO and MPS bonds; the
// W-maps are the single-site one with the second site's (t2, y) as the
// trailing index, then with the first site's (a, s1) as the row.
void op_apply_heff_two_site(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wc, int wr, const void* L,
                            const void* W1, const void* W2, const void* R, const void* psi2, void* out) {
  if (p == D3S_BF16) throw Error{D3S_EINVAL, "two-site H_eff: FP64 or FP32"};
  const size_t esz = (p == D3S_F64) ? 8 : 4;
  const long dm = (long)d * mr;
  void* T1 = ws_get(c, WS_T1, esz * (size_t)std::max((long)ml * wl * d * dm, (long)ml * d * d * wr * mr));
  void* T2 = ws_get(c, WS_T2, esz * (size_t)ml * d * wc * dm);
  GemmArgs g1{ml * wl, (int)(d * dm), ml, L, ml, true, 0, psi2, d * dm, false, 0, T1, d * dm, 0, 1.0, 0.0, 1};
  tuned_gemm(c, p, g1);
  // T1[a, w, t1, (t2, y)] -> T2[(a, s1), (v1, t2, y)]
  wmap_l2r(c, p, T1, W1, T2, (long)wc * dm, ml, d, (int)dm, wl, wc, 1.0);
  // T2[(a, s1), v1, t2, y] -> T3[(a, s1, s2), (v2, y)] (into T1's buffer)
  wmap_l2r(c, p, T2, W2, T1, (long)wr * mr, ml * d, d, mr, wc, wr, 1.0);
  GemmArgs g2{ml * d * d, mr, wr * mr, T1, (long)wr * mr, true, 0, R, (long)wr * mr, true, 0, out, mr, 0,
              1.0, 0.0, 1};
  tuned_gemm(c, p, g2);
}

// Centre-matrix (CWF) application with the enlarged environment
// Lt[(a,s), v, (x,t)]: GEMM over (x,t), then over (v, y).
void op_apply_cwf(Ctx* c, d3s_prec p, int mlp, int mr, int wr, const void* Lt, const void* R, const void* C,
                  void* out) {
  if (p == D3S_BF16) throw Error{D3S_EINVAL, "centre-matrix application: FP64 or FP32"};
  const size_t esz = (p == D3S_F64) ? 8 : 4;
  void* T1 = ws_get(c, WS_T1, esz * (size_t)mlp * wr * mr);
  GemmArgs g1{mlp * wr, mr, mlp, Lt, mlp, true, 0, C, mr, false, 0, T1, mr, 0, 1.0, 0.0, 1};
  tuned_gemm(c, p, g1);
  GemmArgs g2{mlp, mr, wr * mr, T1, (long)wr * mr, true, 0, R, (long)wr * mr, true, 0, out, mr, 0, 1.0, 0.0, 1};
  tuned_gemm(c, p, g2);
}

// ---------------------------------------------------------------- expansion
void op_expand(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* env,
               const double* W, const double* psi, double alpha, double* Mt) {
  if (dir == D3S_L2R) {
    // Mt = [psi | alpha L psi W]  ((ml d) x (mr + wr mr))
    const long ldm = (long)(1 + wr) * mr;
    double* T1 = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * wl * d * mr);
    GemmArgs g1{ml * wl, d * mr, ml, env, ml, true, 0, psi, (long)d * mr, false, 0, T1, (long)d * mr, 0,
                1.0, 0.0, 1};
    gemm_f64(c, g1);
    wmap_l2r(c, D3S_F64, T1, W, Mt + mr, ldm, ml, d, mr, wl, wr, alpha);
    copy2d_f64(c, psi, mr, Mt, ldm, (long)ml * d, mr);
  } else {
    // Mt = [psi ; alpha W psi R]  ((ml + wl ml) x (d mr)); Y[(x,t),(b,v)] = psi R^T over y
    double* Y = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * d * mr * wr);
    GemmArgs g1{ml * d, mr * wr, mr, psi, mr, true, 0, env, mr, true, 0, Y, (long)mr * wr, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);
    wmap_r2l(c, D3S_F64, Y, W, Mt + (long)ml * d * mr, ml, d, mr, wl, wr, alpha);
    copy_f64(c, psi, Mt, (long)ml * d * mr);
  }
}

// ---------------------------------------------------------------- environments
void op_update_env(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* env_in,
                   const double* W, const double* site, double* env_out) {
  if (dir == D3S_L2R) {
    double* T1 = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * wl * d * mr);
    double* T2 = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)ml * d * wr * mr);
    GemmArgs g1{ml * wl, d * mr, ml, env_in, ml, true, 0, site, (long)d * mr, false, 0, T1, (long)d * mr, 0,
                1.0, 0.0, 1};
    gemm_f64(c, g1);
    wmap_l2r(c, D3S_F64, T1, W, T2, (long)wr * mr, ml, d, mr, wl, wr, 1.0);
    // env_out[b][(v,y)] = sum_{(a,s)} A[(a,s)][b] T2[(a,s)][(v,y)]
    GemmArgs g2{mr, wr * mr, ml * d, site, mr, false, 0, T2, (long)wr * mr, false, 0, env_out,
                (long)wr * mr, 0, 1.0, 0.0, 1};
    gemm_f64(c, g2);
  } else {
    double* Y = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * d * mr * wr);
    double* Z = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)wl * ml * d * mr);
    GemmArgs g1{ml * d, mr * wr, mr, site, mr, true, 0, env_in, mr, true, 0, Y, (long)mr * wr, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);
    wmap_r2l(c, D3S_F64, Y, W, Z, ml, d, mr, wl, wr, 1.0);
    // env_out[a][(w,x)] = sum_{(s,b)} B[a][(s,b)] Z[(w,x)][(s,b)]
    GemmArgs g2{ml, wl * ml, d * mr, site, (long)d * mr, true, 0, Z, (long)d * mr, true, 0, env_out,
                (long)wl * ml, 0, 1.0, 0.0, 1};
    gemm_f64(c, g2);
  }
}

// ---------------------------------------------------------------- exact residual
// Environment of the channel pairs of H^2 (the metric of the residual's
// near-side vectors): the ordinary environment update with the channel-pair
// MPO W2 of bond w^2.
void op_update_env_h2(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* env_in,
                      const double* W, const double* site, double* env_out) {
  double* W2 = (double*)ws_get(c, WS_W2, sizeof(double) * (size_t)wl * wl * wr * wr * d * d);
  mpo_square(c, W, W2, wl, wr, d);
  op_update_env(c, dir, ml, d, mr, wl * wl, wr * wr, env_in, W2, site, env_out);
}

// Gram matrix of the expanded tensor with the exact residual
// Z = H Psi - E Psi as its expansion part (far side projected onto the
// state's basis, near side exact):
//   L2R: G = M M^T + alpha^2 Zc Q Zc^T,  Zc = [-E M | L M W]   ((ml d) x (1+wr) mr)
//   R2L: G = M^T M + alpha^2 Zc^T Q Zc,  Zc = [-E M ; W M R]   ((1+wl) ml x (d mr))
// with Q the metric of the near-side vectors (residual_metric) built from
// the ordinary and the H^2 environment of that side.
void op_residual_gram(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                      const double* R, const double* h2, const double* W, const double* psi, double energy,
                      double alpha, double* gram) {
  const double a2 = alpha * alpha;
  if (dir == D3S_L2R) {
    const int n = ml * d, ng = (1 + wr) * mr;
    double* Zc = (double*)ws_get(c, WS_RZ, sizeof(double) * (size_t)n * ng);
    op_expand(c, D3S_L2R, ml, d, mr, wl, wr, L, W, psi, 1.0, Zc);
    scale2d_f64(c, Zc, ng, n, mr, -energy);
    double* Q = (double*)ws_get(c, WS_RMET, sizeof(double) * (size_t)ng * ng);
    residual_metric(c, R, h2, mr, wr, Q);
    double* T = (double*)ws_get(c, WS_RT, sizeof(double) * (size_t)n * ng);
    GemmArgs g1{n, ng, ng, Zc, ng, true, 0, Q, ng, false, 0, T, ng, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);
    GemmArgs g2{n, n, ng, T, ng, true, 0, Zc, ng, true, 0, gram, n, 0, a2, 0.0, 1};
    gemm_f64(c, g2);
    GemmArgs g3{n, n, mr, psi, mr, true, 0, psi, mr, true, 0, gram, n, 0, 1.0, 1.0, 1};
    gemm_f64(c, g3);
  } else {
    const int n = d * mr, ng = (1 + wl) * ml;
    double* Zc = (double*)ws_get(c, WS_RZ, sizeof(double) * (size_t)ng * n);
    op_expand(c, D3S_R2L, ml, d, mr, wl, wr, R, W, psi, 1.0, Zc);
    scale_f64(c, Zc, (long)ml * n, -energy);
    double* Q = (double*)ws_get(c, WS_RMET, sizeof(double) * (size_t)ng * ng);
    residual_metric(c, L, h2, ml, wl, Q);
    double* T = (double*)ws_get(c, WS_RT, sizeof(double) * (size_t)ng * n);
    GemmArgs g1{ng, n, ng, Q, ng, true, 0, Zc, n, false, 0, T, n, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);
    GemmArgs g2{n, n, ng, Zc, n, false, 0, T, n, false, 0, gram, n, 0, a2, 0.0, 1};
    gemm_f64(c, g2);
    GemmArgs g3{n, n, ml, psi, n, false, 0, psi, n, false, 0, gram, n, 0, 1.0, 1.0, 1};
    gemm_f64(c, g3);
  }
}

// ---------------------------------------------------------------- eigensolvers
// `batch` symmetric n x n matrices stored one after the other (column-major);
// eigenvalues ascending into evals[b*n + i], eigenvectors overwrite A.
void syevd_batched_f64(Ctx* c, int n, int batch, double* A, double* evals) {
  if (batch <= 0) return;
  if (!c->solver) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success)
      throw Error{D3S_EDEVICE, "rocblas_create_handle failed"};
    c->solver = h;
  }
  rocblas_handle h = (rocblas_handle)c->solver;
  if (rocblas_set_stream(h, c->stream) != rocblas_status_success)
    throw Error{D3S_EDEVICE, "rocblas_set_stream failed"};
  rocblas_int* info = (rocblas_int*)ws_get(c, WS_INFO, sizeof(rocblas_int) * (size_t)std::max(batch, 16) * 2);
  // Jacobi (one kernel family, few launches) for small matrices, divide and
  // conquer for large ones; d3s_set_eigensolver overrides the choice
  const bool jacobi = (c->eig_kind == 2) || (c->eig_kind == 0 && n <= c->eig_jacobi_max);
  rocblas_status st;
  if (jacobi) {
    double* res = (double*)ws_get(c, WS_EIGTMP, sizeof(double) * (size_t)std::max(batch, 16));
    st = rocsolver_dsyevj_strided_batched(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper, n,
                                          A, n, (rocblas_stride)n * n, 0.0, res, 100, info + batch, evals, n, info,
                                          batch);
  } else {
    double* E = (double*)ws_get(c, WS_EIGTMP, sizeof(double) * (size_t)n * batch);
    st = rocsolver_dsyevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, n, A, n,
                                          (rocblas_stride)n * n, evals, n, E, n, info, batch);
  }
  if (st != rocblas_status_success)
    throw Error{D3S_EDEVICE, "rocsolver batched eigensolver failed (status " + std::to_string((int)st) + ")"};
  std::vector<rocblas_int> hinfo(batch);
  D3S_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * batch, hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  for (int b = 0; b < batch; ++b)
    if (hinfo[b] != 0)
      throw Error{D3S_EDEVICE, "rocsolver batched eigensolver did not converge (info " +
                                   std::to_string(hinfo[b]) + ")"};
}

// Lowest eigenpair of the symmetric tridiagonal matrix with diagonal a[0..n)
// and off-diagonal b[0..n-1): the eigenvalue by bisection on the Sturm
// sequence count (to a few ulps), the eigenvector by inverse iteration with a
// partially pivoted tridiagonal LU factorisation.  O(n) per bisection step.
// Returns false when the iteration did not produce a finite unit vector.
bool tridiag_lowest(int n, const double* a, const double* b, double* theta, double* y) {
  if (n <= 0) return false;
  if (n == 1) {
    *theta = a[0];
    y[0] = 1.0;
    return std::isfinite(a[0]);
  }
  // Gershgorin interval
  double lo = a[0], hi = a[0], scale = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
    scale = std::max(scale, std::fabs(a[i]) + r);
  }
  if (!(scale > 0.0)) {
    *theta = 0.0;
    for (int i = 0; i < n; ++i) y[i] = (i == 0) ? 1.0 : 0.0;
    return true;
  }
  const double tiny = DBL_MIN / DBL_EPSILON;
  // number of eigenvalues < x (Sturm count of the LDL^T pivots of T - x)
  auto count_below = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0.0) ++c;
    for (int i = 1; i < n; ++i) {
      if (std::fabs(q) < tiny) q = (q < 0.0) ? -tiny : tiny;
      q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
      if (q < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 4.0 * DBL_EPSILON * std::max(std::fabs(lo), std::fabs(hi)) + tiny; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double th = 0.5 * (lo + hi);
  *theta = th;
  // inverse iteration on T - th (shifted off the eigenvalue by a few ulps of
  // the matrix scale so that the factorisation is never exactly singular)
  const double shift = th - 8.0 * DBL_EPSILON * scale;
  std::vector<double> d(n), du(n), du2(n), dl(n);
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) d[i] = a[i] - shift;
  for (int i = 0; i + 1 < n; ++i) du[i] = dl[i] = b[i];
  // LU with partial pivoting (rows i, i+1), U has two superdiagonals
  for (int i = 0; i < n; ++i) du2[i] = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {
      piv[i] = i;
      if (std::fabs(d[i]) < tiny) d[i] = tiny;
      const double f = dl[i] / d[i];
      dl[i] = f;
      d[i + 1] -= f * du[i];
      du2[i] = 0.0;
    } else {
      piv[i] = i + 1;
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = d[i + 1];
      d[i + 1] = t - f * d[i + 1];
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
    }
  }
  if (std::fabs(d[n - 1]) < tiny) d[n - 1] = tiny;
  piv[n - 1] = n - 1;
  for (int i = 0; i < n; ++i) y[i] = 1.0 / std::sqrt((double)n) * (1.0 + 1e-3 * (i % 7));
  for (int rep = 0; rep < 3; ++rep) {
    // solve L U x = y: forward with the row interchanges, then back substitution
    for (int i = 0; i + 1 < n; ++i) {
      if (piv[i] == i) {
        y[i + 1] -= dl[i] * y[i];
      } else {
        const double t = y[i];
        y[i] = y[i + 1];
        y[i + 1] = t - dl[i] * y[i + 1];
      }
    }
    y[n - 1] /= d[n - 1];
    if (n >= 2) y[n - 2] = (y[n - 2] - du[n - 2] * y[n - 1]) / d[n - 2];
    for (int i = n - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / d[i];
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
    for (int i = 0; i < n; ++i) y[i] /= nrm;
  }
  // sign convention: largest component positive
  int im = 0;
  for (int i = 1; i < n; ++i)
    if (std::fabs(y[i]) > std::fabs(y[im])) im = i;
  if (y[im] < 0.0)
    for (int i = 0; i < n; ++i) y[i] = -y[i];
  return true;
}

// Cyclic Jacobi eigensolver for a small dense symmetric matrix (row-major A,
// destroyed).  Eigenvalues ascending; evecs[j*n + i] = component i of vector j.
void jacobi_eigh(int n, std::vector<double>& A, std::vector<double>& evals, std::vector<double>& evecs) {
  std::vector<double> V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p) {
      diag += A[(size_t)p * n + p] * A[(size_t)p * n + p];
      for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
    }
    if (off <= 1e-34 * (diag + 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = cs * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = cs * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {   // eigenvector columns
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return A[(size_t)x * n + x] < A[(size_t)y * n + y]; });
  evals.assign(n, 0.0);
  evecs.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    evals[j] = A[(size_t)order[j] * n + order[j]];
    for (int i = 0; i < n; ++i) evecs[(size_t)j * n + i] = V[(size_t)i * n + order[j]];
  }
}

// ---------------------------------------------------------------- truncation
// Steps 4-5 of the site update on a dense expanded tensor: its left (L2R) or
// right (R2L) singular vectors from the truncation engine (the rows of Mt,
// or of its transpose, are the matrix whose left vectors it finds), the new
// site tensor from the kept ones, and the neighbour through U_k^T psi_mat
// (or psi_mat V_k): only that block of S V^T meets the nonzero rows of the
// zero-padded neighbour.
TruncResult op_truncate(Ctx* c, d3s_dir dir, int ml, int d, int mr, long width, const double* Mt,
                        const double* psi, int kmax, double eps, const double* nbr, long nbr_other,
                        double* site_out, double* nbr_out, double* s_host, bool renormalize) {
  const int n = (dir == D3S_L2R) ? ml * d : d * mr;
  TruncMats tm;
  if (dir == D3S_L2R) {
    tm.X = Mt;
  } else {
    double* Xt = (double*)ws_get(c, WS_TR_XT, sizeof(double) * (size_t)n * width);
    transpose_f64(c, Mt, width, n, Xt);
    tm.X = Xt;
  }
  tm.xoff = {0};
  tm.nr = {n};
  tm.nc = {(int)width};
  TruncSel sel;
  trunc_solve(c, tm, kmax, eps, sel);
  if (!(sel.total > 0.0) || !std::isfinite(sel.total))
    throw Error{D3S_ENUMERIC, "truncate: the expanded tensor is zero or not finite"};
  const int k = sel.k;
  if (k <= 0) throw Error{D3S_ENUMERIC, "truncate: no singular value above the cutoff"};
  if (s_host) {
    std::vector<double> all(sel.s[0]);
    all.insert(all.end(), sel.rest[0].begin(), sel.rest[0].end());
    std::sort(all.begin(), all.end(), std::greater<double>());
    for (int j = 0; j < n; ++j) s_host[j] = j < (int)all.size() ? all[j] : 0.0;
  }
  // U_k^T (k x n), one kept vector per row
  double* Ukt = (double*)ws_get(c, WS_UKT, sizeof(double) * (size_t)k * n);
  {
    std::map<const double*, std::vector<CopyDesc>> cp;
    kept_copies(sel, 0, 0, n, 0, n, 1, cp);
    run_copies(c, cp, Ukt);
  }
  if (dir == D3S_L2R) {
    transpose_f64(c, Ukt, k, n, site_out);                      // A = U_k, (ml d) x k
    // without a neighbour (the split of a two-site tensor) X = S_k V_k^T is the output
    double* X = nbr ? (double*)ws_get(c, WS_X, sizeof(double) * (size_t)k * mr) : nbr_out;
    GemmArgs g1{k, mr, n, Ukt, n, true, 0, psi, mr, false, 0, X, mr, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);                                            // X = U_k^T psi_mat
    if (nbr) {
      GemmArgs g2{k, (int)nbr_other, mr, X, mr, true, 0, nbr, nbr_other, false, 0, nbr_out, nbr_other, 0,
                  1.0, 0.0, 1};
      gemm_f64(c, g2);                                          // B~ = X B
    }
  } else {
    copy_f64(c, Ukt, site_out, (long)k * n);                    // B = V_k^T, k x (d mr)
    double* X = nbr ? (double*)ws_get(c, WS_X, sizeof(double) * (size_t)ml * k) : nbr_out;
    GemmArgs g1{ml, k, n, psi, n, true, 0, Ukt, n, true, 0, X, k, 0, 1.0, 0.0, 1};
    gemm_f64(c, g1);                                            // X = psi_mat V_k
    if (nbr) {
      GemmArgs g2{(int)nbr_other, k, ml, nbr, ml, true, 0, X, k, false, 0, nbr_out, k, 0, 1.0, 0.0, 1};
      gemm_f64(c, g2);                                          // A~ = A X
    }
  }
  if (renormalize) {
    const long nn = (long)k * nbr_other;
    double* r = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 512);
    dot_f64(c, nbr_out, nbr_out, nn, r);
    const double nrm2 = read_scalar(c, r);
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
      throw Error{D3S_ENUMERIC, "truncate: neighbour norm is zero or not finite"};
    scale_f64(c, nbr_out, nn, 1.0 / std::sqrt(nrm2));
  }
  return TruncResult{k, std::max(0.0, sel.total - sel.kept), sel.total};
}

// The exact-residual expanded tensor with its expansion part written on an
// orthonormal basis of the far-side vectors |B_y>, H_v|B_y> (L2R; |A_a>,
// H_w|A_a> R2L).  Those vectors are linearly dependent (the far-side
// operator of the completed MPO channel is the identity), so their metric
// Q = F F^T is factored through its eigen-decomposition, eigenvalues at or
// below ng u lambda_max taken as the exact zeros of those dependences:
//   L2R: [M | alpha Zc F],  Zc = [-E M | L M W]  ((ml d) x (mr + r))
//   R2L: [M ; alpha F^T Zc], Zc = [-E M ; W M R] ((ml + r) x (d mr))
// Its SVD is the truncation of the residual expansion; Mt Mt^T (M^T M) is
// the Gram matrix of op_residual_gram.
long op_residual_expand(Ctx* c, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                        const double* R, const double* h2, const double* W, const double* psi, double energy,
                        double alpha, double* Mt) {
  const bool l2r = dir == D3S_L2R;
  const int n = l2r ? ml * d : d * mr;
  const int ng = l2r ? (1 + wr) * mr : (1 + wl) * ml;
  const int mnear = l2r ? mr : ml;
  double* Zc = (double*)ws_get(c, WS_RZ, sizeof(double) * (size_t)n * ng);
  op_expand(c, dir, ml, d, mr, wl, wr, l2r ? L : R, W, psi, 1.0, Zc);
  if (l2r) scale2d_f64(c, Zc, ng, n, mr, -energy);
  else scale_f64(c, Zc, (long)ml * n, -energy);
  double* Q = (double*)ws_get(c, WS_RMET, sizeof(double) * (size_t)ng * ng);
  residual_metric(c, l2r ? R : L, h2, mnear, l2r ? wr : wl, Q);
  double* ev = (double*)ws_get(c, WS_EIGVAL, sizeof(double) * (size_t)ng);
  eig_batched_f64(c, ng, 1, Q, ev);          // the metric holds an identity block: norm >= 1
  std::vector<double> lam(ng);
  read_many(c, lam.data(), ev, ng);
  const double lmax = lam[ng - 1];
  if (!(lmax > 0.0) || !std::isfinite(lmax)) throw Error{D3S_ENUMERIC, "residual: metric is zero or not finite"};
  int r = 0;
  while (r < ng && lam[ng - 1 - r] > (double)ng * DBL_EPSILON * lmax) ++r;
  // F^T (r x ng): eigenvectors ng-r .. ng-1 (rows of the column-major Q) scaled by sqrt(lambda)
  double* Ft = Q + (long)(ng - r) * ng;
  std::vector<double> f(r);
  for (int j = 0; j < r; ++j) f[j] = std::sqrt(lam[ng - r + j]);
  scale_rows_f64(c, Ft, ng, r, ng, f);
  if (l2r) {
    const long ldm = (long)mr + r;
    GemmArgs g{n, r, ng, Zc, ng, true, 0, Ft, ng, true, 0, Mt + mr, ldm, 0, alpha, 0.0, 1};
    gemm_f64(c, g);
    copy2d_f64(c, psi, mr, Mt, ldm, n, mr);
    return ldm;
  }
  GemmArgs g{r, n, ng, Ft, ng, true, 0, Zc, n, false, 0, Mt + (long)ml * n, n, 0, alpha, 0.0, 1};
  gemm_f64(c, g);
  copy_f64(c, psi, Mt, (long)ml * n);
  return (long)ml + r;
}

// ---------------------------------------------------------------- energy
double op_energy(Ctx* c, int ml, int d, int mr, int wl, int wr, const double* L, const double* W,
                 const double* R, const double* psi) {
  const long n = (long)ml * d * mr;
  double* hp = (double*)ws_get(c, WS_REF, sizeof(double) * n);
  op_apply_heff(c, D3S_F64, ml, d, mr, wl, wr, L, W, R, psi, hp);
  double* r = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 512);
  dot_f64(c, psi, hp, n, r);
  dot_f64(c, psi, psi, n, r + 1);
  double h[2];
  read_many(c, h, r, 2);
  if (!(h[1] > 0.0)) throw Error{D3S_ENUMERIC, "energy: zero state"};
  const double e = h[0] / h[1];
  if (!std::isfinite(e)) throw Error{D3S_ENUMERIC, "energy: not finite"};
  return e;
}

// ---------------------------------------------------------------- adjoint
void op_heff_grad_W(Ctx* c, int ml, int d, int mr, int wl, int wr, const double* L, const double* R,
                    const double* psi, const double* ybar, double* Wbar) {
  double* T1 = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * wl * d * mr);
  double* U = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)ml * d * wr * mr);
  // T1[(a,w),(t,y)] = L psi (GEMM over the left MPS bond, as in H_eff)
  GemmArgs g1{ml * wl, d * mr, ml, L, ml, true, 0, psi, (long)d * mr, false, 0, T1, (long)d * mr, 0,
              1.0, 0.0, 1};
  gemm_f64(c, g1);
  // U[(a,s),(v,y)] = sum_b ybar[(a,s), b] R[b, (v,y)]
  GemmArgs g2{ml * d, wr * mr, mr, ybar, mr, true, 0, R, (long)wr * mr, false, 0, U, (long)wr * mr, 0,
              1.0, 0.0, 1};
  gemm_f64(c, g2);
  adjoint_reduce_f64(c, T1, U, Wbar, ml, d, mr, wl, wr);
}

// ---------------------------------------------------------------- Lanczos
namespace {
struct Matvec {
  Ctx* c;
  d3s_prec p;
  int ml, d, mr, wl, wr;
  const double *L, *W, *R;
  const void *Lc = nullptr, *Wc = nullptr, *Rc = nullptr;   // low-precision copies
  void* xin = nullptr;
  float* yout = nullptr;
  long n;
  BlockHeff* plan = nullptr;     // block-sparse products when set
  LowpTwin* tw = nullptr;        // their low-precision products run on the plan's padded twin
  bool use_graph = false;
  long nl_ = 0, nr_ = 0;         // elements of L and R when not dense (packed block environments)
  void prepare() {
    if (p == D3S_F64) return;
    const long nl = nl_ ? nl_ : (long)ml * wl * ml, nr = nr_ ? nr_ : (long)mr * wr * mr;
    const long nw = (long)wl * wr * d * d;
    float* Wf = (float*)ws_get(c, WS_CAST_W, 4 * nw);
    cast_f64_to_f32(c, W, Wf, nw);
    Wc = Wf;
    if (plan) {
      // L and R converted once into the twin's padded packed layouts
      tw = &ensure_lowp(c, *plan, p);
      const int kind = (p == D3S_F32) ? RL_F32 : RL_BF16;
      const size_t esz = (p == D3S_F32) ? 4 : 2;
      void* Lp = ws_get(c, WS_CAST_L, esz * (size_t)plan_nl(tw->h));
      void* Rp = ws_get(c, WS_CAST_R, esz * (size_t)plan_nr(tw->h));
      relayout_tiles(c, RL_F64, kind, L, Lp, tw->d_L, tw->nL);
      relayout_tiles(c, RL_F64, kind, R, Rp, tw->d_R, tw->nR);
      Lc = Lp;
      Rc = Rp;
      xin = ws_get(c, WS_CAST_X, esz * (size_t)tw->h.npacked);
      yout = (float*)ws_get(c, WS_CAST_Y, 4 * (size_t)tw->h.npacked);
      return;
    }
    if (p == D3S_F32) {
      float* Lf = (float*)ws_get(c, WS_CAST_L, 4 * nl);
      float* Rf = (float*)ws_get(c, WS_CAST_R, 4 * nr);
      cast_f64_to_f32(c, L, Lf, nl);
      cast_f64_to_f32(c, R, Rf, nr);
      Lc = Lf;
      Rc = Rf;
      xin = ws_get(c, WS_CAST_X, 4 * n);
    } else {
      bf16_t* Lb = (bf16_t*)ws_get(c, WS_CAST_L, 2 * nl);
      bf16_t* Rb = (bf16_t*)ws_get(c, WS_CAST_R, 2 * nr);
      cast_f64_to_bf16(c, L, Lb, nl);
      cast_f64_to_bf16(c, R, Rb, nr);
      Lc = Lb;
      Rc = Rb;
      xin = ws_get(c, WS_CAST_X, 2 * n);
    }
    yout = (float*)ws_get(c, WS_CAST_Y, 4 * n);
  }
  // y = H x without any per-product graph (the caller may be capturing):
  // FP64, or the low-precision product with casts around it
  void product(const double* x, double* y, bool f64) {
    if (f64 || p == D3S_F64) {
      if (plan) op_apply_heff_blocks(c, *plan, D3S_F64, L, W, R, x, y, false);
      else op_apply_heff(c, D3S_F64, ml, d, mr, wl, wr, L, W, R, x, y);
      return;
    }
    if (tw) {
      lowp_product(c, *plan, *tw, p, Lc, Wc, Rc, x, y, xin, yout, false);
      return;
    }
    if (p == D3S_F32) cast_f64_to_f32(c, x, (float*)xin, n);
    else cast_f64_to_bf16(c, x, (bf16_t*)xin, n);
    op_apply_heff(c, p, ml, d, mr, wl, wr, Lc, Wc, Rc, xin, yout);
    cast_f32_to_f64(c, yout, y, n);
  }
};

// One Lanczos run (with restarts) on the operator `mv`, starting from x
// (normalised in place, overwritten by the Ritz vector).
//
// A step runs entirely on the device and reads its index k from device
// memory: V_k is copied to a fixed input buffer, multiplied, orthogonalised
// twice (classical Gram-Schmidt) against V_0..V_k, normalised into V_{k+1},
// (alpha_k, beta_k) are stored and k is incremented.  Because nothing in it
// depends on the host, the same step serves every k: with mv.use_graph it
// is captured once into a hipGraph (after a first eager step has sized
// every buffer) and replayed per step.  The host copies (alpha_k, beta_k)
// to pinned memory, enqueues step k+1 before it reads step k and solves the
// tridiagonal problem, so the device does not idle while the host tests
// convergence; a step enqueued past convergence is discarded (the Ritz
// vector uses V_0..V_k only).
LanczosResult lanczos_core(Ctx* c, Matvec& mv, double* x, long n, double tol, int kmax, int max_mv,
                           bool use_f64) {
  const int kk = (int)std::min<long>(kmax, n);
  if (kk > 64) throw Error{D3S_EINVAL, "lanczos: at most 64 Krylov vectors"};
  double* V = (double*)ws_get(c, WS_LZ_V, sizeof(double) * (size_t)(kk + 1) * n);
  double* w = (double*)ws_get(c, WS_LZ_W, sizeof(double) * n);
  double* xin = (double*)ws_get(c, WS_BLK_X, sizeof(double) * n);
  double* cf = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 1024);
  int* kdev = (int*)ws_get(c, WS_LZ_K, 256);
  double* cf1 = cf;          // first Gram-Schmidt coefficients
  double* cf2 = cf + 128;    // second pass
  double* sc = cf + 256;     // scalars
  double* ydev = cf + 384;   // Ritz coefficients
  double* ab = cf + 512;     // (alpha_k, beta_k) per step
  double* hab = c->host_red + 256;   // pinned host copy of ab
  LanczosResult res{0.0, 0, false, 0};
  if (!c->lz_ev[0]) {
    D3S_HIP(hipEventCreateWithFlags((hipEvent_t*)&c->lz_ev[0], hipEventDisableTiming));
    D3S_HIP(hipEventCreateWithFlags((hipEvent_t*)&c->lz_ev[1], hipEventDisableTiming));
  }
  // normalise the start vector (a zero one has no direction: start from the
  // constant vector; a non-finite one is an error)
  dot_f64(c, x, x, n, sc);
  double nrm2 = read_scalar(c, sc);
  if (!std::isfinite(nrm2)) throw Error{D3S_ENUMERIC, "lanczos: the start vector is not finite"};
  if (!(nrm2 > 0.0)) {
    fill_f64(c, x, n, 1.0);
    nrm2 = (double)n;
  }
  scale_f64(c, x, n, 1.0 / std::sqrt(nrm2));
  copy_f64(c, x, V, n);
  double* npart = (double*)ws_get(c, WS_GS_NORM, sizeof(double) * kGsMaxBlocks);
  auto body = [&]() {
    copy_row_f64(c, V, n, kdev, xin);
    mv.product(xin, w, use_f64);
    // classical Gram-Schmidt twice against V_0..V_k, three passes over V:
    // c1 = V^T w;  w -= V c1 with c2 = V^T w;  w -= V c2 with |w|^2
    mdot_f64(c, V, n, kk, w, n, cf1, kdev);
    gs_second_pass(c, V, n, kk, kdev, cf1, w, n, cf2);
    gs_update_norm(c, V, n, kk, kdev, cf2, w, n, npart);
    lanczos_tail(c, w, n, npart, cf1, cf2, 0, kdev, kk, V, ab);
    set_int_dev(c, kdev, 1, true);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;
  const bool want_graph = mv.use_graph && !c->prof;
  auto cleanup = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    gexec = nullptr;
    graph = nullptr;
    cap = nullptr;
  };
  auto enqueue_step = [&](int k) {
    if (gexec) {
      D3S_HIP(hipGraphLaunch(gexec, c->stream));
    } else {
      body();
      if (want_graph) {
        // every buffer is sized now: capture the step on a private stream
        hipStream_t keep = c->stream;
        D3S_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        c->stream = cap;
        D3S_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
          body();
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cap, &g);
          if (g) (void)hipGraphDestroy(g);
          c->stream = keep;
          throw;
        }
        c->stream = keep;
        D3S_HIP(hipStreamEndCapture(cap, &graph));
        D3S_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      }
    }
    D3S_HIP(hipMemcpyAsync(hab + 2 * k, ab + 2 * k, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    D3S_HIP(hipEventRecord((hipEvent_t)c->lz_ev[k & 1], c->stream));
    res.matvecs++;
  };
  std::vector<double> alphas, betas, T, ev, evec;
  try {
    for (;;) {
      alphas.clear();
      betas.clear();
      bool stop = false;
      std::vector<double> y;
      set_int_dev(c, kdev, 0, false);
      enqueue_step(0);
      int enq = 1;
      for (int k = 0; k < kk; ++k) {
        if (enq == k + 1 && k + 1 < kk && res.matvecs < max_mv) {
          enqueue_step(k + 1);
          ++enq;
        }
        D3S_HIP(hipEventSynchronize((hipEvent_t)c->lz_ev[k & 1]));
        const double a = hab[2 * k];
        const double b = hab[2 * k + 1];
        if (!std::isfinite(a) || !std::isfinite(b)) throw Error{D3S_ENUMERIC, "lanczos: non-finite value"};
        alphas.push_back(a);
        const int m = k + 1;
        y.assign(m, 0.0);
        if (!tridiag_lowest(m, alphas.data(), betas.data(), &res.theta, y.data())) {
          T.assign((size_t)m * m, 0.0);
          for (int i = 0; i < m; ++i) T[(size_t)i * m + i] = alphas[i];
          for (int i = 0; i + 1 < m; ++i) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = betas[i];
          jacobi_eigh(m, T, ev, evec);
          res.theta = ev[0];
          y.assign(evec.begin(), evec.begin() + m);
        }
        const double scale = std::max(1.0, std::fabs(res.theta));
        const double resid = std::fabs(b * y[m - 1]);
        if (resid <= tol * scale || b <= 1e-15 * scale || m == n) {
          res.converged = true;
          stop = true;
          break;
        }
        if (enq == k + 1 && res.matvecs >= max_mv) {
          stop = true;
          break;
        }
        betas.push_back(b);
      }
      const int m = (int)y.size();
      // Ritz vector x = sum_j y_j V_j (stream-ordered after any step still in flight)
      write_many(c, ydev, y.data(), m);
      fill_f64(c, x, n, 0.0);
      maxpy_f64(c, V, n, m, ydev, 1.0, x, n);
      dot_f64(c, x, x, n, sc);
      const double xn = read_scalar(c, sc);
      scale_f64(c, x, n, 1.0 / std::sqrt(xn));
      if (stop) break;
      res.restarts++;
      copy_f64(c, x, V, n);
    }
  } catch (...) {
    (void)hipStreamSynchronize(c->stream);
    cleanup();
    throw;
  }
  D3S_HIP(hipStreamSynchronize(c->stream));
  cleanup();
  if (use_f64) res.f64_matvecs = res.matvecs;
  return res;
}
}  // namespace

static LanczosResult lanczos_with(Ctx* c, Matvec& mv, d3s_prec p, double* psi, long n, double tol, int kmax,
                                  int max_matvecs);

LanczosResult op_lanczos_blocks(Ctx* c, d3s_prec p, BlockHeff& plan, const double* L, const double* W,
                                const double* R, double* psi, double tol, int kmax, int max_matvecs,
                                bool use_graph, double* packed_out) {
  const long n = plan.packed ? plan.npacked : (long)plan.ml * plan.d * plan.mr;
  if (n <= 0) throw Error{D3S_EINVAL, "lanczos: the site has no symmetry-allowed block"};
  Matvec mv{c, p, plan.ml, plan.d, plan.mr, plan.wl, plan.wr, L, W, R};
  mv.n = n;
  mv.plan = &plan;
  mv.use_graph = use_graph;
  mv.nl_ = plan_nl(plan);
  mv.nr_ = plan_nr(plan);
  mv.prepare();
  if (!plan.packed) return lanczos_with(c, mv, p, psi, n, tol, kmax, max_matvecs);
  double* x = packed_out ? packed_out : (double*)ws_get(c, WS_PK, sizeof(double) * (size_t)n);
  pack_psi(c, plan, psi, x);
  LanczosResult r = lanczos_with(c, mv, p, x, n, tol, kmax, max_matvecs);
  unpack_psi(c, plan, x, psi, plan.mr, true);
  return r;
}

LanczosResult op_lanczos(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const double* L,
                         const double* W, const double* R, double* psi, double tol, int kmax,
                         int max_matvecs) {
  const long n = (long)ml * d * mr;
  Matvec mv{c, p, ml, d, mr, wl, wr, L, W, R};
  mv.n = n;
  mv.prepare();
  return lanczos_with(c, mv, p, psi, n, tol, kmax, max_matvecs);
}

// FP64 iterative refinement of a Ritz pair with low-precision inner solves
// (the mixed-precision eigensolver's second phase).
//
// An FP64 search space V (orthonormal) with W = H V (FP64 products) is
// grown one vector per outer step.  The lowest Ritz pair (theta, u = V s)
// of V^T W gives the exact FP64 residual r = W s - theta u without another
// product.  The new direction t approximately solves the projected
// correction equation (I - u u^T)(H - theta)(I - u u^T) t = -r, t _|_ u
// (Jacobi-Davidson), by conjugate gradients whose products are the
// low-precision ones (the projected operator is positive definite on u's
// complement once theta is below the second eigenvalue); the FP64 outer
// step then removes the error the low-precision products leave.  So nearly
// all products run in low precision and each outer step costs one FP64
// product.  The space restarts from u after kJdMax vectors.
namespace {
constexpr int kJdMax = 12;

LanczosResult jd_refine(Ctx* c, Matvec& mv, double* x, long n, double tol, int max_mv, int n_inner,
                        double eta) {
  LanczosResult res{0.0, 0, false, 0};
  double* V = (double*)ws_get(c, WS_JD_V, sizeof(double) * (size_t)(kJdMax + 1) * n);
  double* Wm = (double*)ws_get(c, WS_JD_W, sizeof(double) * (size_t)(kJdMax + 1) * n);
  // work vectors, contiguous rows: u, p, rs (CG residual), q, t, r
  double* Z = (double*)ws_get(c, WS_JD_Z, sizeof(double) * (size_t)6 * n);
  double* u = Z;
  double* pv = Z + n;
  double* rs = Z + 2 * n;
  double* q = Z + 3 * n;
  double* t = Z + 4 * n;
  double* r = Z + 5 * n;
  double* cf = (double*)ws_get(c, WS_JD_COEF, sizeof(double) * 256);
  double h[8];
  auto dots = [&](const double* rows, int k, const double* v, double* out_host) {
    mdot_f64(c, rows, n, k, v, n, cf);
    D3S_HIP(hipMemcpyAsync(out_host, cf, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    D3S_HIP(hipStreamSynchronize(c->stream));
  };
  // start: V = [x / |x|], W = [H x]
  dots(x, 1, x, h);
  if (!(h[0] > 0.0) || !std::isfinite(h[0])) throw Error{D3S_ENUMERIC, "refinement: zero start vector"};
  axpby_f64(c, 1.0 / std::sqrt(h[0]), x, 0.0, V, n);
  mv.product(V, Wm, true);
  res.matvecs++;
  res.f64_matvecs++;
  int k = 1;
  std::vector<double> S((size_t)kJdMax * kJdMax, 0.0);
  dots(V, 1, Wm, h);
  S[0] = h[0];
  std::vector<double> A, ev, evec, sv;
  for (;;) {
    // lowest Ritz pair of S = V^T W (symmetric, k x k)
    A.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = 0.5 * (S[(size_t)i * kJdMax + j] + S[(size_t)j * kJdMax + i]);
    jacobi_eigh(k, A, ev, evec);
    const double th = ev[0];
    sv.assign(evec.begin(), evec.begin() + k);
    res.theta = th;
    // u = V s, r = W s - th u, |r|
    write_many(c, cf + 128, sv.data(), k);
    fill_f64(c, u, n, 0.0);
    maxpy_f64(c, V, n, k, cf + 128, 1.0, u, n);
    fill_f64(c, r, n, 0.0);
    maxpy_f64(c, Wm, n, k, cf + 128, 1.0, r, n);
    axpby_f64(c, -th, u, 1.0, r, n);
    dots(r, 1, r, h);
    const double rn = std::sqrt(std::max(h[0], 0.0));
    const double scale = std::max(1.0, std::fabs(th));
    if (!std::isfinite(rn)) throw Error{D3S_ENUMERIC, "refinement: non-finite residual"};
    if (rn <= tol * scale) {
      res.converged = true;
      break;
    }
    if (res.matvecs >= max_mv) break;
    // restart the search space from u, with W_0 = H u = r + th u
    if (k >= kJdMax) {
      copy_f64(c, u, V, n);
      axpby_f64(c, 1.0, r, 0.0, Wm, n);
      axpby_f64(c, th, u, 1.0, Wm, n);
      k = 1;
      S.assign((size_t)kJdMax * kJdMax, 0.0);
      S[0] = th;
      res.restarts++;
    }
    // CG on the projected correction equation; t = 0, rs = -r (_|_ u), p = rs
    fill_f64(c, t, n, 0.0);
    axpby_f64(c, -1.0, r, 0.0, rs, n);
    copy_f64(c, rs, pv, n);
    double rr = h[0];
    for (int it = 0; it < n_inner && res.matvecs < max_mv; ++it) {
      mv.product(pv, q, false);
      res.matvecs++;
      axpby_f64(c, -th, pv, 1.0, q, n);                 // q = (H - th) p
      dots(u, 2, q, h);                                 // h0 = u.q, h1 = p.q
      axpby_f64(c, -h[0], u, 1.0, q, n);                // q -= u (u.q); p.q is unchanged as p _|_ u
      const double pq = h[1];
      if (!(pq > 0.0) || !std::isfinite(pq)) break;     // not positive definite here: keep t
      const double al = rr / pq;
      axpby_f64(c, al, pv, 1.0, t, n);
      axpby_f64(c, -al, q, 1.0, rs, n);
      dots(rs, 1, rs, h + 2);
      const double rr_new = h[2];
      if (std::sqrt(std::max(rr_new, 0.0)) <= eta * rn) break;
      axpby_f64(c, 1.0, rs, rr_new / rr, pv, n);        // p = rs + beta p
      dots(u, 1, pv, h + 3);
      axpby_f64(c, -h[3], u, 1.0, pv, n);               // keep p _|_ u
      rr = rr_new;
    }
    // first step broke down: fall back to the residual direction
    dots(t, 1, t, h);
    if (!(h[0] > 0.0)) axpby_f64(c, -1.0, r, 0.0, t, n);
    // orthonormalise t against V (twice) and extend V, W
    for (int pass = 0; pass < 2; ++pass) {
      mdot_f64(c, V, n, k, t, n, cf);
      maxpy_f64(c, V, n, k, cf, -1.0, t, n);
    }
    dots(t, 1, t, h);
    if (!(h[0] > 1e-28)) break;                           // nothing new: as converged as it gets
    double* vk = V + (long)k * n;
    double* wk = Wm + (long)k * n;
    axpby_f64(c, 1.0 / std::sqrt(h[0]), t, 0.0, vk, n);
    mv.product(vk, wk, true);
    res.matvecs++;
    res.f64_matvecs++;
    std::vector<double> col(k + 1);
    dots(V, k + 1, wk, col.data());
    for (int i = 0; i <= k; ++i) {
      S[(size_t)i * kJdMax + k] = col[i];
      S[(size_t)k * kJdMax + i] = col[i];
    }
    ++k;
  }
  // x = u (normalised)
  copy_f64(c, u, x, n);
  return res;
}
}  // namespace

static LanczosResult lanczos_with(Ctx* c, Matvec& mv, d3s_prec p, double* psi, long n, double tol, int kmax,
                                  int max_matvecs) {
  if (p == D3S_F64) return lanczos_core(c, mv, psi, n, tol, kmax, max_matvecs, true);
  // Mixed precision (products in FP32 / BF16; Krylov and search vectors,
  // orthogonalisation and the small eigenproblems in FP64):
  // 1. Lanczos on the low-precision operator down to what it resolves;
  // 2. FP64 iterative refinement of that Ritz vector (jd_refine) to the
  //    caller's tolerance on the exact FP64 residual.  The Ritz value is an
  //    FP64 Rayleigh quotient, whose error is quadratic in the residual.
  const double low_tol = (c->refine_low_tol > 0.0) ? c->refine_low_tol : (p == D3S_F32) ? 1e-6 : 3e-3;
  LanczosResult r1 = lanczos_core(c, mv, psi, n, std::max(tol, low_tol), kmax, max_matvecs, false);
  if (n <= 2 * kJdMax) {
    LanczosResult r2 = lanczos_core(c, mv, psi, n, tol, kmax, std::max(1, max_matvecs - r1.matvecs), true);
    r2.matvecs += r1.matvecs;
    r2.restarts += r1.restarts;
    return r2;
  }
  LanczosResult r2 = jd_refine(c, mv, psi, n, tol, std::max(2, max_matvecs - r1.matvecs), c->refine_inner,
                               c->refine_eta);
  r2.matvecs += r1.matvecs;
  r2.restarts += r1.restarts;
  return r2;
}

}  // namespace d3s
