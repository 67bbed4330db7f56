// The C-ABI of libdmrg3s: argument checks before any launch, then the
// operations of ops.hip / sweep.hip.  No exception crosses this boundary.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "d3s_internal.h"

struct d3s_ctx_s {
  d3s::Ctx c;
};

struct d3s_block_plan_s {
  d3s::BlockHeff h;
  d3s::Sectors left, right;
};

namespace {

using d3s::Error;

template <typename F>
d3s_status guarded(d3s_ctx ctx, F&& body) {
  if (!ctx) return D3S_EINVAL;
  try {
    ctx->c.last_error.clear();
    if (hipSetDevice(ctx->c.device) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{D3S_EDEVICE, "hipSetDevice failed"};
    }
    return body();
  } catch (const Error& e) {
    ctx->c.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->c.last_error = "host allocation failed";
    return D3S_ENOMEM;
  } catch (...) {
    ctx->c.last_error = "unexpected exception";
    return D3S_EDEVICE;
  }
}

void check_dims(int ml, int d, int mr, int wl, int wr) {
  D3S_REQUIRE(ml >= 1 && d >= 1 && mr >= 1 && wl >= 1 && wr >= 1, "dimensions must be >= 1");
  D3S_REQUIRE((long)wl * d <= 80 && (long)wr * d <= 80, "w * d must be <= 80");
  D3S_REQUIRE((long)ml * wl * d * mr < (1L << 40), "tensor too large");
  D3S_REQUIRE((long)ml * wl <= 0x7fffffffL && (long)wr * mr <= 0x7fffffffL && (long)d * mr <= 0x7fffffffL,
              "GEMM extent exceeds 2^31");
}

void check_prec(d3s_prec p) {
  D3S_REQUIRE(p == D3S_F64 || p == D3S_F32 || p == D3S_BF16, "invalid precision");
}

void check_dir(d3s_dir dir) { D3S_REQUIRE(dir == D3S_L2R || dir == D3S_R2L, "invalid direction"); }

}  // namespace

extern "C" {

const char* d3s_version(void) { return "dmrg3s-mi355x 0.1 (gfx950)"; }

d3s_status d3s_create(d3s_ctx* out, int device, void* stream, const d3s_allocator* alloc) {
  if (!out) return D3S_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return D3S_EINVAL;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) return D3S_EINVAL;
  d3s_ctx ctx = new (std::nothrow) d3s_ctx_s();
  if (!ctx) return D3S_ENOMEM;
  ctx->c.device = device;
  ctx->c.stream = (hipStream_t)stream;
  if (alloc) {
    ctx->c.alloc = *alloc;
    ctx->c.has_alloc = true;
  }
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&ctx->c.host_red, 512 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return D3S_EDEVICE;
  }
  try {
    d3s::noalloc_init(device);   // the device address of this GPU's scratch array
  } catch (...) {
    (void)hipHostFree(ctx->c.host_red);
    delete ctx;
    return D3S_EDEVICE;
  }
  *out = ctx;
  return D3S_OK;
}

void d3s_destroy(d3s_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  (void)hipStreamSynchronize(ctx->c.stream);
  for (hipEvent_t e : ctx->c.prof_ev) (void)hipEventDestroy(e);
  d3s::eig_pool_destroy(&ctx->c);
  d3s::ws_release_all(&ctx->c);
  if (ctx->c.solver) rocblas_destroy_handle((rocblas_handle)ctx->c.solver);
  if (ctx->c.host_red) (void)hipHostFree(ctx->c.host_red);
  for (void* e : ctx->c.lz_ev)
    if (e) (void)hipEventDestroy((hipEvent_t)e);
  delete ctx;
}

const char* d3s_last_error(d3s_ctx ctx) { return ctx ? ctx->c.last_error.c_str() : "null context"; }

d3s_status d3s_set_stream(d3s_ctx ctx, void* stream) {
  return guarded(ctx, [&] {
    ctx->c.stream = (hipStream_t)stream;
    return D3S_OK;
  });
}

d3s_status d3s_synchronize(d3s_ctx ctx) {
  return guarded(ctx, [&] {
    D3S_HIP(hipStreamSynchronize(ctx->c.stream));
    return D3S_OK;
  });
}

d3s_status d3s_set_block_split(d3s_ctx ctx, double min_gflop) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(std::isfinite(min_gflop), "min_gflop must be finite");
    ctx->c.block_split_gflop = min_gflop;
    return D3S_OK;
  });
}

d3s_status d3s_set_grouped_tile(d3s_ctx ctx, int cfg) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(cfg >= -1 && cfg <= 5, "grouped tile configuration must be in [-1, 5]");
    ctx->c.grouped_cfg = cfg;
    return D3S_OK;
  });
}

d3s_status d3s_set_tile_config(d3s_ctx ctx, int cfg) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(cfg >= -1 && cfg <= 4, "tile config must be in [-1, 4]");
    ctx->c.tile_config = cfg;
    return D3S_OK;
  });
}

d3s_status d3s_set_autotune(d3s_ctx ctx, int enable, const char* cache_path) {
  return guarded(ctx, [&] {
    ctx->c.autotune = (enable != 0);
    ctx->c.tune_path = cache_path ? std::string(cache_path) : std::string();
    d3s::autotune_load(&ctx->c);
    return D3S_OK;
  });
}

d3s_status d3s_tridiag_lowest(int n, const double* alpha, const double* beta, double* theta, double* y) {
  if (n < 1 || !alpha || !theta || !y || (n > 1 && !beta)) return D3S_EINVAL;
  try {
    return d3s::tridiag_lowest(n, alpha, beta, theta, y) ? D3S_OK : D3S_ENUMERIC;
  } catch (...) {
    return D3S_ENOMEM;
  }
}

d3s_status d3s_eig_batched(d3s_ctx ctx, int n, int batch, double* A, double* W) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(n >= 1 && batch >= 1, "n and batch must be >= 1");
    D3S_REQUIRE(A && W, "null pointer");
    // one batch of equal size through the normalised solve of the truncations
    d3s::EigPlan ep;
    std::vector<int> ns(batch, n);
    ep.npad.assign(batch, n);
    ep.goff.resize(batch);
    ep.voff.resize(batch);
    ep.members.emplace_back();
    for (int b = 0; b < batch; ++b) {
      ep.goff[b] = (long)b * n * n;
      ep.voff[b] = (long)b * n;
      ep.members[0].push_back(b);
    }
    ep.bucket_n = {n};
    ep.bucket_goff = {0};
    ep.bucket_voff = {0};
    ep.gtot = (long)batch * n * n;
    ep.vtot = (long)batch * n;
    std::vector<double> scale;
    d3s::eig_run(&ctx->c, ep, ns, A, W, scale);
    for (int b = 0; b < batch; ++b)
      if (scale[b] != 1.0) d3s::scale_f64(&ctx->c, W + (long)b * n, n, scale[b]);
    D3S_HIP(hipStreamSynchronize(ctx->c.stream));
    return D3S_OK;
  });
}

d3s_status d3s_set_eigensolver(d3s_ctx ctx, int kind, int jacobi_max_n) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(kind >= 0 && kind <= 3,
                "kind must be 0 (auto), 1 (divide and conquer), 2 (Jacobi) or 3 (LDS solver up to n = 128)");
    D3S_REQUIRE(jacobi_max_n >= 0, "jacobi_max_n must be >= 0");
    ctx->c.eig_kind = kind;
    ctx->c.eig_jacobi_max = jacobi_max_n;
    return D3S_OK;
  });
}

d3s_status d3s_set_eig_workers(d3s_ctx ctx, int workers) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(workers >= 1 && workers <= 8, "workers must be 1 to 8");
    ctx->c.eig_workers = workers;
    return D3S_OK;
  });
}

d3s_status d3s_set_refinement(d3s_ctx ctx, double eta, int inner_max, double low_tol) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(eta > 0.0 && eta < 1.0, "eta must lie in (0, 1)");
    D3S_REQUIRE(inner_max >= 1 && inner_max <= 1000, "inner_max must be 1 to 1000");
    D3S_REQUIRE(std::isfinite(low_tol) && low_tol < 1.0, "low_tol must be below 1");
    ctx->c.refine_eta = eta;
    ctx->c.refine_inner = inner_max;
    ctx->c.refine_low_tol = low_tol;
    return D3S_OK;
  });
}

d3s_status d3s_set_splitk(d3s_ctx ctx, int enable) {
  return guarded(ctx, [&] {
    ctx->c.splitk_off = (enable == 0);
    return D3S_OK;
  });
}

d3s_status d3s_profile_begin(d3s_ctx ctx, int capacity) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(capacity >= 1 && capacity <= 100000, "capacity must be in [1, 100000]");
    while ((int)ctx->c.prof_ev.size() < 4 * capacity) {
      hipEvent_t e;
      D3S_HIP(hipEventCreate(&e));
      ctx->c.prof_ev.push_back(e);
    }
    ctx->c.prof_cap = capacity;
    ctx->c.prof_n = 0;
    ctx->c.prof = true;
    return D3S_OK;
  });
}

d3s_status d3s_profile_end(d3s_ctx ctx, double* total_ms, int* count) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(total_ms && count, "null output");
    D3S_HIP(hipStreamSynchronize(ctx->c.stream));
    total_ms[0] = total_ms[1] = total_ms[2] = 0.0;
    for (int i = 0; i < ctx->c.prof_n; ++i) {
      for (int k = 0; k < 3; ++k) {
        float ms = 0.f;
        D3S_HIP(hipEventElapsedTime(&ms, ctx->c.prof_ev[4 * i + k], ctx->c.prof_ev[4 * i + k + 1]));
        total_ms[k] += ms;
      }
    }
    *count = ctx->c.prof_n;
    ctx->c.prof = false;
    ctx->c.prof_n = 0;
    return D3S_OK;
  });
}

d3s_status d3s_apply_heff(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr, const void* L,
                          const void* W, const void* R, const void* psi, void* out) {
  return guarded(ctx, [&] {
    check_prec(prec);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(L && W && R && psi && out, "null tensor pointer");
    D3S_REQUIRE(out != psi && out != L && out != R, "out must not alias an input");
    d3s::op_apply_heff(&ctx->c, prec, ml, d, mr, wl, wr, L, W, R, psi, out);
    return D3S_OK;
  });
}

d3s_status d3s_apply_heff_noalloc(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr,
                                  const void* L, const void* W, const void* R, const void* psi, void* out) {
  return guarded(ctx, [&] {
    check_prec(prec);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(L && W && R && psi && out, "null tensor pointer");
    D3S_REQUIRE(out != psi && out != L && out != R, "out must not alias an input");
    d3s::op_apply_heff_noalloc(&ctx->c, prec, ml, d, mr, wl, wr, L, W, R, psi, out);
    return D3S_OK;
  });
}

d3s_status d3s_expand_subspace(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                               const double* env, const double* W, const double* psi, double alpha,
                               double* Mtilde) {
  return guarded(ctx, [&] {
    check_dir(dir);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(env && W && psi && Mtilde, "null tensor pointer");
    D3S_REQUIRE(std::isfinite(alpha), "alpha must be finite");
    d3s::op_expand(&ctx->c, dir, ml, d, mr, wl, wr, env, W, psi, alpha, Mtilde);
    return D3S_OK;
  });
}

d3s_status d3s_truncate(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, long width, const double* Mtilde,
                        const double* psi, int kmax, double rel_cutoff, const double* nbr_in, long nbr_other,
                        double* site_out, double* nbr_out, int renormalize, double* s_host, int* k_out,
                        double* discarded) {
  return guarded(ctx, [&] {
    check_dir(dir);
    D3S_REQUIRE(ml >= 1 && d >= 1 && mr >= 1 && width >= 1 && nbr_other >= 1 && kmax >= 1,
                "dimensions must be >= 1");
    D3S_REQUIRE(Mtilde && psi && site_out && nbr_out && k_out && discarded, "null pointer");
    if (!nbr_in)
      D3S_REQUIRE(nbr_other == (dir == D3S_L2R ? mr : ml),
                  "without a neighbour, nbr_other must be m_r (L2R) or m_l (R2L)");
    D3S_REQUIRE(rel_cutoff >= 0.0, "rel_cutoff must be >= 0");
    const long n = (dir == D3S_L2R) ? (long)ml * d : (long)d * mr;
    D3S_REQUIRE(n <= 46340, "Gram dimension too large (n^2 must fit in int)");
    if (dir == D3S_L2R) D3S_REQUIRE(width >= mr, "L2R: width must be >= m_r (psi occupies the first m_r columns)");
    else D3S_REQUIRE(width >= ml, "R2L: width must be >= m_l (psi occupies the first m_l rows)");
    D3S_REQUIRE(width <= 0x7fffffffL, "width too large");
    d3s::TruncResult t = d3s::op_truncate(&ctx->c, dir, ml, d, mr, width, Mtilde, psi, kmax, rel_cutoff, nbr_in,
                                          nbr_other, site_out, nbr_out, s_host, renormalize != 0);
    D3S_HIP(hipStreamSynchronize(ctx->c.stream));
    *k_out = t.k;
    *discarded = t.discarded;
    return D3S_OK;
  });
}

d3s_status d3s_update_env_h2(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr,
                             const double* env_in, const double* W, const double* site, double* env_out) {
  return guarded(ctx, [&] {
    check_dir(dir);
    D3S_REQUIRE(ml >= 1 && d >= 1 && mr >= 1 && wl >= 1 && wr >= 1, "dimensions must be >= 1");
    D3S_REQUIRE(wl <= 64 && wr <= 64 && d <= 64, "H^2 environment: w and d must be <= 64");
    D3S_REQUIRE((long)ml * wl * wl * d * mr < (1L << 36) && (long)ml * wr * wr * d * mr < (1L << 36),
                "H^2 environment: tensors too large");
    D3S_REQUIRE(env_in && W && site && env_out, "null tensor pointer");
    d3s::op_update_env_h2(&ctx->c, dir, ml, d, mr, wl, wr, env_in, W, site, env_out);
    return D3S_OK;
  });
}

d3s_status d3s_residual_gram(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                             const double* R, const double* h2, const double* W, const double* psi, double energy,
                             double alpha, double* gram) {
  return guarded(ctx, [&] {
    check_dir(dir);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(wl <= 64 && wr <= 64, "residual: w must be <= 64");
    D3S_REQUIRE(std::isfinite(energy) && std::isfinite(alpha), "energy and alpha must be finite");
    const long n = (dir == D3S_L2R) ? (long)ml * d : (long)d * mr;
    const long ng = (dir == D3S_L2R) ? (long)(1 + wr) * mr : (long)(1 + wl) * ml;
    D3S_REQUIRE(n <= 46340 && ng <= 46340, "residual: Gram or metric dimension too large");
    D3S_REQUIRE(L && R && h2 && W && psi && gram, "null tensor pointer");
    d3s::op_residual_gram(&ctx->c, dir, ml, d, mr, wl, wr, L, R, h2, W, psi, energy, alpha, gram);
    return D3S_OK;
  });
}

d3s_status d3s_residual_expand(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* L,
                               const double* R, const double* h2, const double* W, const double* psi, double energy,
                               double alpha, double* Mtilde, long* extent) {
  return guarded(ctx, [&] {
    check_dir(dir);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(wl <= 64 && wr <= 64, "residual: w must be <= 64");
    D3S_REQUIRE(std::isfinite(energy) && std::isfinite(alpha), "energy and alpha must be finite");
    const long n = (dir == D3S_L2R) ? (long)ml * d : (long)d * mr;
    const long ng = (dir == D3S_L2R) ? (long)(1 + wr) * mr : (long)(1 + wl) * ml;
    D3S_REQUIRE(n <= 46340 && ng <= 46340, "residual: Gram or metric dimension too large");
    D3S_REQUIRE(L && R && h2 && W && psi && Mtilde && extent, "null pointer");
    *extent = d3s::op_residual_expand(&ctx->c, dir, ml, d, mr, wl, wr, L, R, h2, W, psi, energy, alpha, Mtilde);
    return D3S_OK;
  });
}

d3s_status d3s_update_env(d3s_ctx ctx, d3s_dir dir, int ml, int d, int mr, int wl, int wr, const double* env_in,
                          const double* W, const double* site, double* env_out) {
  return guarded(ctx, [&] {
    check_dir(dir);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(env_in && W && site && env_out, "null tensor pointer");
    D3S_REQUIRE(env_out != env_in && env_out != site, "env_out must not alias an input");
    d3s::op_update_env(&ctx->c, dir, ml, d, mr, wl, wr, env_in, W, site, env_out);
    return D3S_OK;
  });
}

d3s_status d3s_lanczos(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wr, const double* L,
                       const double* W, const double* R, double* psi, double tol, int kmax, int max_matvecs,
                       double* theta, int* matvecs) {
  return guarded(ctx, [&] {
    check_prec(prec);
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(L && W && R && psi && theta, "null pointer");
    D3S_REQUIRE(kmax >= 2 && kmax <= 64, "kmax must be in [2, 64]");
    D3S_REQUIRE(max_matvecs >= 1, "max_matvecs must be >= 1");
    D3S_REQUIRE(tol > 0.0, "tol must be > 0");
    d3s::LanczosResult r = d3s::op_lanczos(&ctx->c, prec, ml, d, mr, wl, wr, L, W, R, psi, tol, kmax, max_matvecs);
    *theta = r.theta;
    if (matvecs) *matvecs = r.matvecs;
    return r.converged ? D3S_OK : D3S_ENOCONV;
  });
}

d3s_status d3s_energy(d3s_ctx ctx, int ml, int d, int mr, int wl, int wr, const double* L, const double* W,
                      const double* R, const double* psi, double* energy) {
  return guarded(ctx, [&] {
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(L && W && R && psi && energy, "null pointer");
    *energy = d3s::op_energy(&ctx->c, ml, d, mr, wl, wr, L, W, R, psi);
    return D3S_OK;
  });
}

d3s_status d3s_heff_grad_W(d3s_ctx ctx, int ml, int d, int mr, int wl, int wr, const double* L, const double* R,
                           const double* psi, const double* ybar, double* Wbar) {
  return guarded(ctx, [&] {
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(L && R && psi && ybar && Wbar, "null pointer");
    d3s::op_heff_grad_W(&ctx->c, ml, d, mr, wl, wr, L, R, psi, ybar, Wbar);
    return D3S_OK;
  });
}

static void check_state(const d3s_state* s) {
  D3S_REQUIRE(s, "null state");
  D3S_REQUIRE(s->l >= 2 && s->d >= 1 && s->mmax >= 1, "state: need l >= 2, d >= 1, mmax >= 1");
  D3S_REQUIRE(s->m && s->w && s->site && s->mpo && s->lenv && s->renv, "state: null array");
  D3S_REQUIRE(s->m[0] == 1 && s->m[s->l] == 1 && s->w[0] == 1 && s->w[s->l] == 1,
              "state: boundary bonds must be 1");
  for (int i = 0; i < s->l; ++i) {
    D3S_REQUIRE(s->site[i] && s->mpo[i] && s->lenv[i] && s->renv[i], "state: null tensor pointer");
    D3S_REQUIRE(s->m[i] >= 1 && s->m[i] <= s->mmax, "state: bond dimension out of range");
    D3S_REQUIRE(s->w[i] >= 1 && (long)s->w[i] * s->d <= 80, "state: MPO bond out of range");
  }
}

d3s_status d3s_prepare(d3s_ctx ctx, d3s_state* state, double* energy) {
  return guarded(ctx, [&] {
    check_state(state);
    D3S_REQUIRE(energy, "null energy pointer");
    D3S_REQUIRE((long)state->d * state->mmax <= 46340, "d * mmax too large for the Gram route");
    *energy = d3s::op_prepare(&ctx->c, state, 1e-14);
    return D3S_OK;
  });
}

d3s_status d3s_sweep(d3s_ctx ctx, d3s_state* state, d3s_sweep_params* params, d3s_sweep_stats* stats) {
  return guarded(ctx, [&] {
    check_state(state);
    D3S_REQUIRE(params && stats, "null params or stats");
    D3S_REQUIRE(stats->records || stats->capacity == 0, "stats: null records with capacity > 0");
    check_prec(params->prec);
    D3S_REQUIRE(params->lanczos_kmax >= 2 && params->lanczos_kmax <= 64, "lanczos_kmax must be in [2, 64]");
    D3S_REQUIRE(params->lanczos_tol > 0.0 && params->lanczos_max_matvecs >= 1, "bad eigensolver limits");
    D3S_REQUIRE(params->alpha >= 0.0 && std::isfinite(params->alpha), "alpha must be finite and >= 0");
    D3S_REQUIRE(params->mixed_min_gflop >= 0.0, "mixed_min_gflop must be >= 0");
    D3S_REQUIRE(params->expansion == 0 || params->expansion == 1, "expansion must be 0 or 1");
    D3S_REQUIRE((long)state->d * state->mmax <= 46340, "d * mmax too large for the Gram route");
    d3s::op_sweep(&ctx->c, state, params, stats);
    if (!std::isfinite(stats->energy)) throw Error{D3S_ENUMERIC, "sweep: non-finite energy"};
    return stats->nonconverged ? D3S_ENOCONV : D3S_OK;
  });
}

d3s_status d3s_energy_gradients(d3s_ctx ctx, d3s_state* state, double** grads) {
  return guarded(ctx, [&] {
    check_state(state);
    D3S_REQUIRE(grads, "null gradient array");
    for (int i = 0; i < state->l; ++i) D3S_REQUIRE(grads[i], "null gradient pointer");
    D3S_REQUIRE((long)state->d * state->mmax <= 46340, "d * mmax too large for the Gram route");
    d3s::op_gradients(&ctx->c, state, grads);
    return D3S_OK;
  });
}

static void check_sectors(const d3s_sectors* s, int nq, const char* name) {
  D3S_REQUIRE(s && s->nsec >= 1 && s->q && s->dim, std::string(name) + ": null or empty sector list");
  long tot = 0;
  for (int i = 0; i < s->nsec; ++i) {
    D3S_REQUIRE(s->dim[i] >= 1, std::string(name) + ": sector dimensions must be >= 1");
    tot += s->dim[i];
  }
  D3S_REQUIRE(tot <= 1 << 20, std::string(name) + ": bond too large");
  d3s::Sectors tmp(nq, s->nsec, s->q, s->dim);
  D3S_REQUIRE((int)tmp.index.size() == s->nsec, std::string(name) + ": repeated charge");
}

d3s_status d3s_block_plan_create_layout(d3s_ctx ctx, int nq, int d, int wl, int wr, const d3s_sectors* left,
                                        const d3s_sectors* right, const int* phys_q, const int* wq_left,
                                        const int* wq_right, int layout, d3s_block_plan* plan, double* flops,
                                        int* ntasks) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan pointer");
    *plan = nullptr;
    D3S_REQUIRE(nq == 1 || nq == 2, "nq must be 1 or 2");
    D3S_REQUIRE(layout == D3S_LAYOUT_DENSE || layout == D3S_LAYOUT_PACKED, "layout must be dense or packed");
    D3S_REQUIRE(phys_q && wq_left && wq_right, "null charge array");
    check_sectors(left, nq, "left");
    check_sectors(right, nq, "right");
    d3s_block_plan p = new d3s_block_plan_s();
    p->left = d3s::Sectors(nq, left->nsec, left->q, left->dim);
    p->right = d3s::Sectors(nq, right->nsec, right->q, right->dim);
    try {
      check_dims(p->left.total, d, p->right.total, wl, wr);
      const bool packed = (layout == D3S_LAYOUT_PACKED);
      d3s::build_block_heff(&ctx->c, p->h, p->left, p->right, d, wl, wr, phys_q, wq_left, wq_right, packed, true,
                            packed);
    } catch (...) {
      d3s::release_block_heff(p->h);
      delete p;
      throw;
    }
    if (flops) *flops = p->h.flops;
    if (ntasks) *ntasks = p->h.g1.ntasks + p->h.g2.ntasks;
    *plan = p;
    return D3S_OK;
  });
}

d3s_status d3s_block_plan_create(d3s_ctx ctx, int nq, int d, int wl, int wr, const d3s_sectors* left,
                                 const d3s_sectors* right, const int* phys_q, const int* wq_left,
                                 const int* wq_right, d3s_block_plan* plan, double* flops, int* ntasks) {
  return d3s_block_plan_create_layout(ctx, nq, d, wl, wr, left, right, phys_q, wq_left, wq_right, D3S_LAYOUT_DENSE,
                                      plan, flops, ntasks);
}

d3s_status d3s_block_plan_sizes(d3s_block_plan plan, long* nl, long* nr, long* npsi) {
  if (!plan || !nl || !nr || !npsi) return D3S_EINVAL;
  *nl = d3s::plan_nl(plan->h);
  *nr = d3s::plan_nr(plan->h);
  *npsi = plan->h.packed ? plan->h.npacked : (long)plan->h.ml * plan->h.d * plan->h.mr;
  return D3S_OK;
}

void d3s_block_plan_destroy(d3s_ctx ctx, d3s_block_plan plan) {
  if (!plan) return;
  if (ctx) (void)hipSetDevice(ctx->c.device);
  d3s::release_block_heff(plan->h);
  delete plan;
}

d3s_status d3s_apply_heff_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_prec prec, const void* L, const void* W,
                                 const void* R, const void* psi, void* out, int use_graph) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    check_prec(prec);
    D3S_REQUIRE(L && W && R && psi && out, "null tensor pointer");
    D3S_REQUIRE(out != psi && out != L && out != R, "out must not alias an input");
    d3s::op_apply_heff_blocks(&ctx->c, plan->h, prec, L, W, R, psi, out, use_graph != 0);
    return D3S_OK;
  });
}

d3s_status d3s_block_plan_bind(d3s_ctx ctx, d3s_block_plan plan, d3s_prec prec, const double* L, const double* W,
                               const double* R) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    D3S_REQUIRE(prec == D3S_F32 || prec == D3S_BF16, "bind: prec must be D3S_F32 or D3S_BF16");
    D3S_REQUIRE(L && W && R, "null tensor pointer");
    d3s::op_block_bind(&ctx->c, plan->h, prec, L, W, R);
    return D3S_OK;
  });
}

d3s_status d3s_apply_heff_blocks_bound(d3s_ctx ctx, d3s_block_plan plan, const double* psi, double* out,
                                       int use_graph) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    D3S_REQUIRE(psi && out, "null tensor pointer");
    D3S_REQUIRE(out != psi, "out must not alias psi");
    d3s::op_apply_heff_blocks_bound(&ctx->c, plan->h, psi, out, use_graph != 0);
    return D3S_OK;
  });
}

d3s_status d3s_apply_heff_two_site(d3s_ctx ctx, d3s_prec prec, int ml, int d, int mr, int wl, int wc, int wr,
                                   const void* L, const void* W1, const void* W2, const void* R, const void* psi2,
                                   void* out) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(prec == D3S_F64 || prec == D3S_F32, "two-site H_eff: prec must be D3S_F64 or D3S_F32");
    check_dims(ml, d, mr, wl, wr);
    D3S_REQUIRE(wc >= 1 && wc <= 80, "wc out of range");
    D3S_REQUIRE((long)d * d * mr <= (1L << 30) && (long)ml * d * d <= (1L << 30) && (long)ml * d <= 65535 &&
                    (long)wl * d <= 80 && (long)wc * d <= 80 && (long)ml * wl * d * d * mr < (1L << 40) &&
                    (long)ml * wc * d * d * mr < (1L << 40) && (long)ml * wr * d * d * mr < (1L << 40),
                "two-site H_eff: dimensions out of range");
    D3S_REQUIRE(L && W1 && W2 && R && psi2 && out, "null tensor pointer");
    D3S_REQUIRE(out != psi2, "out must not alias psi2");
    d3s::op_apply_heff_two_site(&ctx->c, prec, ml, d, mr, wl, wc, wr, L, W1, W2, R, psi2, out);
    return D3S_OK;
  });
}

d3s_status d3s_cwf_environment(d3s_ctx ctx, int ml, int d, int wl, int wr, const double* L, const double* W,
                               double* Lt) {
  return guarded(ctx, [&] {
    check_dims(ml, d, 1, wl, wr);
    D3S_REQUIRE(L && W && Lt, "null tensor pointer");
    d3s::cwf_environment(&ctx->c, ml, d, wl, wr, L, W, Lt);
    return D3S_OK;
  });
}

d3s_status d3s_apply_cwf(d3s_ctx ctx, d3s_prec prec, int mlp, int mr, int wr, const void* Lt, const void* R,
                         const void* C, void* out) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(prec == D3S_F64 || prec == D3S_F32, "centre-matrix application: prec must be D3S_F64 or D3S_F32");
    check_dims(mlp, 1, mr, wr, wr);
    D3S_REQUIRE(Lt && R && C && out, "null tensor pointer");
    D3S_REQUIRE(out != C, "out must not alias C");
    d3s::op_apply_cwf(&ctx->c, prec, mlp, mr, wr, Lt, R, C, out);
    return D3S_OK;
  });
}

d3s_status d3s_expand_subspace_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* env,
                                      const double* W, const double* psi, double alpha, double* Mt) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    D3S_REQUIRE(!plan->h.packed, "this operation needs a plan of the dense layout");
    D3S_REQUIRE(dir == D3S_L2R || dir == D3S_R2L, "dir must be D3S_L2R or D3S_R2L");
    D3S_REQUIRE(env && W && psi && Mt, "null tensor pointer");
    D3S_REQUIRE(Mt != psi && Mt != env, "Mt must not alias an input");
    D3S_REQUIRE(std::isfinite(alpha), "alpha must be finite");
    d3s::op_expand_blocks(&ctx->c, plan->h, dir, env, W, psi, alpha, Mt);
    return D3S_OK;
  });
}

d3s_status d3s_truncate_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* Mt, const double* psi,
                               int kmax, double rel_cutoff, const double* nbr_in, long nbr_other, double* site_out,
                               double* nbr_out, int renormalize, int maxsec, int* new_nsec, int* new_q,
                               int* new_dim, int* k_out, double* discarded) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    D3S_REQUIRE(!plan->h.packed, "this operation needs a plan of the dense layout");
    D3S_REQUIRE(dir == D3S_L2R || dir == D3S_R2L, "dir must be D3S_L2R or D3S_R2L");
    D3S_REQUIRE(Mt && psi && nbr_in && site_out && nbr_out, "null tensor pointer");
    D3S_REQUIRE(new_nsec && new_q && new_dim && k_out && discarded, "null output pointer");
    D3S_REQUIRE(kmax >= 1 && nbr_other >= 1 && maxsec >= 1, "kmax, nbr_other and maxsec must be >= 1");
    D3S_REQUIRE(rel_cutoff >= 0.0, "rel_cutoff must be >= 0");
    const d3s::BlockHeff& h = plan->h;
    const bool l2r = dir == D3S_L2R;
    const long width = l2r ? (long)(1 + h.wr) * h.mr : (long)(1 + h.wl) * h.ml;
    d3s::TruncBlocksResult t =
        d3s::op_truncate_blocks(&ctx->c, dir, h.left, h.right, h.d, h.pq.data(), l2r ? h.wqr.data() : h.wql.data(),
                                l2r ? h.wr : h.wl, width, Mt, psi, kmax, rel_cutoff, nbr_in, nbr_other, site_out,
                                nbr_out, renormalize != 0);
    D3S_HIP(hipStreamSynchronize(ctx->c.stream));
    const int ns = (int)t.dim.size();
    D3S_REQUIRE(ns <= maxsec, "truncate_blocks: the new bond has more than maxsec sectors");
    const int nq = h.left.nq;
    for (int i = 0; i < ns; ++i) {
      new_dim[i] = t.dim[i];
      for (int k = 0; k < nq; ++k) new_q[i * nq + k] = t.q[(size_t)i * nq + k];
    }
    *new_nsec = ns;
    *k_out = t.k;
    *discarded = t.discarded;
    return D3S_OK;
  });
}

d3s_status d3s_update_env_blocks(d3s_ctx ctx, d3s_block_plan plan, d3s_dir dir, const double* env_in,
                                 const double* W, const double* site, double* env_out) {
  return guarded(ctx, [&] {
    D3S_REQUIRE(plan, "null plan");
    D3S_REQUIRE(!plan->h.packed, "this operation needs a plan of the dense layout");
    D3S_REQUIRE(dir == D3S_L2R || dir == D3S_R2L, "dir must be D3S_L2R or D3S_R2L");
    D3S_REQUIRE(env_in && W && site && env_out, "null tensor pointer");
    D3S_REQUIRE(env_out != env_in && env_out != site, "env_out must not alias an input");
    d3s::op_update_env_blocks(&ctx->c, plan->h, dir, env_in, W, site, env_out);
    return D3S_OK;
  });
}

static d3s::SymChain read_sym(const d3s_state* s, const d3s_symmetry* y) {
  D3S_REQUIRE(y && (y->nq == 1 || y->nq == 2), "symmetry: nq must be 1 or 2");
  D3S_REQUIRE(y->phys_q && y->mpo_q && y->nsec && y->sec_q && y->sec_dim && y->maxsec >= 1,
              "symmetry: null array");
  d3s::SymChain c;
  c.nq = y->nq;
  int wmax = 1;
  for (int b = 0; b <= s->l; ++b) wmax = std::max(wmax, s->w[b]);
  const long dense_cap = (long)s->mmax * wmax * s->mmax;
  D3S_REQUIRE(y->env_cap >= 0, "symmetry: env_cap must be >= 0");
  c.env_cap = y->env_cap > 0 ? y->env_cap : dense_cap;
  c.phys.assign(y->phys_q, y->phys_q + (size_t)s->d * y->nq);
  for (int b = 0; b <= s->l; ++b) {
    D3S_REQUIRE(y->mpo_q[b] && y->sec_q[b] && y->sec_dim[b], "symmetry: null per-bond array");
    c.wq.emplace_back(y->mpo_q[b], y->mpo_q[b] + (size_t)s->w[b] * y->nq);
    D3S_REQUIRE(y->nsec[b] >= 1 && y->nsec[b] <= y->maxsec, "symmetry: sector count out of range");
    long tot = 0;
    for (int i = 0; i < y->nsec[b]; ++i) {
      D3S_REQUIRE(y->sec_dim[b][i] >= 1, "symmetry: sector dimension must be >= 1");
      tot += y->sec_dim[b][i];
    }
    D3S_REQUIRE(tot == s->m[b], "symmetry: sector dimensions of bond " + std::to_string(b) + " do not add up to m");
    c.bonds.emplace_back(y->nq, y->nsec[b], y->sec_q[b], y->sec_dim[b]);
    D3S_REQUIRE((int)c.bonds.back().index.size() == y->nsec[b], "symmetry: repeated charge on a bond");
  }
  return c;
}

static void write_sym(const d3s::SymChain& c, d3s_symmetry* y) {
  for (size_t b = 0; b < c.bonds.size(); ++b) {
    const d3s::Sectors& s = c.bonds[b];
    const int n = std::min(s.n, y->maxsec);
    y->nsec[b] = n;
    for (int i = 0; i < n; ++i) {
      y->sec_dim[b][i] = s.dim[i];
      for (int k = 0; k < c.nq; ++k) y->sec_q[b][i * c.nq + k] = s.q[(size_t)i * c.nq + k];
    }
  }
}

static void check_sym_capacity(const d3s::SymChain& c, const d3s_symmetry* y) {
  for (const d3s::Sectors& s : c.bonds)
    D3S_REQUIRE(s.n <= y->maxsec, "symmetry: more sectors than maxsec");
}

d3s_status d3s_prepare_blocks(d3s_ctx ctx, d3s_state* state, d3s_symmetry* sym, double* energy) {
  return guarded(ctx, [&] {
    check_state(state);
    D3S_REQUIRE(energy, "null energy pointer");
    d3s::SymChain c = read_sym(state, sym);
    *energy = d3s::op_prepare_blocks(&ctx->c, state, c, 1e-14);
    check_sym_capacity(c, sym);
    write_sym(c, sym);
    return D3S_OK;
  });
}

d3s_status d3s_sweep_blocks(d3s_ctx ctx, d3s_state* state, d3s_symmetry* sym, d3s_sweep_params* params,
                            d3s_sweep_stats* stats, int use_graph) {
  return guarded(ctx, [&] {
    check_state(state);
    D3S_REQUIRE(params && stats, "null params or stats");
    D3S_REQUIRE(stats->records || stats->capacity == 0, "stats: null records with capacity > 0");
    check_prec(params->prec);
    D3S_REQUIRE(params->lanczos_kmax >= 2 && params->lanczos_kmax <= 64, "lanczos_kmax must be in [2, 64]");
    D3S_REQUIRE(params->lanczos_tol > 0.0 && params->lanczos_max_matvecs >= 1, "bad eigensolver limits");
    D3S_REQUIRE(params->alpha >= 0.0 && std::isfinite(params->alpha), "alpha must be finite and >= 0");
    D3S_REQUIRE(params->mixed_min_gflop >= 0.0, "mixed_min_gflop must be >= 0");
    D3S_REQUIRE(params->expansion == 0, "block sweeps: only the expansion term of eq. subexp-ourt (expansion = 0)");
    d3s::SymChain c = read_sym(state, sym);
    try {
      d3s::op_sweep_blocks(&ctx->c, state, c, params, stats, use_graph != 0);
    } catch (...) {
      if ([&] { for (auto& s : c.bonds) if (s.n > sym->maxsec) return false; return true; }()) write_sym(c, sym);
      throw;
    }
    check_sym_capacity(c, sym);
    write_sym(c, sym);
    if (!std::isfinite(stats->energy)) throw Error{D3S_ENUMERIC, "sweep: non-finite energy"};
    return stats->nonconverged ? D3S_ENOCONV : D3S_OK;
  });
}

}  // extern "C"
