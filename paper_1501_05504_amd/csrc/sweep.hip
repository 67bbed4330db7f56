// Sweep driver (Sec. 5, steps 1-8; alpha rule of Sec. 6), host C++.
//
// Readings of points the paper leaves open (the same readings the test
// oracle uses, kept here as constants):
//  - eigensolver: Lanczos with full re-orthogonalisation, warm start from
//    the current site tensor;
//  - truncation target of bond b: min(mmax, d^b, d^(l-b)); singular values
//    s_j <= eps s_0 are dropped;
//  - the neighbour is renormalised after absorbing S V^T, so E_f is a
//    Rayleigh quotient, and E_f becomes E_before of the next site update;
//  - alpha: no change when the truncation discarded no weight (the
//    enrichment had no effect), otherwise shrink by 0.8 when |dE_O| <
//    1e-13 |E|, grow by 1.25 when dE_T < 0.3 |dE_O|, else shrink by 0.8;
//    clamped to [1e-16, 1];
//  - a sweep is right-to-left over sites l-1..1 followed by left-to-right
//    over sites 0..l-2;
//  - with the exact-residual expansion E is the eigenvalue of the site's
//    local problem, and the truncation works from the Gram matrix of the
//    expanded tensor (singular values resolved down to sqrt(n u) s_0, as
//    for the explicit expanded tensor).
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "d3s_internal.h"

namespace d3s {
namespace {

constexpr double kAlphaTarget = 0.3;
constexpr double kAlphaGrow = 1.25;
constexpr double kAlphaShrink = 0.8;
constexpr double kAlphaStall = 1e-13;
constexpr double kAlphaNoCut = 1e-12;
constexpr double kAlphaMin = 1e-16;
constexpr double kAlphaMax = 1.0;

long bond_budget(int l, int d, int mmax, int b) {
  long cap = mmax;
  long left = 1, right = 1;
  for (int i = 0; i < b && left < cap; ++i) left *= d;
  for (int i = 0; i < l - b && right < cap; ++i) right *= d;
  return std::min(cap, std::min(left, right));
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void update_alpha(d3s_sweep_params* p, double lam, double ef, double disc, double total) {
  if (!p->adaptive_alpha) return;
  const double dEO = lam - p->e_before;
  const double dET = ef - lam;
  if (disc <= kAlphaNoCut * total) {
    // the expansion did not change the state: no information on alpha
  } else if (std::fabs(dEO) < kAlphaStall * std::fabs(lam)) {
    p->alpha *= kAlphaShrink;
  } else if (dET < kAlphaTarget * std::fabs(dEO)) {
    p->alpha *= kAlphaGrow;
  } else {
    p->alpha *= kAlphaShrink;
  }
  p->alpha = std::min(kAlphaMax, std::max(kAlphaMin, p->alpha));
}

int wmax_of(const d3s_state* s) {
  int w = 1;
  for (int i = 0; i <= s->l; ++i) w = std::max(w, s->w[i]);
  return w;
}

}  // namespace

double op_prepare(Ctx* c, d3s_state* s, double eps) {
  const int l = s->l, d = s->d;
  for (int b = 0; b <= l; ++b) {
    const long bb = bond_budget(l, d, s->mmax, b);
    if (s->m[b] > bb) throw Error{D3S_EINVAL, "prepare: bond " + std::to_string(b) + " exceeds its budget"};
  }
  const size_t cap = (size_t)s->mmax * d * s->mmax;
  double* tmpS = (double*)ws_get(c, WS_PSI, sizeof(double) * cap);
  double* tmpN = (double*)ws_get(c, WS_NBR, sizeof(double) * cap);
  // the neighbour is renormalised at every step: the state's direction is
  // unchanged, and the norm of a long random MPS cannot overflow the Gram
  // matrices on the way
  for (int i = 0; i + 1 < l; ++i) {
    const int ml = s->m[i], mr = s->m[i + 1];
    const long other = (long)d * s->m[i + 2];
    TruncResult t = op_truncate(c, D3S_L2R, ml, d, mr, mr, s->site[i], s->site[i], (int)bond_budget(l, d, s->mmax, i + 1),
                                eps, s->site[i + 1], other, tmpS, tmpN, nullptr, true);
    copy_f64(c, tmpS, s->site[i], (long)ml * d * t.k);
    copy_f64(c, tmpN, s->site[i + 1], (long)t.k * other);
    s->m[i + 1] = t.k;
  }
  // normalise the last site
  {
    const long n = (long)s->m[l - 1] * d * s->m[l];
    double* r = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 512);
    dot_f64(c, s->site[l - 1], s->site[l - 1], n, r);
    const double nrm2 = read_scalar(c, r);
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2)) throw Error{D3S_ENUMERIC, "prepare: zero state"};
    scale_f64(c, s->site[l - 1], n, 1.0 / std::sqrt(nrm2));
  }
  fill_f64(c, s->lenv[0], 1, 1.0);
  fill_f64(c, s->renv[l - 1], 1, 1.0);
  for (int i = 0; i + 1 < l; ++i)
    op_update_env(c, D3S_L2R, s->m[i], d, s->m[i + 1], s->w[i], s->w[i + 1], s->lenv[i], s->mpo[i],
                  s->site[i], s->lenv[i + 1]);
  s->center = l - 1;
  return op_energy(c, s->m[l - 1], d, s->m[l], s->w[l - 1], s->w[l], s->lenv[l - 1], s->mpo[l - 1],
                   s->renv[l - 1], s->site[l - 1]);
}

void op_sweep(Ctx* c, d3s_state* s, d3s_sweep_params* p, d3s_sweep_stats* st) {
  const int mlim = (p->m_limit > 0 && p->m_limit < s->mmax) ? p->m_limit : s->mmax;
  const int l = s->l, d = s->d;
  if (s->center != l - 1) throw Error{D3S_EINVAL, "sweep: the orthogonality centre must be on site l-1"};
  const int wmax = wmax_of(s);
  const size_t cap = (size_t)s->mmax * d * s->mmax;
  const bool residual = p->expansion == 1;
  // exact residual: H^2 environments, left ones per bond 0..l-1 (h2l[i] left
  // of site i) and right ones per site (h2r[i] right of site i), in one
  // workspace buffer sized for the largest bond each may reach
  std::vector<double*> h2l, h2r;
  if (residual) {
    std::vector<size_t> off_l(l), off_r(l);
    size_t total = 0;
    for (int b = 0; b < l; ++b) {
      const size_t m = (size_t)bond_budget(l, d, s->mmax, b);
      off_l[b] = total;
      total += m * m * s->w[b] * s->w[b];
    }
    for (int i = 0; i < l; ++i) {
      const size_t m = (size_t)bond_budget(l, d, s->mmax, i + 1);
      off_r[i] = total;
      total += m * m * s->w[i + 1] * s->w[i + 1];
    }
    if (total > ((size_t)1 << 32))
      throw Error{D3S_EINVAL, "sweep: the exact-residual expansion needs " + std::to_string(total * 8 >> 30) +
                                  " GiB of H^2 environments; use a smaller mmax"};
    double* base = (double*)ws_get(c, WS_H2, sizeof(double) * total);
    for (int b = 0; b < l; ++b) h2l.push_back(base + off_l[b]);
    for (int i = 0; i < l; ++i) h2r.push_back(base + off_r[i]);
    fill_f64(c, h2l[0], 1, 1.0);
    fill_f64(c, h2r[l - 1], 1, 1.0);
    for (int i = 0; i + 1 < l; ++i)
      op_update_env_h2(c, D3S_L2R, s->m[i], d, s->m[i + 1], s->w[i], s->w[i + 1], h2l[i], s->mpo[i], s->site[i],
                       h2l[i + 1]);
  }
  double* tmpS = (double*)ws_get(c, WS_PSI, sizeof(double) * cap);
  double* tmpN = (double*)ws_get(c, WS_NBR, sizeof(double) * cap);
  // [psi | alpha P] has (1 + w) m columns; the residual's expanded tensor at
  // most m + (1 + w) m
  double* Mt = (double*)ws_get(c, WS_MT, sizeof(double) * (size_t)((residual ? 2 : 1) + wmax) * cap);
  const double t_start = now();
  st->count = 0;
  st->nonconverged = 0;
  auto record = [&](const d3s_site_record& r) {
    if (st->count < st->capacity) st->records[st->count] = r;
    st->count++;
  };
  double lam = p->e_before;
  // right to left
  for (int i = l - 1; i >= 1; --i) {
    d3s_site_record r{};
    r.site = i;
    r.dir = D3S_R2L;
    r.e_before = p->e_before;
    const int ml = s->m[i], mr = s->m[i + 1], wl = s->w[i], wr = s->w[i + 1];
    double t0 = now();
    const double gf = 2e-9 * ((double)wl * d * ml * ml * mr + (double)d * d * wl * wr * ml * mr + (double)wr * d * ml * mr * mr);
    const d3s_prec prec = (gf >= p->mixed_min_gflop) ? p->prec : D3S_F64;
    LanczosResult lz = op_lanczos(c, prec, ml, d, mr, wl, wr, s->lenv[i], s->mpo[i], s->renv[i], s->site[i],
                                  p->lanczos_tol, p->lanczos_kmax, p->lanczos_max_matvecs);
    lam = lz.theta;
    if (!lz.converged) st->nonconverged++;
    double t1 = now();
    long rows = (long)(1 + wl) * ml;
    if (residual)
      rows = op_residual_expand(c, D3S_R2L, ml, d, mr, wl, wr, s->lenv[i], s->renv[i], h2l[i], s->mpo[i],
                                s->site[i], lam, p->alpha, Mt);
    else
      op_expand(c, D3S_R2L, ml, d, mr, wl, wr, s->renv[i], s->mpo[i], s->site[i], p->alpha, Mt);
    D3S_HIP(hipStreamSynchronize(c->stream));
    double t2 = now();
    c->stat_eig_s = 0.0;
    c->stat_passes = 0;
    const int mll = s->m[i - 1];
    TruncResult t = op_truncate(c, D3S_R2L, ml, d, mr, rows, Mt, s->site[i], (int)bond_budget(l, d, mlim, i),
                                p->eps, s->site[i - 1], (long)mll * d, tmpS, tmpN, nullptr, true);
    copy_f64(c, tmpS, s->site[i], (long)t.k * d * mr);
    copy_f64(c, tmpN, s->site[i - 1], (long)mll * d * t.k);
    s->m[i] = t.k;
    double t3 = now();
    r.t_trunc_eig = c->stat_eig_s;
    r.trunc_passes = c->stat_passes;
    op_update_env(c, D3S_R2L, t.k, d, mr, wl, wr, s->renv[i], s->mpo[i], s->site[i], s->renv[i - 1]);
    if (residual)
      op_update_env_h2(c, D3S_R2L, t.k, d, mr, wl, wr, h2r[i], s->mpo[i], s->site[i], h2r[i - 1]);
    D3S_HIP(hipStreamSynchronize(c->stream));
    double t4 = now();
    const double ef = op_energy(c, mll, d, t.k, s->w[i - 1], wl, s->lenv[i - 1], s->mpo[i - 1], s->renv[i - 1],
                                s->site[i - 1]);
    double t5 = now();
    r.k = t.k;
    r.matvecs = lz.matvecs;
    r.f64_matvecs = lz.f64_matvecs;
    r.lambda = lam;
    r.e_f = ef;
    r.alpha = p->alpha;
    r.discarded = t.discarded;
    r.t_eig = t1 - t0; r.t_expand = t2 - t1; r.t_trunc = t3 - t2; r.t_env = t4 - t3; r.t_energy = t5 - t4;
    record(r);
    update_alpha(p, lam, ef, t.discarded, t.total);
    p->e_before = ef;
    s->center = i - 1;
  }
  // left to right
  for (int i = 0; i + 1 < l; ++i) {
    d3s_site_record r{};
    r.site = i;
    r.dir = D3S_L2R;
    r.e_before = p->e_before;
    const int ml = s->m[i], mr = s->m[i + 1], wl = s->w[i], wr = s->w[i + 1];
    double t0 = now();
    const double gf = 2e-9 * ((double)wl * d * ml * ml * mr + (double)d * d * wl * wr * ml * mr + (double)wr * d * ml * mr * mr);
    const d3s_prec prec = (gf >= p->mixed_min_gflop) ? p->prec : D3S_F64;
    LanczosResult lz = op_lanczos(c, prec, ml, d, mr, wl, wr, s->lenv[i], s->mpo[i], s->renv[i], s->site[i],
                                  p->lanczos_tol, p->lanczos_kmax, p->lanczos_max_matvecs);
    lam = lz.theta;
    if (!lz.converged) st->nonconverged++;
    double t1 = now();
    long width = (long)(1 + wr) * mr;
    if (residual)
      width = op_residual_expand(c, D3S_L2R, ml, d, mr, wl, wr, s->lenv[i], s->renv[i], h2r[i], s->mpo[i],
                                 s->site[i], lam, p->alpha, Mt);
    else
      op_expand(c, D3S_L2R, ml, d, mr, wl, wr, s->lenv[i], s->mpo[i], s->site[i], p->alpha, Mt);
    D3S_HIP(hipStreamSynchronize(c->stream));
    double t2 = now();
    c->stat_eig_s = 0.0;
    c->stat_passes = 0;
    const int mrr = s->m[i + 2];
    TruncResult t = op_truncate(c, D3S_L2R, ml, d, mr, width, Mt, s->site[i], (int)bond_budget(l, d, mlim, i + 1),
                                p->eps, s->site[i + 1], (long)d * mrr, tmpS, tmpN, nullptr, true);
    copy_f64(c, tmpS, s->site[i], (long)ml * d * t.k);
    copy_f64(c, tmpN, s->site[i + 1], (long)t.k * d * mrr);
    s->m[i + 1] = t.k;
    double t3 = now();
    r.t_trunc_eig = c->stat_eig_s;
    r.trunc_passes = c->stat_passes;
    op_update_env(c, D3S_L2R, ml, d, t.k, wl, wr, s->lenv[i], s->mpo[i], s->site[i], s->lenv[i + 1]);
    if (residual)
      op_update_env_h2(c, D3S_L2R, ml, d, t.k, wl, wr, h2l[i], s->mpo[i], s->site[i], h2l[i + 1]);
    D3S_HIP(hipStreamSynchronize(c->stream));
    double t4 = now();
    const double ef = op_energy(c, t.k, d, mrr, wr, s->w[i + 2], s->lenv[i + 1], s->mpo[i + 1], s->renv[i + 1],
                                s->site[i + 1]);
    double t5 = now();
    r.k = t.k;
    r.matvecs = lz.matvecs;
    r.f64_matvecs = lz.f64_matvecs;
    r.lambda = lam;
    r.e_f = ef;
    r.alpha = p->alpha;
    r.discarded = t.discarded;
    r.t_eig = t1 - t0; r.t_expand = t2 - t1; r.t_trunc = t3 - t2; r.t_env = t4 - t3; r.t_energy = t5 - t4;
    record(r);
    update_alpha(p, lam, ef, t.discarded, t.total);
    p->e_before = ef;
    s->center = i + 1;
  }
  st->energy = lam;
  st->seconds = now() - t_start;
}

// dE/dW_i of <Psi|H|Psi> for every site i, each taken with the environments
// of the gauge centred on i (product rule over the MPO tensors).  Starts from
// the centre on site l-1 with lenv[0..l-1] valid, walks right to left moving
// the centre by a truncation without expansion that drops only singular
// values below 1e-14 s_0 (the state is unchanged to rounding), and leaves the
// centre on site 0 with renv[0..l-1] valid.
void op_gradients(Ctx* c, d3s_state* s, double** grads) {
  const int l = s->l, d = s->d;
  if (s->center != l - 1) throw Error{D3S_EINVAL, "gradients: the orthogonality centre must be on site l-1"};
  const size_t cap = (size_t)s->mmax * d * s->mmax;
  double* tmpS = (double*)ws_get(c, WS_PSI, sizeof(double) * cap);
  double* tmpN = (double*)ws_get(c, WS_NBR, sizeof(double) * cap);
  for (int i = l - 1; i >= 0; --i) {
    const int ml = s->m[i], mr = s->m[i + 1], wl = s->w[i], wr = s->w[i + 1];
    op_heff_grad_W(c, ml, d, mr, wl, wr, s->lenv[i], s->renv[i], s->site[i], s->site[i], grads[i]);
    if (i == 0) break;
    const int mll = s->m[i - 1];
    TruncResult t = op_truncate(c, D3S_R2L, ml, d, mr, ml, s->site[i], s->site[i], ml, 1e-14, s->site[i - 1],
                                (long)mll * d, tmpS, tmpN, nullptr, false);
    copy_f64(c, tmpS, s->site[i], (long)t.k * d * mr);
    copy_f64(c, tmpN, s->site[i - 1], (long)mll * d * t.k);
    s->m[i] = t.k;
    op_update_env(c, D3S_R2L, t.k, d, mr, wl, wr, s->renv[i], s->mpo[i], s->site[i], s->renv[i - 1]);
    s->center = i - 1;
  }
  D3S_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace d3s
