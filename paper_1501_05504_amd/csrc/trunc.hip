// Truncation of an expanded tensor (steps 4-5 of the site update, Sec. 5;
// Sec. 4.2 notes that the SVD dominates the cost of the expansion) for a set
// of matrices handled together: the charge sectors of a block-diagonal
// truncation, or the single matrix of a dense one.  Every matrix X_q
// (n_q x c_q, row-major) gets its left singular vectors and singular values,
// and the kept states are chosen over all matrices: at most kmax, and only
// s_j > eps * s_0 with s_0 the largest singular value of all.
//
// The singular values come from the FP64 Gram matrix X X^T (an MFMA GEMM)
// and its eigenvalues, but an eigenvalue carries an absolute error of order
// u * lambda_max, so one pass resolves s_j only down to about
// sqrt(n u) s_0 (~1e-6 s_0 at n = 8192), far above eps = 1e-14.  The rest is
// found by deflation:
//  * pass 1: eigenpairs (Y, lambda) of G = X X^T.  Eigenvalues at or above
//    tau^2 lambda_max are accepted, tau^2 = max(1e-10, 64 n u), where the
//    error is a small fraction of the value.
//  * the other eigenvectors T (an orthonormal basis of the complement,
//    orthonormal to rounding) give the tail coefficients Z = T^T X.  Their
//    rows still carry the accepted right singular directions, mixed in at
//    about u s_0^2 / s_i; projecting them off, Z <- Z (1 - v v^T) with v the
//    normalised rows of Y_acc^T X, leaves an error second order in that
//    mixing.
//  * the next pass repeats this on Z Z^T, its eigenvectors mapped back
//    through T; every pass reaches about tau below the previous one.
// A matrix is refined only while its unresolved values (below
// sqrt(2) tau s_max of its last pass) could still be kept, i.e. exceed eps *
// s_0 and the kmax-th largest accepted value over all matrices; at most
// kMaxPass passes.
//
// Batched eigensolves pad every matrix of a batch to a common size.  Each
// matrix is first divided by its largest diagonal entry, and the padding
// gets -1 on its diagonal, so that its eigenvectors separate from the real
// ones (which then sit in the last n columns, supported on the first n rows,
// to rounding).
#include <algorithm>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <map>

#include "d3s_internal.h"

namespace d3s {
namespace {

constexpr int kMaxPass = 4;
constexpr int kThr = 256;

struct PadDesc { long off; int n, npad; };
struct RowScale { long off, ld; int rows, cols; long foff; };

// scale[q] = max_i |G_ii| of the real n x n part of matrix q (1 if zero);
// one workgroup per matrix
__global__ __launch_bounds__(kThr) void gram_scale_kernel(const double* __restrict__ G,
                                                          const PadDesc* __restrict__ desc,
                                                          double* __restrict__ scale) {
  const PadDesc p = desc[blockIdx.x];
  __shared__ double red[kThr];
  // a non-finite diagonal entry (a NaN or Inf in the matrix's rows) makes the
  // maximum +Inf, which the host reports
  double mx = 0.0;
  for (int i = threadIdx.x; i < p.n; i += kThr) {
    const double g = G[p.off + (long)i * p.npad + i];
    mx = isfinite(g) ? fmax(mx, fabs(g)) : INFINITY;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kThr / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[blockIdx.x] = red[0] > 0.0 ? red[0] : 1.0;
}

// the real part of matrix q (grid y) divided by scale[q], its padded
// diagonal set to -1 (the padded off-diagonal entries are zero)
__global__ __launch_bounds__(kThr) void gram_normalize_kernel(double* __restrict__ G,
                                                              const PadDesc* __restrict__ desc,
                                                              const double* __restrict__ scale) {
  const PadDesc p = desc[blockIdx.y];
  const double f = 1.0 / scale[blockIdx.y];
  const long total = (long)p.npad * p.npad;
  for (long e = (long)blockIdx.x * kThr + threadIdx.x; e < total; e += (long)gridDim.x * kThr) {
    const long i = e / p.npad, j = e - i * p.npad;
    if (i < p.n && j < p.n) G[p.off + e] *= f;
    else if (i == j) G[p.off + e] = -1.0;
  }
}

// X[off + r*ld + c] *= f[foff + r] for every descriptor (grid y)
__global__ __launch_bounds__(kThr) void scale_rows_kernel(double* __restrict__ X, const double* __restrict__ f,
                                                          const RowScale* __restrict__ desc) {
  const RowScale d = desc[blockIdx.y];
  const long total = (long)d.rows * d.cols;
  for (long i = (long)blockIdx.x * kThr + threadIdx.x; i < total; i += (long)gridDim.x * kThr) {
    const long r = i / d.cols, col = i - r * d.cols;
    X[d.off + r * d.ld + col] *= f[d.foff + r];
  }
}

double tau2_of(int n) { return std::max(1e-10, 64.0 * (double)n * DBL_EPSILON); }

// One GEMM per matrix of the set: C_q = alpha A_q B_q + beta C_q.  A single
// product goes to the plain GEMM, several to one grouped launch.
struct MTask { int M, N, K; long a_off, lda, b_off, ldb, c_off, ldc; };

void multi_gemm(Ctx* c, const std::vector<MTask>& ts, bool a_kc, bool b_kc, const double* A, const double* B,
                double* C, double alpha, double beta) {
  std::vector<MTask> live;
  for (const MTask& t : ts)
    if (t.M > 0 && t.N > 0 && t.K > 0) live.push_back(t);
  if (live.empty()) return;
  if (live.size() == 1) {
    const MTask& t = live[0];
    GemmArgs g{t.M, t.N, t.K, A + t.a_off, t.lda, a_kc, 0, B + t.b_off, t.ldb, b_kc, 0, C + t.c_off, t.ldc, 0,
               alpha, beta, 1};
    gemm_f64(c, g);
    return;
  }
  GroupedPlan gp;
  gp.a_kc = a_kc;
  gp.b_kc = b_kc;
  gp.table_slot = WS_TR_TAB;
  for (const MTask& t : live) {
    GTask task{t.M, t.N, (int)gp.segs.size(), 1, 0, t.c_off, t.ldc};
    gp.segs.push_back(GSeg{t.K, t.a_off, t.lda, t.b_off, t.ldb});
    gp.tasks.push_back(task);
  }
  grouped_finalize(c, gp);
  grouped_gemm(c, D3S_F64, gp, A, B, C, alpha, beta);
  grouped_release(gp);
}

}  // namespace

// Batches of the eigensolver.  Measured on MI355X (rocSOLVER
// dsyevd_strided_batched): from n = 96 on a call costs about 24 us per
// matrix column whatever the batch size (launch-bound) plus ~1.6e-12 n^3 s
// per matrix, while below n = 96 its batched small-size path grows steeply
// with the batch (n = 64, 40 matrices: 18 ms against 2 ms at n = 96).  With
// the LDS solver chosen, matrices up to 128 may go to it instead (one
// workgroup per matrix, nothing launched per column, about 5e-5 + 6.5e-7 n^2
// s per batch of up to 256).  Sizes are padded (to a multiple of 8 for the
// LDS solver, else to at least 96 and a multiple of 16; a lone matrix is not
// padded), sorted, and grouped contiguously with the least modelled cost
// (dynamic programming).
EigPlan plan_eig(Ctx* c, const std::vector<int>& n) {
  EigPlan ep;
  const int Q = (int)n.size();
  ep.npad.assign(Q, 0);
  ep.goff.assign(Q, 0);
  ep.voff.assign(Q, 0);
  std::vector<int> ord;
  for (int q = 0; q < Q; ++q)
    if (n[q] > 0) ord.push_back(q);
  if (ord.empty()) return ep;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return n[a] < n[b]; });
  auto small = [&](int m) { return eig_small_used(c, (m + 7) / 8 * 8); };
  auto pad = [&](int m, int cnt) {
    if (small(m)) return (m + 7) / 8 * 8;
    return cnt == 1 ? m : std::max(96, (m + 15) / 16 * 16);
  };
  // With K concurrent shares (below) the launch chains of separate calls
  // overlap, so grouping is charged 1/K of a column's serial cost: fewer,
  // padded calls save less than they would one after the other (measured:
  // the full serial cost grouped too much on the cylinder and the chain)
  const int shares = (c->eig_workers >= 2 && c->eig_kind != 2) ? c->eig_workers : 1;
  const double col = 2.4e-5 / shares;
  auto cost = [&](int i, int j) {
    const int cnt = j - i + 1;
    const double np = pad(n[ord[j]], cnt);
    if (small(n[ord[j]])) return (5e-5 + 6.5e-7 * np * np) * ((cnt + 255) / 256);
    return col * np + 1.6e-12 * (double)cnt * np * np * np;
  };
  const int G = (int)ord.size();
  std::vector<double> best(G + 1, 0.0);
  std::vector<int> cut(G + 1, 0);
  for (int j = 1; j <= G; ++j) {
    best[j] = 1e300;
    for (int i = 0; i < j; ++i) {
      const double v = best[i] + cost(i, j - 1);
      if (v < best[j]) {
        best[j] = v;
        cut[j] = i;
      }
    }
  }
  std::vector<std::pair<int, int>> ranges;
  for (int j = G; j > 0; j = cut[j]) ranges.push_back({cut[j], j - 1});
  for (auto& r : ranges) {
    const int cnt = r.second - r.first + 1;
    const int np = pad(n[ord[r.second]], cnt);
    ep.bucket_n.push_back(np);
    ep.bucket_goff.push_back(ep.gtot);
    ep.bucket_voff.push_back(ep.vtot);
    ep.members.emplace_back();
    for (int i = r.first; i <= r.second; ++i) {
      const int q = ord[i];
      ep.npad[q] = np;
      ep.goff[q] = ep.gtot;
      ep.voff[q] = ep.vtot;
      ep.gtot += (long)np * np;
      ep.vtot += np;
      ep.members.back().push_back(q);
    }
    ep.calls.push_back(EigCall{np, cnt, ep.bucket_goff.back(), ep.bucket_voff.back()});
  }
  // Concurrent solves (divide and conquer only): each call's cost model as
  // above; the calls are dealt to the workers largest first, each to the
  // least loaded, and a call of several matrices is halved (its halves are
  // two calls on consecutive matrices) while that lowers the largest load.
  const int K = c->eig_workers;
  bool all_dc = c->eig_kind != 2;
  for (int b : ep.bucket_n)
    all_dc = all_dc && !eig_small_used(c, b) && !(c->eig_kind == 0 && b <= c->eig_jacobi_max);
  if (K >= 2 && all_dc && !ep.calls.empty()) {
    auto cc = [](const EigCall& e) { return 2.4e-5 * e.n + 1.6e-12 * (double)e.batch * e.n * e.n * (double)e.n; };
    auto assign = [&](std::vector<EigCall>& calls, std::vector<int>& who) {
      std::vector<int> ord2(calls.size());
      for (size_t i = 0; i < ord2.size(); ++i) ord2[i] = (int)i;
      std::stable_sort(ord2.begin(), ord2.end(), [&](int a, int b) { return cc(calls[a]) > cc(calls[b]); });
      std::vector<double> load(K, 0.0);
      who.assign(calls.size(), 0);
      for (int i : ord2) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        who[i] = k;
        load[k] += cc(calls[i]);
      }
      return *std::max_element(load.begin(), load.end());
    };
    std::vector<int> who;
    double span = assign(ep.calls, who);
    for (;;) {
      double best = span;
      std::vector<EigCall> best_calls;
      for (size_t i = 0; i < ep.calls.size(); ++i) {
        const EigCall e = ep.calls[i];
        if (e.batch < 2) continue;
        const int h = e.batch / 2;
        std::vector<EigCall> t = ep.calls;
        t[i] = EigCall{e.n, h, e.goff, e.voff};
        t.push_back(EigCall{e.n, e.batch - h, e.goff + (long)h * e.n * e.n, e.voff + (long)h * e.n});
        std::vector<int> w2;
        const double v = assign(t, w2);
        if (v < best - 1e-9) {
          best = v;
          best_calls = t;
        }
      }
      if (best_calls.empty()) break;
      ep.calls = best_calls;
      span = best;
    }
    assign(ep.calls, ep.worker);
    ep.workers = (ep.calls.size() >= 2) ? K : 1;
  }
  return ep;
}

// rocSOLVER's divide and conquer loses accuracy on matrices of small norm
// (measured on MI355X: a graded Gram matrix scaled by 1e-6 / 1e-10 / 1e-20
// had eigen-residuals of 2e-10 / 1e-6 / 1e-2 of its norm against 3e-16 at
// norm 1), and a deflated tail or a light charge sector has a small norm.
// Every matrix is therefore divided by its largest diagonal entry (so its
// norm lies in [1, n]) before the solve; scale[q] (host) returns the factor
// by which its eigenvalues must be multiplied.
void eig_run(Ctx* c, const EigPlan& ep, const std::vector<int>& n, double* G, double* V,
             std::vector<double>& scale) {
  std::vector<PadDesc> mats;
  std::vector<int> qs;
  long maxel = 1;
  for (size_t q = 0; q < n.size(); ++q)
    if (n[q] > 0) {
      mats.push_back(PadDesc{ep.goff[q], n[q], ep.npad[q]});
      qs.push_back((int)q);
      maxel = std::max(maxel, (long)ep.npad[q] * ep.npad[q]);
    }
  scale.assign(n.size(), 1.0);
  if (mats.empty()) return;
  const size_t db = (sizeof(PadDesc) * mats.size() + 255) & ~(size_t)255;
  char* aux = (char*)ws_get(c, WS_TR_AUX, db + sizeof(double) * mats.size());
  PadDesc* d = (PadDesc*)aux;
  double* sc = (double*)(aux + db);
  D3S_HIP(hipMemcpyAsync(d, mats.data(), sizeof(PadDesc) * mats.size(), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(gram_scale_kernel, dim3((unsigned)mats.size()), dim3(kThr), 0, c->stream, G, d, sc);
  D3S_HIP(hipGetLastError());
  std::vector<double> hs(mats.size());
  D3S_HIP(hipMemcpyAsync(hs.data(), sc, sizeof(double) * mats.size(), hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  for (double v : hs)
    if (!std::isfinite(v)) throw Error{D3S_ENUMERIC, "truncate: the expanded tensor is not finite"};
  const unsigned gx = (unsigned)std::min<long>((maxel + kThr - 1) / kThr, 2048);
  hipLaunchKernelGGL(gram_normalize_kernel, dim3(gx, (unsigned)mats.size()), dim3(kThr), 0, c->stream, G, d, sc);
  D3S_HIP(hipGetLastError());
  D3S_HIP(hipStreamSynchronize(c->stream));
  const auto t0 = std::chrono::steady_clock::now();
  if (ep.workers >= 2) {
    eig_calls_parallel(c, ep.calls, ep.worker, ep.workers, G, V);
  } else {
    for (size_t b = 0; b < ep.bucket_n.size(); ++b)
      eig_batched_f64(c, ep.bucket_n[b], (int)ep.members[b].size(), G + ep.bucket_goff[b], V + ep.bucket_voff[b]);
  }
  // every solve path ends with a readback of its convergence flags
  c->stat_eig_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (size_t i = 0; i < qs.size(); ++i) scale[qs[i]] = hs[i];
}

void trunc_solve(Ctx* c, const TruncMats& tm, int kmax, double eps, TruncSel& out) {
  const int Q = (int)tm.nr.size();
  out = TruncSel();
  out.s.assign(Q, {});
  out.vecs.assign(Q, {});
  out.keep.assign(Q, 0);
  out.rest.assign(Q, {});
  // per-matrix state of the current pass: Z (n x nc) and T (n x nr; nullptr
  // base = identity), both row-major with their leading dimensions
  struct St {
    int n = 0;
    const double* zb = nullptr; long zo = 0, zl = 0;
    const double* tb = nullptr; long to = 0, tl = 0;
    std::vector<double> lam;   // eigenvalues of the current problem, ascending, clipped at 0
    double ub = 0.0;
    int kp = 0;                // accepted in the current pass
    const double* vb = nullptr; long vo = 0, vs = 0;   // vectors of the current pass: row j at vb + vo + j*vs
  };
  std::vector<St> st(Q);
  for (int q = 0; q < Q; ++q) {
    st[q].n = tm.nr[q];
    st[q].zb = tm.X;
    st[q].zo = tm.xoff[q];
    st[q].zl = tm.nc[q];
  }
  std::vector<int> solve(Q, 1);
  double s0 = 0.0;
  for (int pass = 1;; ++pass) {
    ++c->stat_passes;
    // ---- Gram matrices of this pass, padded batched eigensolves
    std::vector<int> nsolve(Q, 0);
    for (int q = 0; q < Q; ++q)
      if (solve[q]) nsolve[q] = st[q].n;
    const EigPlan ep = plan_eig(c, nsolve);
    double* G = (double*)ws_get(c, pass == 1 ? WS_GPACK : WS_TR_G, sizeof(double) * (size_t)std::max(ep.gtot, 1L));
    double* V = (double*)ws_get(c, pass == 1 ? WS_GVAL : WS_TR_V, sizeof(double) * (size_t)std::max(ep.vtot, 1L));
    zero_bytes(c, G, sizeof(double) * (size_t)ep.gtot);
    {
      std::vector<MTask> ts;
      for (int q = 0; q < Q; ++q)
        if (nsolve[q] > 0)
          ts.push_back(MTask{st[q].n, st[q].n, tm.nc[q], st[q].zo, st[q].zl, st[q].zo, st[q].zl, ep.goff[q],
                             (long)ep.npad[q]});
      // all Z of one pass live in one buffer
      const double* zb = nullptr;
      for (int q = 0; q < Q; ++q)
        if (nsolve[q] > 0) zb = st[q].zb;
      multi_gemm(c, ts, true, true, zb, zb, G, 1.0, 0.0);
    }
    std::vector<double> gscale;
    eig_run(c, ep, nsolve, G, V, gscale);
    std::vector<double> ev(std::max(ep.vtot, 1L));
    D3S_HIP(hipMemcpyAsync(ev.data(), V, sizeof(double) * (size_t)ep.vtot, hipMemcpyDeviceToHost, c->stream));
    D3S_HIP(hipStreamSynchronize(c->stream));
    // ---- accepted values; the vectors of this pass
    // pass >= 2: T' = Y_real^T T into this pass's own buffer (its accepted
    // rows are the results and must survive later passes)
    double* Tp = nullptr;
    std::vector<long> tpo(Q, 0);
    if (pass >= 2) {
      long tot = 0;
      for (int q = 0; q < Q; ++q)
        if (nsolve[q] > 0) {
          tpo[q] = tot;
          tot += (long)st[q].n * tm.nr[q];
        }
      Tp = (double*)ws_get(c, WS_TR_T2 + (pass - 2), sizeof(double) * (size_t)std::max(tot, 1L));
      std::vector<MTask> ts;
      const double* tb = nullptr;
      for (int q = 0; q < Q; ++q)
        if (nsolve[q] > 0) {
          const int n = st[q].n, np = ep.npad[q];
          ts.push_back(MTask{n, tm.nr[q], n, ep.goff[q] + (long)(np - n) * np, (long)np, st[q].to, st[q].tl,
                             tpo[q], (long)tm.nr[q]});
          tb = st[q].tb;
        }
      multi_gemm(c, ts, true, false, G, tb, Tp, 1.0, 0.0);
    }
    for (int q = 0; q < Q; ++q) {
      if (!nsolve[q]) continue;
      St& s = st[q];
      const int n = s.n, np = ep.npad[q];
      s.lam.assign(n, 0.0);
      for (int j = 0; j < n; ++j) s.lam[j] = std::max(ev[ep.voff[q] + np - n + j], 0.0) * gscale[q];
      if (pass == 1)
        for (int j = 0; j < n; ++j) out.total += s.lam[j];
      const double lmax = s.lam[n - 1];
      const double t2 = tau2_of(n);
      int kp = 0;
      if (lmax > 0.0)
        while (kp < n && s.lam[n - 1 - kp] >= t2 * lmax) ++kp;
      s.kp = kp;
      s.ub = (lmax > 0.0 && kp < n) ? std::sqrt(2.0 * t2 * lmax) : 0.0;
      if (pass == 1) {
        s.vb = G;
        s.vo = ep.goff[q] + (long)(np - n) * np;
        s.vs = np;
      } else {
        s.vb = Tp;
        s.vo = tpo[q];
        s.vs = tm.nr[q];
      }
      for (int i = 0; i < kp; ++i) out.s[q].push_back(std::sqrt(s.lam[n - 1 - i]));
      if (kp > 0) out.vecs[q].push_back(TruncVecSeg{s.vb, s.vo + (long)(n - 1) * s.vs, -s.vs, kp});
      if (pass == 1 && kp > 0) s0 = std::max(s0, out.s[q][0]);
    }
    if (!(out.total > 0.0) || !std::isfinite(out.total)) return;
    // ---- which unresolved tails could still be kept
    const double cut = eps * s0;
    std::vector<double> acc;
    for (int q = 0; q < Q; ++q)
      for (double v : out.s[q])
        if (v > cut) acc.push_back(v);
    double thr = cut;
    if ((long)acc.size() >= (long)kmax && kmax > 0) {
      std::nth_element(acc.begin(), acc.begin() + (kmax - 1), acc.end(), std::greater<double>());
      thr = std::max(thr, acc[kmax - 1]);
    }
    std::vector<int> refine(Q, 0);
    bool any = false;
    for (int q = 0; q < Q; ++q)
      if (nsolve[q] && st[q].ub > thr && st[q].kp < st[q].n && pass < kMaxPass) {
        refine[q] = 1;
        any = true;
      }
    // values left unresolved are reported as they are
    for (int q = 0; q < Q; ++q)
      if (nsolve[q] && !refine[q])
        for (int j = 0; j < st[q].n - st[q].kp; ++j) out.rest[q].push_back(std::sqrt(st[q].lam[j]));
    if (!any) break;
    // ---- deflated tail coefficients of the refined matrices
    //   W = Y_real^T Z (n x nc): the last kp rows are the accepted right
    //   directions (norm s_i), the first n - kp the tail coefficients
    long wtot = 0, ptot = 0;
    std::vector<long> wo(Q, 0), po(Q, 0);
    for (int q = 0; q < Q; ++q)
      if (refine[q]) {
        wo[q] = wtot;
        wtot += (long)st[q].n * tm.nc[q];
        po[q] = ptot;
        ptot += (long)(st[q].n - st[q].kp) * st[q].kp;
      }
    double* W = (double*)ws_get(c, (pass & 1) ? WS_TR_W0 : WS_TR_W1, sizeof(double) * (size_t)std::max(wtot, 1L));
    double* P = (double*)ws_get(c, WS_TR_P, sizeof(double) * (size_t)std::max(ptot, 1L));
    {
      std::vector<MTask> ts;
      const double* zb = nullptr;
      for (int q = 0; q < Q; ++q)
        if (refine[q]) {
          const int n = st[q].n, np = ep.npad[q];
          ts.push_back(MTask{n, tm.nc[q], n, ep.goff[q] + (long)(np - n) * np, (long)np, st[q].zo, st[q].zl,
                             wo[q], (long)tm.nc[q]});
          zb = st[q].zb;
        }
      multi_gemm(c, ts, true, false, G, zb, W, 1.0, 0.0);
    }
    // normalise the accepted right directions
    {
      std::vector<RowScale> rs;
      std::vector<double> f;
      for (int q = 0; q < Q; ++q)
        if (refine[q]) {
          const int n = st[q].n, kp = st[q].kp, nt = n - kp;
          rs.push_back(RowScale{wo[q] + (long)nt * tm.nc[q], (long)tm.nc[q], kp, tm.nc[q], (long)f.size()});
          for (int i = 0; i < kp; ++i) f.push_back(1.0 / std::sqrt(st[q].lam[nt + i]));
        }
      const size_t db = (sizeof(RowScale) * rs.size() + 255) & ~(size_t)255;
      char* aux = (char*)ws_get(c, WS_TR_AUX, db + sizeof(double) * f.size());
      D3S_HIP(hipMemcpyAsync(aux, rs.data(), sizeof(RowScale) * rs.size(), hipMemcpyHostToDevice, c->stream));
      D3S_HIP(hipMemcpyAsync(aux + db, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, c->stream));
      long maxel = 1;
      for (const RowScale& r : rs) maxel = std::max(maxel, (long)r.rows * r.cols);
      const unsigned gx = (unsigned)std::min<long>((maxel + kThr - 1) / kThr, 1024);
      hipLaunchKernelGGL(scale_rows_kernel, dim3(gx, (unsigned)rs.size()), dim3(kThr), 0, c->stream, W,
                         (const double*)(aux + db), (const RowScale*)aux);
      D3S_HIP(hipGetLastError());
      D3S_HIP(hipStreamSynchronize(c->stream));   // the host tables go out of scope
    }
    //   P = W_t V^T, then W_t -= P V
    {
      std::vector<MTask> tp, td;
      for (int q = 0; q < Q; ++q)
        if (refine[q]) {
          const int n = st[q].n, kp = st[q].kp, nt = n - kp, nc = tm.nc[q];
          const long vo = wo[q] + (long)nt * nc;
          tp.push_back(MTask{nt, kp, nc, wo[q], (long)nc, vo, (long)nc, po[q], (long)kp});
          td.push_back(MTask{nt, nc, kp, po[q], (long)kp, vo, (long)nc, wo[q], (long)nc});
        }
      multi_gemm(c, tp, true, true, W, W, P, 1.0, 0.0);
      multi_gemm(c, td, true, false, P, W, W, -1.0, 1.0);
    }
    // ---- next pass: the tail rows of W and of this pass's vectors
    for (int q = 0; q < Q; ++q) {
      solve[q] = refine[q];
      if (!refine[q]) continue;
      St& s = st[q];
      const int nt = s.n - s.kp;
      s.zb = W;
      s.zo = wo[q];
      s.zl = tm.nc[q];
      s.tb = s.vb;
      s.to = s.vo;
      s.tl = s.vs;
      s.n = nt;
    }
  }
  // ---- global selection: at most kmax, only s > eps * s_0; the kept states
  // of a matrix are a prefix of its accepted list
  const double cut = eps * s0;
  struct Cand { double v; int q, i; };
  std::vector<Cand> cand;
  for (int q = 0; q < Q; ++q)
    for (int i = 0; i < (int)out.s[q].size(); ++i)
      if (out.s[q][i] > cut) cand.push_back(Cand{out.s[q][i], q, i});
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.v > b.v; });
  const int k = (int)std::min<long>((long)cand.size(), (long)std::max(kmax, 0));
  for (int i = 0; i < k; ++i) out.keep[cand[i].q]++;
  out.k = k;
  out.kept = 0.0;
  for (int q = 0; q < Q; ++q)
    for (int i = 0; i < out.keep[q]; ++i) out.kept += out.s[q][i] * out.s[q][i];
}

void scale_rows_f64(Ctx* c, double* X, long ld, int rows, int cols, const std::vector<double>& f) {
  if (rows <= 0 || cols <= 0) return;
  const RowScale rs{0, ld, rows, cols, 0};
  const size_t db = 256;
  char* aux = (char*)ws_get(c, WS_TR_AUX, db + sizeof(double) * (size_t)rows);
  D3S_HIP(hipMemcpyAsync(aux, &rs, sizeof(RowScale), hipMemcpyHostToDevice, c->stream));
  D3S_HIP(hipMemcpyAsync(aux + db, f.data(), sizeof(double) * (size_t)rows, hipMemcpyHostToDevice, c->stream));
  const long el = (long)rows * cols;
  const unsigned gx = (unsigned)std::min<long>((el + kThr - 1) / kThr, 1024);
  hipLaunchKernelGGL(scale_rows_kernel, dim3(gx, 1), dim3(kThr), 0, c->stream, X, (const double*)(aux + db),
                     (const RowScale*)aux);
  D3S_HIP(hipGetLastError());
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void kept_copies(const TruncSel& sel, int q, int e0, int ne, long dst_off, long dst_js, long dst_es,
                 std::map<const double*, std::vector<CopyDesc>>& out) {
  int j = 0;
  for (const TruncVecSeg& seg : sel.vecs[q]) {
    if (j >= sel.keep[q]) break;
    const int cnt = std::min(seg.count, sel.keep[q] - j);
    out[seg.base].push_back(CopyDesc{seg.start + e0, seg.step, 1, dst_off + (long)j * dst_js, dst_js, dst_es, cnt,
                                     ne});
    j += cnt;
  }
}

void run_copies(Ctx* c, const std::map<const double*, std::vector<CopyDesc>>& cp, double* dst) {
  for (const auto& kv : cp) copy_blocks(c, kv.first, dst, kv.second);
}

}  // namespace d3s
