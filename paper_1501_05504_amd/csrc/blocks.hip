// Abelian (U(1) or U(1)xU(1)) block structure of the H_eff contraction.
//
// Every bond basis is ordered by charge sector, and tensors keep their dense
// row-major layout; a symmetry-allowed block is then a strided sub-matrix.
// With charges q of bond states, q_s of physical states and Delta_w of MPO
// channels (the charge the operators placed so far have added):
//   psi[a,s,b]  allowed iff  q_a + q_s = q_b
//   W[w,v,s,t]  allowed iff  q_s - q_t = Delta_v - Delta_w
//   L[a,w,x]    allowed iff  q_a - q_x = Delta_w      (and R[b,v,y] likewise)
// (the first is the flux rule of a U(1)-symmetric MPS, the others follow from
// it and the definitions of L_i, R_i in Sec. 2).  The three contractions of
// the Sec. 5 ordering become:
//   GEMM-1: one task per (left sector i, channel w, physical t): the block
//           L[i, w, x in i'] (i' fixed by Delta_w) times psi[i', t, j']
//           (j' fixed by q_t), written into T1[(i,w), (t,j')];
//   W-map:  dense over (w, t) (T1 is zero outside the written blocks);
//   GEMM-2: one task per output block out[(i,s), j] with q_i + q_s = q_j,
//           whose K-segments run over the channels v with the right-bond
//           sector j'' = sector(q_j - Delta_v): T2[(i,s),(v,j'')] R[j,v,j''].
// Tasks are the "uneven blocks" of a symmetric DMRG; all of them go into one
// grouped launch per contraction.
#include <algorithm>
#include <unordered_map>

#include "d3s_internal.h"

namespace d3s {

namespace {
long charge_key(const int* q, int nq) {
  long k = 0;
  for (int i = 0; i < nq; ++i) k = k * 2097152L + (long)(q[i] + 1048576);
  return k;
}
}  // namespace

Sectors::Sectors(int nq_, int n_, const int* q_, const int* dim_) : nq(nq_), n(n_) {
  q.assign(q_, q_ + (size_t)n * nq);
  dim.assign(dim_, dim_ + n);
  off.resize(n);
  total = 0;
  for (int i = 0; i < n; ++i) {
    off[i] = total;
    total += dim[i];
    index[charge_key(&q[(size_t)i * nq], nq)] = i;
  }
}

int Sectors::find(const int* charge) const {
  auto it = index.find(charge_key(charge, nq));
  return it == index.end() ? -1 : it->second;
}

void grouped_finalize(Ctx* c, GroupedPlan& g) {
  // largest tasks first (by flops), then tile prefix sums
  std::vector<int> order(g.tasks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  auto work = [&](const GTask& t) {
    long k = 0;
    for (int s = t.seg0; s < t.seg0 + t.nseg; ++s) k += g.segs[s].K;
    return (double)t.M * t.N * (double)k;
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return work(g.tasks[a]) > work(g.tasks[b]); });
  std::vector<GTask> sorted;
  sorted.reserve(order.size());
  g.flops = 0.0;
  for (int i : order) {
    sorted.push_back(g.tasks[i]);
    g.flops += 2.0 * work(g.tasks[i]);
  }
  g.tasks.swap(sorted);
  // 128x128 tiles when the blocks are large enough to fill them
  long t64 = 0, t128 = 0;
  for (const GTask& t : g.tasks) {
    t64 += (long)((t.M + 63) / 64) * ((t.N + 63) / 64);
    t128 += (long)((t.M + 127) / 128) * ((t.N + 127) / 128);
  }
  g.cfg = (t128 >= 512 && 4 * t128 <= t64 + t64 / 4) ? 0 : 1;
  const int tile = grouped_tile(g.cfg);
  int acc = 0;
  for (GTask& t : g.tasks) {
    t.tile0 = acc;
    acc += ((t.M + tile - 1) / tile) * ((t.N + tile - 1) / tile);
  }
  g.total_tiles = acc;
  g.ntasks = (int)g.tasks.size();
  grouped_release(g);
  if (g.ntasks == 0) return;
  D3S_HIP(hipMalloc((void**)&g.d_tasks, sizeof(GTask) * g.tasks.size()));
  D3S_HIP(hipMalloc((void**)&g.d_segs, sizeof(GSeg) * std::max<size_t>(1, g.segs.size())));
  D3S_HIP(hipMemcpyAsync(g.d_tasks, g.tasks.data(), sizeof(GTask) * g.tasks.size(), hipMemcpyHostToDevice,
                         c->stream));
  if (!g.segs.empty())
    D3S_HIP(hipMemcpyAsync(g.d_segs, g.segs.data(), sizeof(GSeg) * g.segs.size(), hipMemcpyHostToDevice,
                           c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void grouped_release(GroupedPlan& g) {
  if (g.d_tasks) (void)hipFree(g.d_tasks);
  if (g.d_segs) (void)hipFree(g.d_segs);
  g.d_tasks = nullptr;
  g.d_segs = nullptr;
}

void build_block_heff(Ctx* c, BlockHeff& h, const Sectors& left, const Sectors& right, int d, int wl, int wr,
                      const int* pq, const int* wql, const int* wqr) {
  const int nq = left.nq;
  const int ml = left.total, mr = right.total;
  h.ml = ml;
  h.mr = mr;
  h.d = d;
  h.wl = wl;
  h.wr = wr;
  h.g1 = GroupedPlan();
  h.g2 = GroupedPlan();
  std::vector<int> qq(nq);
  // GEMM-1: T1[(a,w),(t,y)] = sum_x L[(a,w),x] psi[x,(t,y)]
  h.g1.a_kc = true;
  h.g1.b_kc = false;
  for (int i = 0; i < left.n; ++i)
    for (int w = 0; w < wl; ++w) {
      for (int k = 0; k < nq; ++k) qq[k] = left.q[(size_t)i * nq + k] - wql[w * nq + k];
      const int ip = left.find(qq.data());
      if (ip < 0) continue;
      for (int t = 0; t < d; ++t) {
        for (int k = 0; k < nq; ++k) qq[k] = left.q[(size_t)ip * nq + k] + pq[t * nq + k];
        const int jp = right.find(qq.data());
        if (jp < 0) continue;
        GSeg sg;
        sg.K = left.dim[ip];
        sg.a_off = ((long)left.off[i] * wl + w) * ml + left.off[ip];
        sg.lda = (long)wl * ml;
        sg.b_off = ((long)left.off[ip] * d + t) * mr + right.off[jp];
        sg.ldb = (long)d * mr;
        GTask tk;
        tk.M = left.dim[i];
        tk.N = right.dim[jp];
        tk.seg0 = (int)h.g1.segs.size();
        tk.nseg = 1;
        tk.tile0 = 0;
        tk.c_off = (((long)left.off[i] * wl + w) * d + t) * mr + right.off[jp];
        tk.ldc = (long)wl * d * mr;
        h.g1.segs.push_back(sg);
        h.g1.tasks.push_back(tk);
      }
    }
  // GEMM-2: out[(a,s), b] = sum_{v,y} T2[(a,s),(v,y)] R[b,(v,y)]
  h.g2.a_kc = true;
  h.g2.b_kc = true;
  for (int i = 0; i < left.n; ++i)
    for (int s = 0; s < d; ++s) {
      for (int k = 0; k < nq; ++k) qq[k] = left.q[(size_t)i * nq + k] + pq[s * nq + k];
      const int j = right.find(qq.data());
      if (j < 0) continue;
      GTask tk;
      tk.M = left.dim[i];
      tk.N = right.dim[j];
      tk.seg0 = (int)h.g2.segs.size();
      tk.nseg = 0;
      tk.tile0 = 0;
      tk.c_off = ((long)left.off[i] * d + s) * mr + right.off[j];
      tk.ldc = (long)d * mr;
      for (int v = 0; v < wr; ++v) {
        for (int k = 0; k < nq; ++k) qq[k] = right.q[(size_t)j * nq + k] - wqr[v * nq + k];
        const int jpp = right.find(qq.data());
        if (jpp < 0) continue;
        GSeg sg;
        sg.K = right.dim[jpp];
        sg.a_off = (((long)left.off[i] * d + s) * wr + v) * mr + right.off[jpp];
        sg.lda = (long)d * wr * mr;
        sg.b_off = ((long)right.off[j] * wr + v) * mr + right.off[jpp];
        sg.ldb = (long)wr * mr;
        h.g2.segs.push_back(sg);
        tk.nseg++;
      }
      h.g2.tasks.push_back(tk);
    }
  grouped_finalize(c, h.g1);
  grouped_finalize(c, h.g2);
  // the dense W-map is part of the work; count its flops over the allowed T1 rows only
  h.flops = h.g1.flops + h.g2.flops;
}

void release_block_heff(BlockHeff& h) {
  grouped_release(h.g1);
  grouped_release(h.g2);
  if (h.graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)h.graph_exec);
  if (h.graph) (void)hipGraphDestroy((hipGraph_t)h.graph);
  if (h.cap_stream) (void)hipStreamDestroy((hipStream_t)h.cap_stream);
  if (h.ev_in) (void)hipEventDestroy((hipEvent_t)h.ev_in);
  if (h.ev_out) (void)hipEventDestroy((hipEvent_t)h.ev_out);
  h.graph_exec = h.graph = h.cap_stream = h.ev_in = h.ev_out = nullptr;
}

// The four launches of one block-sparse H_eff on stream s.
static void enqueue_block_heff(Ctx* c, hipStream_t s, const BlockHeff& h, d3s_prec p, const void* L, const void* W,
                               const void* R, const void* psi, void* out, void* T1, void* T2) {
  hipStream_t keep = c->stream;
  c->stream = s;
  const size_t tsz = (p == D3S_F64) ? 8 : 4;
  const size_t osz = (p == D3S_F64) ? 8 : 4;
  zero_bytes(c, T1, tsz * (size_t)h.ml * h.wl * h.d * h.mr);
  grouped_gemm(c, p, h.g1, L, psi, T1, 1.0);
  wmap_l2r(c, p, T1, W, T2, (long)h.wr * h.mr, h.ml, h.d, h.mr, h.wl, h.wr, 1.0);
  zero_bytes(c, out, osz * (size_t)h.ml * h.d * h.mr);
  grouped_gemm(c, p, h.g2, T2, R, out, 1.0);
  c->stream = keep;
}

void op_apply_heff_blocks(Ctx* c, BlockHeff& h, d3s_prec p, const void* L, const void* W, const void* R,
                          const void* psi, void* out, bool use_graph) {
  const size_t tsz = (p == D3S_F64) ? 8 : 4;
  const size_t t2sz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  void* T1 = ws_get(c, WS_T1, tsz * (size_t)h.ml * h.wl * h.d * h.mr);
  void* T2 = ws_get(c, WS_T2, t2sz * (size_t)h.ml * h.d * h.wr * h.mr);
  if (!use_graph) {
    enqueue_block_heff(c, c->stream, h, p, L, W, R, psi, out, T1, T2);
    return;
  }
  // One hipGraph per (plan, buffers): captured on a private stream on first
  // use, replayed afterwards; events order it after / before the context's
  // stream work.
  const void* key[7] = {L, W, R, psi, out, T1, T2};
  bool same = h.graph_exec != nullptr && h.graph_prec == (int)p;
  for (int i = 0; i < 7 && same; ++i) same = (h.graph_key[i] == key[i]);
  if (!h.cap_stream) {
    hipStream_t cs;
    D3S_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    h.cap_stream = cs;
    hipEvent_t e1, e2;
    D3S_HIP(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
    D3S_HIP(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
    h.ev_in = e1;
    h.ev_out = e2;
  }
  hipStream_t cs = (hipStream_t)h.cap_stream;
  if (!same) {
    if (h.graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)h.graph_exec);
    if (h.graph) (void)hipGraphDestroy((hipGraph_t)h.graph);
    h.graph_exec = h.graph = nullptr;
    D3S_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_block_heff(c, cs, h, p, L, W, R, psi, out, T1, T2);
    } catch (...) {
      hipGraph_t g;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipGraph_t g;
    D3S_HIP(hipStreamEndCapture(cs, &g));
    h.graph = g;
    hipGraphExec_t ge;
    D3S_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    h.graph_exec = ge;
    for (int i = 0; i < 7; ++i) h.graph_key[i] = key[i];
    h.graph_prec = (int)p;
  }
  D3S_HIP(hipEventRecord((hipEvent_t)h.ev_in, c->stream));
  D3S_HIP(hipStreamWaitEvent(cs, (hipEvent_t)h.ev_in, 0));
  D3S_HIP(hipGraphLaunch((hipGraphExec_t)h.graph_exec, cs));
  D3S_HIP(hipEventRecord((hipEvent_t)h.ev_out, cs));
  D3S_HIP(hipStreamWaitEvent(c->stream, (hipEvent_t)h.ev_out, 0));
}

}  // namespace d3s
