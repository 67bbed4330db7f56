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
#include <cstring>
#include <cfloat>
#include <chrono>
#include <cmath>
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

// Tile size (measured on MI355X with the sectors of a 4096-state cylinder
// bond, ~45 sectors: 64x64 tiles beat 96x96 and 128x128 in FP64 and FP32,
// their smaller register footprint keeping more waves in flight): 64x64 by
// default, 128x128 only when the blocks nearly fill them, 32x32 when 64x64
// tiles would be more than half empty.  BF16: the 8-wave 128x128 tile beats
// 64x64 by 14 % at that site, where 128x128 tiles cover at most ~40 % more
// area than 64x64 ones; at half the bond 64x64 wins.  The autotuner, when
// on, times all six.
int grouped_pick_cfg(const Ctx* c, const GroupedPlan& g, d3s_prec p) {
  if (c->grouped_cfg >= 0) return c->grouped_cfg;
  long t64 = 0, t128 = 0;
  double a32 = 0.0, a64 = 0.0;
  for (const GTask& t : g.tasks) {
    t64 += (long)((t.M + 63) / 64) * ((t.N + 63) / 64);
    t128 += (long)((t.M + 127) / 128) * ((t.N + 127) / 128);
    a32 += 1024.0 * ((t.M + 31) / 32) * ((t.N + 31) / 32);
    a64 += 4096.0 * ((t.M + 63) / 64) * ((t.N + 63) / 64);
  }
  if (p == D3S_BF16 && t128 >= 256 && 4 * t128 <= t64 + (2 * t64) / 5) return 4;
  if (t128 >= 512 && 4 * t128 <= t64 + t64 / 4) return 0;
  if (a64 > 2.0 * a32) return 3;
  return 1;
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
  g.cfg = grouped_pick_cfg(c, g, c->tune_prec);
  g.ntasks = (int)g.tasks.size();
  grouped_release(g);
  if (g.ntasks == 0) return;
  // low-precision launches load whole 16-byte chunks: every offset and
  // leading dimension, and the extent that is cut into chunks (K of a
  // K-contiguous operand, else its row or column count), a multiple of the
  // chunk's element count
  auto chunked = [&](long ve) {
    for (const GTask& t : g.tasks)
      for (int q = t.seg0; q < t.seg0 + t.nseg; ++q) {
        const GSeg& sg = g.segs[q];
        if (sg.a_off % ve || sg.lda % ve || sg.b_off % ve || sg.ldb % ve) return false;
        if ((g.a_kc ? sg.K : t.M) % ve || (g.b_kc ? sg.K : t.N) % ve) return false;
      }
    return true;
  };
  g.chunked32 = chunked(4);
  g.chunked16 = chunked(8);
  // the grouped kernel addresses a tile's chunks by 32-bit byte offsets
  for (const GSeg& sg : g.segs)
    if (std::max(sg.lda, sg.ldb) > ((1L << 31) - (1L << 20)) / (256 * 8))
      throw Error{D3S_EINVAL, "grouped GEMM: leading dimension above 2^20 elements"};
  // one allocation: tasks, segments and the tile -> task table, the latter
  // sized for the configuration with the most tiles (the autotuner may
  // switch configurations)
  g.tile_cap = 1;
  for (int cfg = 0; cfg <= 5; ++cfg) {
    int bm, bn;
    grouped_tile_dims(cfg, bm, bn);
    long n = 0;
    for (const GTask& t : g.tasks) n += (long)((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
    g.tile_cap = std::max(g.tile_cap, n);
  }
  if (g.tile_cap > (1L << 30)) throw Error{D3S_EINVAL, "grouped GEMM: too many tiles"};
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t tb = up(sizeof(GTask) * g.tasks.size()), sb = up(sizeof(GSeg) * std::max<size_t>(1, g.segs.size()));
  const size_t bytes = tb + sb + sizeof(int) * (size_t)g.tile_cap;
  char* base;
  if (g.table_slot >= 0) {
    base = (char*)ws_get(c, g.table_slot, bytes);      // a short-lived plan: not owned
  } else {
    g.owner = c;
    base = (char*)dev_alloc(c, bytes);
  }
  g.d_tasks = (GTask*)base;
  g.d_segs = (GSeg*)(base + tb);
  g.d_tile = (int*)(base + tb + sb);
  if (!g.segs.empty())
    D3S_HIP(hipMemcpyAsync(g.d_segs, g.segs.data(), sizeof(GSeg) * g.segs.size(), hipMemcpyHostToDevice,
                           c->stream));
  grouped_retile(c, g);
}

void grouped_retile(Ctx* c, GroupedPlan& g) {
  int bm, bn;
  grouped_tile_dims(g.cfg, bm, bn);
  // tiles are dispatched in table order; a task's tiles cost about its
  // summed K, so the tasks go longest first (the short tiles fill the tail)
  std::vector<long> klen(g.tasks.size(), 0);
  for (size_t k = 0; k < g.tasks.size(); ++k)
    for (int q = 0; q < g.tasks[k].nseg; ++q) klen[k] += g.segs[(size_t)g.tasks[k].seg0 + q].K;
  std::vector<int> ord(g.tasks.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return klen[a] > klen[b]; });
  int acc = 0;
  for (int k : ord) {
    GTask& t = g.tasks[k];
    t.tile0 = acc;
    acc += ((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
  }
  g.total_tiles = acc;
  if (g.ntasks == 0 || !g.d_tasks) return;
  if (acc > g.tile_cap) throw Error{D3S_EDEVICE, "grouped GEMM: tile table too small"};
  std::vector<int> tt((size_t)acc);
  for (int k = 0; k < g.ntasks; ++k) {
    const GTask& t = g.tasks[k];
    const int n = ((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
    for (int q = 0; q < n; ++q) tt[(size_t)t.tile0 + q] = k;
  }
  D3S_HIP(hipMemcpyAsync(g.d_tasks, g.tasks.data(), sizeof(GTask) * g.tasks.size(), hipMemcpyHostToDevice,
                         c->stream));
  if (acc > 0)
    D3S_HIP(hipMemcpyAsync(g.d_tile, tt.data(), sizeof(int) * (size_t)acc, hipMemcpyHostToDevice, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void grouped_release(GroupedPlan& g) {
  if (g.table_slot < 0) dev_free(g.owner, g.d_tasks);
  g.d_tasks = nullptr;
  g.d_segs = nullptr;
  g.d_tile = nullptr;
  g.tile_cap = 0;
}

namespace {

// offset and row stride of the psi block (i, t) whose right sector is j
long psi_off(const BlockHeff& h, int i, int t, int j) {
  return h.packed ? h.poff[(size_t)i * h.d + t] : ((long)h.left.off[i] * h.d + t) * h.mr + h.right.off[j];
}
long psi_ld(const BlockHeff& h, int j) { return h.packed ? (long)h.right.dim[j] : (long)h.d * h.mr; }

// block (i, c, ip) of an environment on the left bond (L, or the new R of a
// right-to-left update) / on the right bond (R, or the new L)
long envl_off(const BlockHeff& h, int i, int c, int ip) {
  return h.penv ? h.epl.off[(size_t)i * h.wl + c] : ((long)h.left.off[i] * h.wl + c) * h.ml + h.left.off[ip];
}
long envl_ld(const BlockHeff& h, int ip) { return h.penv ? (long)h.left.dim[ip] : (long)h.wl * h.ml; }
long envr_off(const BlockHeff& h, int j, int c, int jp) {
  return h.penv ? h.epr.off[(size_t)j * h.wr + c] : ((long)h.right.off[j] * h.wr + c) * h.mr + h.right.off[jp];
}
long envr_ld(const BlockHeff& h, int jp) { return h.penv ? (long)h.right.dim[jp] : (long)h.wr * h.mr; }

const int* qv(const std::vector<int>& q, int i, int nq) { return q.data() + (size_t)i * nq; }

// right sector of q_i + q_t (or -1)
int right_of(const BlockHeff& h, int i, int t) {
  const int nq = h.left.nq;
  int qq[4];
  for (int k = 0; k < nq; ++k) qq[k] = h.left.q[(size_t)i * nq + k] + h.pq[t * nq + k];
  return h.right.find(qq);
}

// W-map tasks of a left-to-right contraction: input T1[a,w,t,y] (rows a of
// length wl*d*mr), outputs the pairs (s,v) at out_base + s*out_ss + v*mr in
// rows of length out_rs.
void build_wmap_l2r(const BlockHeff& h, WmapPlan& wm, long out_base, long out_ss, long out_rs) {
  const Sectors &L = h.left, &R = h.right;
  const int nq = L.nq, d = h.d, wl = h.wl, wr = h.wr, mr = h.mr;
  wm = WmapPlan();
  wm.in_rs = (long)wl * d * mr;
  wm.out_rs = out_rs;
  std::vector<WmapEnt> ins, outs;
  int qq[4];
  for (int i = 0; i < L.n; ++i)
    for (int j = 0; j < R.n; ++j) {
      ins.clear();
      outs.clear();
      for (int w = 0; w < wl; ++w) {
        for (int k = 0; k < nq; ++k) qq[k] = L.q[(size_t)i * nq + k] - h.wql[w * nq + k];
        if (L.find(qq) < 0) continue;     // the first GEMM writes no T1 block for this w
        for (int t = 0; t < d; ++t) {
          bool ok = true;
          for (int k = 0; k < nq; ++k) ok = ok && (qq[k] + h.pq[t * nq + k] == R.q[(size_t)j * nq + k]);
          if (ok) ins.push_back(WmapEnt{(long)(w * d + t) * mr, w * wr * d * d + t, 0});
        }
      }
      for (int sg = 0; sg < d; ++sg)
        for (int v = 0; v < wr; ++v) {
          bool ok = true;
          for (int k = 0; k < nq; ++k)
            ok = ok && (L.q[(size_t)i * nq + k] + h.pq[sg * nq + k] == R.q[(size_t)j * nq + k] + h.wqr[v * nq + k]);
          if (ok) outs.push_back(WmapEnt{out_base + (long)sg * out_ss + (long)v * mr, v * d * d + sg * d, 0});
        }
      wmap_add(wm, L.off[i], L.dim[i], R.off[j], R.dim[j], ins, outs);
    }
}

// W-map tasks of a right-to-left contraction: input Y[x,t,v,b] (rows x of
// length d*wr*mr), outputs the pairs (w,s) at out_base + w*out_ws + s*mr in
// rows of length d*mr.
void build_wmap_r2l(const BlockHeff& h, WmapPlan& wm, long out_base, long out_ws) {
  const Sectors &L = h.left, &R = h.right;
  const int nq = L.nq, d = h.d, wl = h.wl, wr = h.wr, mr = h.mr;
  wm = WmapPlan();
  wm.in_rs = (long)d * wr * mr;
  wm.out_rs = (long)d * mr;
  std::vector<WmapEnt> ins, outs;
  for (int i = 0; i < L.n; ++i)
    for (int j = 0; j < R.n; ++j) {
      ins.clear();
      outs.clear();
      for (int t = 0; t < d; ++t) {
        const int jp = right_of(h, i, t);      // sector of y
        if (jp < 0) continue;
        for (int v = 0; v < wr; ++v) {
          bool ok = true;
          for (int k = 0; k < nq; ++k)
            ok = ok && (R.q[(size_t)jp * nq + k] + h.wqr[v * nq + k] == R.q[(size_t)j * nq + k]);
          if (ok) ins.push_back(WmapEnt{(long)(t * wr + v) * mr, v * d * d + t, 0});
        }
      }
      for (int w = 0; w < wl; ++w)
        for (int sg = 0; sg < d; ++sg) {
          bool ok = true;
          for (int k = 0; k < nq; ++k)
            ok = ok && (L.q[(size_t)i * nq + k] + h.wql[w * nq + k] + h.pq[sg * nq + k] == R.q[(size_t)j * nq + k]);
          if (ok) outs.push_back(WmapEnt{out_base + (long)w * out_ws + (long)sg * mr, w * wr * d * d + sg * d, 0});
        }
      wmap_add(wm, L.off[i], L.dim[i], R.off[j], R.dim[j], ins, outs);
    }
}

// time the tile configurations on zeroed operands of the launch's extents
// (in c->tune_prec)
void retune(Ctx* c, GroupedPlan& g) {
  const size_t na = g.tune_n[0], nb = g.tune_n[1], nc = g.tune_n[2];
  if (!c->autotune || g.ntasks == 0 || na + nb + nc == 0) return;
  double* s = (double*)ws_get(c, WS_TUNE, sizeof(double) * (na + nb + nc));
  zero_bytes(c, s, sizeof(double) * (na + nb + nc));
  tune_grouped(c, g, s, s + na, s + na + nb);
}

void finalize_and_tune(Ctx* c, GroupedPlan& g, size_t na, size_t nb, size_t nc) {
  grouped_finalize(c, g);
  g.tune_n[0] = na;
  g.tune_n[1] = nb;
  g.tune_n[2] = nc;
  retune(c, g);
}

}  // namespace

void wmap_add(WmapPlan& w, int i_off, int di, int j_off, int dj, const std::vector<WmapEnt>& ins,
              const std::vector<WmapEnt>& outs) {
  if (outs.empty() || di <= 0 || dj <= 0) return;
  WmapTask t;
  t.i_off = i_off;
  t.di = di;
  t.j_off = j_off;
  t.dj = dj;
  t.nin = (int)ins.size();
  t.nout = (int)outs.size();
  t.idx0 = (int)w.ents.size();
  t.chunk0 = w.chunks;
  w.chunks += (int)(((long)di * dj + kWmapChunk - 1) / kWmapChunk);
  w.ents.insert(w.ents.end(), ins.begin(), ins.end());
  w.ents.insert(w.ents.end(), outs.begin(), outs.end());
  w.maxk = std::max(w.maxk, std::max(t.nin, t.nout));
  w.tasks.push_back(t);
}

void wmap_upload(Ctx* c, WmapPlan& w) {
  wmap_release(w);
  if (w.maxk > 80) throw Error{D3S_EINVAL, "block W-map: more than 80 channel pairs per block"};
  if (w.tasks.empty()) return;
  // four consecutive elements of a row per thread where every start and
  // length is a multiple of 4 (the padded twin's tables)
  w.vec4 = (w.in_rs % 4 == 0) && (w.out_rs % 4 == 0);
  for (const WmapTask& k : w.tasks) w.vec4 = w.vec4 && (k.j_off % 4 == 0) && (k.dj % 4 == 0);
  for (const WmapEnt& e : w.ents) w.vec4 = w.vec4 && (e.off % 4 == 0);
  // tasks, entries and the chunk -> task table in one allocation, one copy
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bt = up(sizeof(WmapTask) * w.tasks.size()), be = up(sizeof(WmapEnt) * w.ents.size());
  const size_t bc = up(sizeof(int) * (size_t)w.chunks);
  std::vector<unsigned char> host(bt + be + bc, 0);
  std::memcpy(host.data(), w.tasks.data(), sizeof(WmapTask) * w.tasks.size());
  if (!w.ents.empty()) std::memcpy(host.data() + bt, w.ents.data(), sizeof(WmapEnt) * w.ents.size());
  int* ct = reinterpret_cast<int*>(host.data() + bt + be);
  for (size_t t = 0; t < w.tasks.size(); ++t) {
    const WmapTask& k = w.tasks[t];
    const int n = (int)(((long)k.di * k.dj + kWmapChunk - 1) / kWmapChunk);
    for (int q = 0; q < n; ++q) ct[(size_t)k.chunk0 + q] = (int)t;
  }
  w.owner = c;
  unsigned char* base = (unsigned char*)dev_alloc(c, host.size());
  w.d_tasks = reinterpret_cast<WmapTask*>(base);
  w.d_ents = reinterpret_cast<WmapEnt*>(base + bt);
  w.d_ctask = reinterpret_cast<int*>(base + bt + be);
  D3S_HIP(hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
}

void wmap_release(WmapPlan& w) {
  // one allocation holds the tasks, the entries and the chunk table
  dev_free(w.owner, w.d_tasks);
  w.d_tasks = nullptr;
  w.d_ents = nullptr;
  w.d_ctask = nullptr;
}

EnvPack build_envpack(const Sectors& s, const int* wq, int w) {
  EnvPack e;
  const int nq = s.nq;
  e.off.assign((size_t)s.n * w, -1);
  int qq[4];
  for (int i = 0; i < s.n; ++i)
    for (int c = 0; c < w; ++c) {
      for (int k = 0; k < nq; ++k) qq[k] = s.q[(size_t)i * nq + k] - wq[c * nq + k];
      const int ip = s.find(qq);
      if (ip < 0) continue;
      e.off[(size_t)i * w + c] = e.total;
      e.total += (long)s.dim[i] * s.dim[ip];
    }
  return e;
}

void build_block_heff(Ctx* c, BlockHeff& h, const Sectors& left, const Sectors& right, int d, int wl, int wr,
                      const int* pq, const int* wql, const int* wqr, bool packed, bool with_g2, bool packed_env,
                      bool with_psit) {
  const int nq = left.nq;
  if (nq < 1 || nq > 4) throw Error{D3S_EINVAL, "blocks: 1 to 4 charges per state"};
  const int ml = left.total, mr = right.total;
  h.owner = c;
  h.left = left;
  h.right = right;
  h.ml = ml;
  h.mr = mr;
  h.d = d;
  h.wl = wl;
  h.wr = wr;
  h.pq.assign(pq, pq + (size_t)d * nq);
  h.wql.assign(wql, wql + (size_t)wl * nq);
  h.wqr.assign(wqr, wqr + (size_t)wr * nq);
  h.packed = packed;
  h.penv = packed_env;
  if (packed_env) {
    h.epl = build_envpack(left, wql, wl);
    h.epr = build_envpack(right, wqr, wr);
  } else {
    h.epl = EnvPack();
    h.epr = EnvPack();
  }
  h.poff.assign((size_t)left.n * d, -1);
  h.npacked = 0;
  for (int i = 0; i < left.n; ++i)
    for (int t = 0; t < d; ++t) {
      const int j = right_of(h, i, t);
      if (j < 0) continue;
      h.poff[(size_t)i * d + t] = h.npacked;
      h.npacked += (long)left.dim[i] * right.dim[j];
    }
  h.g1 = GroupedPlan();
  h.g1t = GroupedPlan();
  h.g2 = GroupedPlan();
  int qq[4];
  // GEMM-1: T1[(a,w),(t,y)] = sum_x L[(a,w),x] psi[x,(t,y)]; g1t reads the
  // block-transposed psi (block (x-sector, t) at poff, dim_y rows of length dim_x)
  h.g1.a_kc = true;
  h.g1.b_kc = false;
  h.g1t.a_kc = true;
  h.g1t.b_kc = true;
  for (int i = 0; i < left.n; ++i)
    for (int w = 0; w < wl; ++w) {
      for (int k = 0; k < nq; ++k) qq[k] = left.q[(size_t)i * nq + k] - wql[w * nq + k];
      const int ip = left.find(qq);
      if (ip < 0) continue;
      for (int t = 0; t < d; ++t) {
        const int jp = right_of(h, ip, t);
        if (jp < 0) continue;
        GSeg sg;
        sg.K = left.dim[ip];
        sg.a_off = envl_off(h, i, w, ip);
        sg.lda = envl_ld(h, ip);
        sg.b_off = psi_off(h, ip, t, jp);
        sg.ldb = psi_ld(h, jp);
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
        if (!with_psit) continue;
        sg.b_off = h.poff[(size_t)ip * d + t];
        sg.ldb = left.dim[ip];
        h.g1t.segs.push_back(sg);
        h.g1t.tasks.push_back(tk);
      }
    }
  // tiles of the block transpose psi -> psi^T
  if (with_psit) {
    std::vector<TrTile> trt;
    for (int i = 0; i < left.n; ++i)
      for (int t = 0; t < d; ++t) {
        const int j = right_of(h, i, t);
        if (j < 0) continue;
        const long src = psi_off(h, i, t, j), dst = h.poff[(size_t)i * d + t];
        const int R = left.dim[i], C = right.dim[j];
        const int sld = (int)psi_ld(h, j);
        for (int r0 = 0; r0 < R; r0 += 32)
          for (int c0 = 0; c0 < C; c0 += 32)
            trt.push_back(TrTile{src + (long)r0 * sld + c0, dst + (long)c0 * R + r0, sld, R, std::min(32, R - r0),
                                 std::min(32, C - c0)});
      }
    h.ntrt = (int)trt.size();
    if (!trt.empty()) {
      h.d_trt = (TrTile*)dev_alloc(c, sizeof(TrTile) * trt.size());
      D3S_HIP(hipMemcpyAsync(h.d_trt, trt.data(), sizeof(TrTile) * trt.size(), hipMemcpyHostToDevice, c->stream));
      D3S_HIP(hipStreamSynchronize(c->stream));
    }
  }
  // GEMM-2: out[(a,s), b] = sum_{v,y} T2[(a,s),(v,y)] R[b,(v,y)]
  h.g2.a_kc = true;
  h.g2.b_kc = true;
  if (with_g2)
    for (int i = 0; i < left.n; ++i)
      for (int s = 0; s < d; ++s) {
        const int j = right_of(h, i, s);
        if (j < 0) continue;
        GTask tk;
        tk.M = left.dim[i];
        tk.N = right.dim[j];
        tk.seg0 = (int)h.g2.segs.size();
        tk.nseg = 0;
        tk.tile0 = 0;
        tk.c_off = psi_off(h, i, s, j);
        tk.ldc = psi_ld(h, j);
        for (int v = 0; v < wr; ++v) {
          for (int k = 0; k < nq; ++k) qq[k] = right.q[(size_t)j * nq + k] - wqr[v * nq + k];
          const int jpp = right.find(qq);
          if (jpp < 0) continue;
          GSeg sg;
          sg.K = right.dim[jpp];
          sg.a_off = (((long)left.off[i] * d + s) * wr + v) * mr + right.off[jpp];
          sg.lda = (long)d * wr * mr;
          sg.b_off = envr_off(h, j, v, jpp);
          sg.ldb = envr_ld(h, jpp);
          h.g2.segs.push_back(sg);
          tk.nseg++;
        }
        h.g2.tasks.push_back(tk);
      }
  // Split-K of the second GEMM for packed outputs: its tasks (one per output
  // block, K up to w_r blocks long) are few, so when they would not give the
  // device a few thousand tiles each task's channel segments are dealt to
  // up to four sub-tasks writing separate partial outputs, summed afterwards
  // in a fixed order (deterministic).
  h.g2_split = 1;
  if (with_g2 && packed && !h.g2.tasks.empty()) {
    long tiles = 0;
    int maxseg = 1;
    double fl = 0.0;
    for (const GTask& t : h.g2.tasks) {
      tiles += (long)((t.M + 63) / 64) * ((t.N + 63) / 64);
      maxseg = std::max(maxseg, t.nseg);
      for (int q = t.seg0; q < t.seg0 + t.nseg; ++q) fl += 2.0 * t.M * t.N * h.g2.segs[q].K;
    }
    // small products are launch-bound: the extra summation launch would cost more than it saves
    const bool on = c->block_split_gflop >= 0.0 && fl >= c->block_split_gflop * 1e9;
    const int S = !on ? 1 : (int)std::min<long>(std::min(4, maxseg), std::max<long>(1, (4096 + tiles - 1) / tiles));
    if (S > 1) {
      std::vector<GTask> split;
      split.reserve(h.g2.tasks.size() * S);
      for (const GTask& t : h.g2.tasks) {
        const int per = (t.nseg + S - 1) / S;
        for (int j = 0; j < S; ++j) {
          GTask u = t;
          u.seg0 = t.seg0 + std::min(t.nseg, j * per);
          u.nseg = std::max(0, std::min(t.nseg, (j + 1) * per) - std::min(t.nseg, j * per));
          u.c_off = t.c_off + (long)j * h.npacked;
          split.push_back(u);
        }
      }
      h.g2.tasks.swap(split);
      h.g2_split = S;
    }
  }
  build_wmap_l2r(h, h.wm, 0, (long)wr * mr, (long)d * wr * mr);
  wmap_upload(c, h.wm);
  const size_t nL = (size_t)ml * wl * ml, nP = (size_t)ml * d * mr, nR = (size_t)mr * wr * mr;
  const size_t nT = (size_t)ml * std::max(wl, wr) * d * mr;
  finalize_and_tune(c, h.g1, nL, nP, nT);
  if (with_psit) finalize_and_tune(c, h.g1t, nL, nP, nT);
  finalize_and_tune(c, h.g2, nT, nR, nP * h.g2_split);
  // flops of the allowed block products of the two GEMMs (the W-map is not counted)
  h.flops = h.g1.flops + h.g2.flops;
}

namespace {

// tiles of one block: real R x C (row stride sld) -> padded PR x PC (row
// stride dld), zeros in the padding
void add_rl_tiles(std::vector<RlTile>& v, long src, int sld, long dst, int dld, int R, int C, int PR, int PC) {
  for (int r0 = 0; r0 < PR; r0 += 32)
    for (int c0 = 0; c0 < PC; c0 += 32) {
      RlTile t;
      t.prows = std::min(32, PR - r0);
      t.pcols = std::min(32, PC - c0);
      t.rows = std::max(0, std::min(t.prows, R - r0));
      t.cols = std::max(0, std::min(t.pcols, C - c0));
      t.src = (t.rows > 0 && t.cols > 0) ? src + (long)r0 * sld + c0 : 0;
      t.dst = dst + (long)r0 * dld + c0;
      t.src_ld = sld;
      t.dst_ld = dld;
      v.push_back(t);
    }
}

RlTile* upload_rl(Ctx* c, const std::vector<RlTile>& v) {
  if (v.empty()) return nullptr;
  RlTile* d = (RlTile*)dev_alloc(c, sizeof(RlTile) * v.size());
  D3S_HIP(hipMemcpyAsync(d, v.data(), sizeof(RlTile) * v.size(), hipMemcpyHostToDevice, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  return d;
}

Sectors padded_sectors(const Sectors& s) {
  std::vector<int> pd(s.dim);
  for (int& x : pd) x = (x + 7) / 8 * 8;
  return Sectors(s.nq, s.n, s.q.data(), pd.data());
}

}  // namespace

LowpTwin& ensure_lowp(Ctx* c, BlockHeff& h, d3s_prec p) {
  if (h.padded) throw Error{D3S_EINVAL, "blocks: a padded plan has no twin"};
  if (h.lp) {
    // built for the other low precision: its launches get that precision's
    // tile rule, or with the autotuner on are timed again in it
    if (h.lp->prec != p) {
      if (!c->autotune) {
        for (GroupedPlan* g : {&h.lp->h.g1, &h.lp->h.g1t, &h.lp->h.g2}) {
          const int cfg = grouped_pick_cfg(c, *g, p);
          if (g->ntasks > 0 && cfg != g->cfg) {
            g->cfg = cfg;
            grouped_retile(c, *g);
          }
        }
      } else {
        c->tune_prec = p;
        try {
          for (GroupedPlan* g : {&h.lp->h.g1, &h.lp->h.g1t, &h.lp->h.g2}) retune(c, *g);
        } catch (...) {
          c->tune_prec = D3S_F64;
          throw;
        }
        c->tune_prec = D3S_F64;
      }
    }
    h.lp->prec = p;
    return *h.lp;
  }
  LowpTwin* tw = new LowpTwin();
  try {
    const Sectors pl = padded_sectors(h.left), pr = padded_sectors(h.right);
    const int nq = h.left.nq;
    c->tune_prec = p;
    try {
      build_block_heff(c, tw->h, pl, pr, h.d, h.wl, h.wr, h.pq.data(), h.wql.data(), h.wqr.data(), true, true,
                       true, true);
    } catch (...) {
      c->tune_prec = D3S_F64;
      throw;
    }
    c->tune_prec = D3S_F64;
    tw->h.padded = true;
    tw->prec = p;
    const BlockHeff& t = tw->h;
    std::vector<RlTile> vl, vr, vx, vy;
    int qq[4];
    for (int i = 0; i < h.left.n; ++i)
      for (int w = 0; w < h.wl; ++w) {
        for (int k = 0; k < nq; ++k) qq[k] = h.left.q[(size_t)i * nq + k] - h.wql[w * nq + k];
        const int ip = h.left.find(qq);
        if (ip < 0) continue;
        add_rl_tiles(vl, envl_off(h, i, w, ip), (int)envl_ld(h, ip), t.epl.off[(size_t)i * h.wl + w], pl.dim[ip],
                     h.left.dim[i], h.left.dim[ip], pl.dim[i], pl.dim[ip]);
      }
    for (int j = 0; j < h.right.n; ++j)
      for (int v = 0; v < h.wr; ++v) {
        for (int k = 0; k < nq; ++k) qq[k] = h.right.q[(size_t)j * nq + k] - h.wqr[v * nq + k];
        const int jp = h.right.find(qq);
        if (jp < 0) continue;
        add_rl_tiles(vr, envr_off(h, j, v, jp), (int)envr_ld(h, jp), t.epr.off[(size_t)j * h.wr + v], pr.dim[jp],
                     h.right.dim[j], h.right.dim[jp], pr.dim[j], pr.dim[jp]);
      }
    for (int i = 0; i < h.left.n; ++i)
      for (int s = 0; s < h.d; ++s) {
        const int j = right_of(h, i, s);
        if (j < 0) continue;
        const long po = t.poff[(size_t)i * h.d + s];
        add_rl_tiles(vx, psi_off(h, i, s, j), (int)psi_ld(h, j), po, pr.dim[j], h.left.dim[i], h.right.dim[j],
                     pl.dim[i], pr.dim[j]);
        add_rl_tiles(vy, po, pr.dim[j], psi_off(h, i, s, j), (int)psi_ld(h, j), h.left.dim[i], h.right.dim[j],
                     h.left.dim[i], h.right.dim[j]);
      }
    tw->d_L = upload_rl(c, vl);
    tw->d_R = upload_rl(c, vr);
    tw->d_X = upload_rl(c, vx);
    tw->d_Y = upload_rl(c, vy);
    tw->nL = (int)vl.size();
    tw->nR = (int)vr.size();
    tw->nX = (int)vx.size();
    tw->nY = (int)vy.size();
  } catch (...) {
    release_block_heff(tw->h);
    for (RlTile* p : {tw->d_L, tw->d_R, tw->d_X, tw->d_Y}) dev_free(c, p);
    delete tw;
    throw;
  }
  h.lp = tw;
  return *tw;
}

void release_block_heff(BlockHeff& h) {
  if (h.lp) {
    release_block_heff(h.lp->h);
    for (RlTile* p : {h.lp->d_L, h.lp->d_R, h.lp->d_X, h.lp->d_Y}) dev_free(h.owner, p);
    for (void* p : {h.lp->bL, h.lp->bR, h.lp->bW}) dev_free(h.owner, p);
    delete h.lp;
    h.lp = nullptr;
  }
  grouped_release(h.g1);
  grouped_release(h.g1t);
  dev_free(h.owner, h.d_trt);
  h.d_trt = nullptr;
  h.ntrt = 0;
  grouped_release(h.g2);
  grouped_release(h.g_el);
  grouped_release(h.g_y);
  grouped_release(h.g_er);
  wmap_release(h.wm);
  wmap_release(h.wm_x);
  wmap_release(h.wm_yx);
  wmap_release(h.wm_yz);
  h.g_el = GroupedPlan();
  h.g_y = GroupedPlan();
  h.g_er = GroupedPlan();
  h.wm_x = WmapPlan();
  h.wm_yx = WmapPlan();
  h.wm_yz = WmapPlan();
  if (h.graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)h.graph_exec);
  if (h.graph) (void)hipGraphDestroy((hipGraph_t)h.graph);
  if (h.cap_stream) (void)hipStreamDestroy((hipStream_t)h.cap_stream);
  if (h.ev_in) (void)hipEventDestroy((hipEvent_t)h.ev_in);
  if (h.ev_out) (void)hipEventDestroy((hipEvent_t)h.ev_out);
  h.graph_exec = h.graph = h.cap_stream = h.ev_in = h.ev_out = nullptr;
}

namespace {

std::vector<CopyDesc> psi_blocks(const BlockHeff& h, bool to_packed, long rowlen) {
  std::vector<CopyDesc> v;
  const int d = h.d;
  for (int i = 0; i < h.left.n; ++i)
    for (int t = 0; t < d; ++t) {
      const long po = h.poff[(size_t)i * d + t];
      if (po < 0) continue;
      const int j = right_of(h, i, t);
      const long doff = ((long)h.left.off[i] * d + t) * rowlen + h.right.off[j];
      const long drs = (long)d * rowlen, prs = h.right.dim[j];
      if (to_packed) v.push_back(CopyDesc{doff, drs, 1, po, prs, 1, h.left.dim[i], h.right.dim[j]});
      else v.push_back(CopyDesc{po, prs, 1, doff, drs, 1, h.left.dim[i], h.right.dim[j]});
    }
  return v;
}

// Y = psi * R^T over the allowed blocks: Y[(x,t),(v,b)] = sum_y psi[(x,t),y] R[(b,v),y]
void ensure_y(Ctx* c, BlockHeff& h) {
  if (h.g_y.ntasks != 0 || !h.g_y.tasks.empty()) return;
  const Sectors &L = h.left, &R = h.right;
  const int nq = L.nq, d = h.d, wr = h.wr, mr = h.mr;
  GroupedPlan& g = h.g_y;
  g.a_kc = true;
  g.b_kc = true;
  int qq[4];
  for (int i = 0; i < L.n; ++i)
    for (int t = 0; t < d; ++t) {
      const int jp = right_of(h, i, t);
      if (jp < 0) continue;
      for (int v = 0; v < wr; ++v) {
        for (int k = 0; k < nq; ++k) qq[k] = R.q[(size_t)jp * nq + k] + h.wqr[v * nq + k];
        const int j = R.find(qq);
        if (j < 0) continue;
        GSeg sg;
        sg.K = R.dim[jp];
        sg.a_off = psi_off(h, i, t, jp);
        sg.lda = psi_ld(h, jp);
        sg.b_off = envr_off(h, j, v, jp);
        sg.ldb = envr_ld(h, jp);
        GTask tk;
        tk.M = L.dim[i];
        tk.N = R.dim[j];
        tk.seg0 = (int)g.segs.size();
        tk.nseg = 1;
        tk.tile0 = 0;
        tk.c_off = (((long)L.off[i] * d + t) * wr + v) * mr + R.off[j];
        tk.ldc = (long)d * wr * mr;
        g.segs.push_back(sg);
        g.tasks.push_back(tk);
      }
    }
  const size_t nP = (size_t)h.ml * d * mr, nR = (size_t)mr * wr * mr, nY = (size_t)h.ml * d * wr * mr;
  finalize_and_tune(c, g, nP, nR, nY);
  if (g.tasks.empty()) g.ntasks = -1;   // built, nothing to do
}

// L2R environment: Lnew[(b),(v,y)] = sum_{(a,s)} site[(a,s),b] T2[(a,s),(v,y)]
void ensure_env_l2r(Ctx* c, BlockHeff& h) {
  if (h.g_el.ntasks != 0 || !h.g_el.tasks.empty()) return;
  if (h.packed) throw Error{D3S_EINVAL, "blocks: environment updates need a dense-layout plan"};
  const Sectors &L = h.left, &R = h.right;
  const int nq = L.nq, d = h.d, wr = h.wr, mr = h.mr;
  GroupedPlan& g = h.g_el;
  g.a_kc = false;
  g.b_kc = false;
  int qq[4];
  for (int j = 0; j < R.n; ++j)
    for (int v = 0; v < wr; ++v) {
      for (int k = 0; k < nq; ++k) qq[k] = R.q[(size_t)j * nq + k] - h.wqr[v * nq + k];
      const int jpp = R.find(qq);
      if (jpp < 0) continue;
      GTask tk;
      tk.M = R.dim[j];
      tk.N = R.dim[jpp];
      tk.seg0 = (int)g.segs.size();
      tk.nseg = 0;
      tk.tile0 = 0;
      tk.c_off = envr_off(h, j, v, jpp);
      tk.ldc = envr_ld(h, jpp);
      for (int i = 0; i < L.n; ++i)
        for (int s = 0; s < d; ++s) {
          if (right_of(h, i, s) != j) continue;
          GSeg sg;
          sg.K = L.dim[i];
          sg.a_off = ((long)L.off[i] * d + s) * mr + R.off[j];
          sg.lda = (long)d * mr;
          sg.b_off = (((long)L.off[i] * d + s) * wr + v) * mr + R.off[jpp];
          sg.ldb = (long)d * wr * mr;
          g.segs.push_back(sg);
          tk.nseg++;
        }
      if (tk.nseg > 0) g.tasks.push_back(tk);
    }
  const size_t nP = (size_t)h.ml * d * mr, nT = (size_t)h.ml * d * wr * mr, nE = (size_t)mr * wr * mr;
  finalize_and_tune(c, g, nP, nT, nE);
  if (g.tasks.empty()) g.ntasks = -1;
}

// R2L environment: Rnew[a,(w,x)] = sum_{(s,b)} site[a,(s,b)] Z[(w,x),(s,b)]
void ensure_env_r2l(Ctx* c, BlockHeff& h) {
  if (h.g_er.ntasks != 0 || !h.g_er.tasks.empty()) return;
  if (h.packed) throw Error{D3S_EINVAL, "blocks: environment updates need a dense-layout plan"};
  const Sectors& L = h.left;
  const int nq = L.nq, d = h.d, wl = h.wl, ml = h.ml, mr = h.mr;
  build_wmap_r2l(h, h.wm_yz, 0, (long)ml * d * mr);
  wmap_upload(c, h.wm_yz);
  GroupedPlan& g = h.g_er;
  g.a_kc = true;
  g.b_kc = true;
  int qq[4];
  for (int i = 0; i < L.n; ++i)
    for (int w = 0; w < wl; ++w) {
      for (int k = 0; k < nq; ++k) qq[k] = L.q[(size_t)i * nq + k] - h.wql[w * nq + k];
      const int ip = L.find(qq);
      if (ip < 0) continue;
      GTask tk;
      tk.M = L.dim[i];
      tk.N = L.dim[ip];
      tk.seg0 = (int)g.segs.size();
      tk.nseg = 0;
      tk.tile0 = 0;
      tk.c_off = envl_off(h, i, w, ip);
      tk.ldc = envl_ld(h, ip);
      for (int s = 0; s < d; ++s) {
        const int j = right_of(h, i, s);
        if (j < 0) continue;
        GSeg sg;
        sg.K = h.right.dim[j];
        sg.a_off = ((long)L.off[i] * d + s) * mr + h.right.off[j];
        sg.lda = (long)d * mr;
        sg.b_off = (((long)w * ml + L.off[ip]) * d + s) * mr + h.right.off[j];
        sg.ldb = (long)d * mr;
        g.segs.push_back(sg);
        tk.nseg++;
      }
      if (tk.nseg > 0) g.tasks.push_back(tk);
    }
  const size_t nP = (size_t)ml * d * mr, nZ = (size_t)wl * ml * d * mr, nE = (size_t)ml * wl * ml;
  finalize_and_tune(c, g, nP, nZ, nE);
  if (g.tasks.empty()) g.ntasks = -1;
}

}  // namespace

void pack_psi(Ctx* c, const BlockHeff& h, const double* dense, double* packed) {
  if (!h.packed) throw Error{D3S_EINVAL, "blocks: pack needs a packed plan"};
  copy_blocks(c, dense, packed, psi_blocks(h, true, h.mr));
}

void unpack_psi(Ctx* c, const BlockHeff& h, const double* packed, double* dense, long rowlen, bool clear) {
  if (!h.packed) throw Error{D3S_EINVAL, "blocks: unpack needs a packed plan"};
  if (clear) zero_bytes(c, dense, sizeof(double) * (size_t)h.ml * h.d * rowlen);
  copy_blocks(c, packed, dense, psi_blocks(h, false, rowlen));
}

void op_expand_blocks(Ctx* c, BlockHeff& h, d3s_dir dir, const double* env, const double* W, const double* psi,
                      double alpha, double* Mt) {
  const int ml = h.ml, d = h.d, mr = h.mr, wl = h.wl, wr = h.wr;
  if (dir == D3S_L2R) {
    if (h.wm_x.tasks.empty() && !h.wm_x.d_tasks) {
      build_wmap_l2r(h, h.wm_x, mr, (long)(1 + wr) * mr, (long)d * (1 + wr) * mr);
      wmap_upload(c, h.wm_x);
    }
    double* T1 = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * wl * d * mr);
    grouped_gemm(c, D3S_F64, h.g1, env, psi, T1, 1.0);
    const long rowlen = (long)(1 + wr) * mr;
    if (h.packed) {
      unpack_psi(c, h, psi, Mt, rowlen, true);
    } else {
      zero_bytes(c, Mt, sizeof(double) * (size_t)ml * d * rowlen);
      copy2d_f64(c, psi, mr, Mt, rowlen, (long)ml * d, mr);
    }
    wmap_blocks(c, D3S_F64, T1, W, Mt, h.wm_x, alpha);
  } else {
    if (h.wm_yx.tasks.empty() && !h.wm_yx.d_tasks) {
      build_wmap_r2l(h, h.wm_yx, (long)ml * d * mr, (long)ml * d * mr);
      wmap_upload(c, h.wm_yx);
    }
    ensure_y(c, h);
    double* Y = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)ml * d * wr * mr);
    if (h.g_y.ntasks > 0) grouped_gemm(c, D3S_F64, h.g_y, psi, env, Y, 1.0);
    const size_t nrows = (size_t)(1 + wl) * ml;
    if (h.packed) {
      zero_bytes(c, Mt, sizeof(double) * nrows * d * mr);
      unpack_psi(c, h, psi, Mt, mr, false);
    } else {
      zero_bytes(c, Mt + (size_t)ml * d * mr, sizeof(double) * (size_t)wl * ml * d * mr);
      copy_f64(c, psi, Mt, (long)ml * d * mr);
    }
    wmap_blocks(c, D3S_F64, Y, W, Mt, h.wm_yx, alpha);
  }
}

void op_update_env_blocks(Ctx* c, BlockHeff& h, d3s_dir dir, const double* env_in, const double* W,
                          const double* site, double* env_out) {
  const int ml = h.ml, d = h.d, mr = h.mr, wl = h.wl, wr = h.wr;
  if (dir == D3S_L2R) {
    ensure_env_l2r(c, h);
    double* T1 = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)ml * wl * d * mr);
    double* T2 = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)ml * d * wr * mr);
    grouped_gemm(c, D3S_F64, h.g1, env_in, site, T1, 1.0);
    wmap_blocks(c, D3S_F64, T1, W, T2, h.wm, 1.0);
    zero_bytes(c, env_out, sizeof(double) * (size_t)plan_nr(h));
    if (h.g_el.ntasks > 0) grouped_gemm(c, D3S_F64, h.g_el, site, T2, env_out, 1.0);
  } else {
    ensure_y(c, h);
    ensure_env_r2l(c, h);
    double* Y = (double*)ws_get(c, WS_T2, sizeof(double) * (size_t)ml * d * wr * mr);
    double* Z = (double*)ws_get(c, WS_T1, sizeof(double) * (size_t)wl * ml * d * mr);
    if (h.g_y.ntasks > 0) grouped_gemm(c, D3S_F64, h.g_y, site, env_in, Y, 1.0);
    wmap_blocks(c, D3S_F64, Y, W, Z, h.wm_yz, 1.0);
    zero_bytes(c, env_out, sizeof(double) * (size_t)plan_nl(h));
    if (h.g_er.ntasks > 0) grouped_gemm(c, D3S_F64, h.g_er, site, Z, env_out, 1.0);
  }
}

// The launches of one block-sparse H_eff on stream s.
// FP32 / BF16 products run GEMM-1 on the block-transposed psi (psiT, at
// least npacked elements): a K-contiguous operand is staged into LDS with
// 16-byte writes instead of one write per element.
static bool uses_psit(const BlockHeff& h, d3s_prec p) { return p != D3S_F64 && h.ntrt > 0; }

static void enqueue_block_heff(Ctx* c, hipStream_t s, const BlockHeff& h, d3s_prec p, const void* L, const void* W,
                               const void* R, const void* psi, void* out, void* T1, void* T2, void* part,
                               void* psiT) {
  hipStream_t keep = c->stream;
  c->stream = s;
  const size_t osz = (p == D3S_F64) ? 8 : 4;
  // only allowed blocks of T1 / T2 are written and read, so they need no clearing;
  // the output's forbidden blocks are cleared
  if (uses_psit(h, p)) {
    transpose_tiles(c, p == D3S_F64 ? 8 : (p == D3S_F32 ? 4 : 2), psi, psiT, h.d_trt, h.ntrt);
    grouped_gemm(c, p, h.g1t, L, psiT, T1, 1.0);
  } else {
    grouped_gemm(c, p, h.g1, L, psi, T1, 1.0);
  }
  wmap_blocks(c, p, T1, W, T2, h.wm, 1.0);
  // packed outputs have no forbidden entries; dense ones are cleared first
  if (!h.packed) zero_bytes(c, out, osz * (size_t)h.ml * h.d * h.mr);
  if (h.g2_split > 1) {
    grouped_gemm(c, p, h.g2, T2, R, part, 1.0);
    sum_partials(c, p == D3S_F64, part, h.g2_split, h.npacked, out);
  } else {
    grouped_gemm(c, p, h.g2, T2, R, out, 1.0);
  }
  c->stream = keep;
}

void op_apply_heff_blocks(Ctx* c, BlockHeff& h, d3s_prec p, const void* L, const void* W, const void* R,
                          const void* psi, void* out, bool use_graph) {
  if (p != D3S_F64 && !h.padded) {
    // operands of the plan's layouts, in the product's element type: moved
    // into the padded twin's layouts, multiplied there, the product moved back
    LowpTwin& tw = ensure_lowp(c, h, p);
    const int kind = (p == D3S_F32) ? RL_F32 : RL_BF16;
    const size_t esz = (p == D3S_F32) ? 4 : 2;
    void* Lp = ws_get(c, WS_LP_L, esz * (size_t)plan_nl(tw.h));
    void* Rp = ws_get(c, WS_LP_R, esz * (size_t)plan_nr(tw.h));
    void* Xp = ws_get(c, WS_LP_X, esz * (size_t)tw.h.npacked);
    float* Yp = (float*)ws_get(c, WS_LP_Y, 4 * (size_t)tw.h.npacked);
    relayout_tiles(c, kind, kind, L, Lp, tw.d_L, tw.nL);
    relayout_tiles(c, kind, kind, R, Rp, tw.d_R, tw.nR);
    relayout_tiles(c, kind, kind, psi, Xp, tw.d_X, tw.nX);
    op_apply_heff_blocks(c, tw.h, p, Lp, W, Rp, Xp, Yp, use_graph);
    if (!h.packed) zero_bytes(c, out, 4 * (size_t)h.ml * h.d * h.mr);
    relayout_tiles(c, RL_F32, RL_F32, Yp, out, tw.d_Y, tw.nY);
    return;
  }
  const size_t tsz = (p == D3S_F64) ? 8 : 4;
  const size_t t2sz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  void* T1 = ws_get(c, WS_T1, tsz * (size_t)h.ml * h.wl * h.d * h.mr);
  void* T2 = ws_get(c, WS_T2, t2sz * (size_t)h.ml * h.d * h.wr * h.mr);
  void* part = (h.g2_split > 1) ? ws_get(c, WS_G2_PART, tsz * (size_t)h.g2_split * h.npacked) : nullptr;
  void* psiT = uses_psit(h, p) ? ws_get(c, WS_PSIT, t2sz * (size_t)h.npacked) : nullptr;
  if (!use_graph) {
    enqueue_block_heff(c, c->stream, h, p, L, W, R, psi, out, T1, T2, part, psiT);
    return;
  }
  // One hipGraph per (plan, buffers): captured on a private stream on first
  // use, replayed afterwards; events order it after / before the context's
  // stream work.
  const void* key[9] = {L, W, R, psi, out, T1, T2, part, psiT};
  bool same = h.graph_exec != nullptr && h.graph_prec == (int)p;
  for (int i = 0; i < 9 && same; ++i) same = (h.graph_key[i] == key[i]);
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
      enqueue_block_heff(c, cs, h, p, L, W, R, psi, out, T1, T2, part, psiT);
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
    for (int i = 0; i < 9; ++i) h.graph_key[i] = key[i];
    h.graph_prec = (int)p;
  }
  D3S_HIP(hipEventRecord((hipEvent_t)h.ev_in, c->stream));
  D3S_HIP(hipStreamWaitEvent(cs, (hipEvent_t)h.ev_in, 0));
  D3S_HIP(hipGraphLaunch((hipGraphExec_t)h.graph_exec, cs));
  D3S_HIP(hipEventRecord((hipEvent_t)h.ev_out, cs));
  D3S_HIP(hipStreamWaitEvent(c->stream, (hipEvent_t)h.ev_out, 0));
}

void lowp_product(Ctx* c, BlockHeff& h, LowpTwin& tw, d3s_prec p, const void* Lc, const void* Wc, const void* Rc,
                  const double* x, double* y, void* xin, float* yout, bool use_graph) {
  relayout_tiles(c, RL_F64, p == D3S_F32 ? RL_F32 : RL_BF16, x, xin, tw.d_X, tw.nX);
  op_apply_heff_blocks(c, tw.h, p, Lc, Wc, Rc, xin, yout, use_graph);
  // the dense layout's forbidden entries are not written by the relayout
  if (!h.packed) zero_bytes(c, y, sizeof(double) * (size_t)h.ml * h.d * h.mr);
  relayout_tiles(c, RL_F32, RL_F64, yout, y, tw.d_Y, tw.nY);
}

void op_block_bind(Ctx* c, BlockHeff& h, d3s_prec p, const double* L, const double* W, const double* R) {
  if (p != D3S_F32 && p != D3S_BF16) throw Error{D3S_EINVAL, "bind: prec must be D3S_F32 or D3S_BF16"};
  if (h.padded) throw Error{D3S_EINVAL, "blocks: a padded plan has no twin"};
  LowpTwin& tw = ensure_lowp(c, h, p);
  dev_free(h.owner, tw.bL);
  dev_free(h.owner, tw.bR);
  dev_free(h.owner, tw.bW);
  tw.bL = tw.bR = tw.bW = nullptr;
  tw.bprec = D3S_F64;
  const size_t esz = (p == D3S_F32) ? 4 : 2;
  const long nw = (long)h.wl * h.wr * h.d * h.d;
  tw.bL = dev_alloc(c, esz * (size_t)std::max(1L, plan_nl(tw.h)));
  tw.bR = dev_alloc(c, esz * (size_t)std::max(1L, plan_nr(tw.h)));
  tw.bW = dev_alloc(c, sizeof(float) * (size_t)nw);
  // the relayout tiles cover every padded block, padding included (zeros)
  const int kind = (p == D3S_F32) ? RL_F32 : RL_BF16;
  relayout_tiles(c, RL_F64, kind, L, tw.bL, tw.d_L, tw.nL);
  relayout_tiles(c, RL_F64, kind, R, tw.bR, tw.d_R, tw.nR);
  cast_f64_to_f32(c, W, (float*)tw.bW, nw);
  tw.bprec = p;
}

void op_apply_heff_blocks_bound(Ctx* c, BlockHeff& h, const double* psi, double* out, bool use_graph) {
  if (!h.lp || h.lp->bprec == D3S_F64) throw Error{D3S_EINVAL, "no operator bound to the plan"};
  LowpTwin& tw = *h.lp;
  const d3s_prec p = tw.bprec;
  const size_t esz = (p == D3S_F32) ? 4 : 2;
  void* xin = ws_get(c, WS_LP_X, esz * (size_t)tw.h.npacked);
  float* yout = (float*)ws_get(c, WS_LP_Y, 4 * (size_t)tw.h.npacked);
  lowp_product(c, h, tw, p, tw.bL, tw.bW, tw.bR, psi, out, xin, yout, use_graph);
}

}  // namespace d3s

// ============================================================ block sweeps
namespace d3s {

int charge_lkey(const int* q, int nq) { return nq == 1 ? q[0] : q[0] * 32768 + q[1]; }

namespace {

struct RowGroup { long start, stride; int count, local; };
struct ColGroup { long start; int count, local; };
struct SecGroup {
  std::vector<int> q;
  std::vector<RowGroup> rows;
  std::vector<ColGroup> cols;
  int nrows = 0, ncols = 0;
  long xoff = 0;          // offset of the packed X_Q
  int keep = 0, new_off = 0;
};

long budget_of(int l, int d, int mmax, int b) {
  long cap = mmax, left = 1, right = 1;
  for (int i = 0; i < b && left < cap; ++i) left *= d;
  for (int i = 0; i < l - b && right < cap; ++i) right *= d;
  return std::min(cap, std::min(left, right));
}

}  // namespace

TruncBlocksResult op_truncate_blocks(Ctx* c, d3s_dir dir, const Sectors& left, const Sectors& right, int d,
                                     const int* pq, const int* wq_exp, int wexp, long width, const double* Mt,
                                     const double* psi, int kmax, double eps, const double* nbr, long nbr_other,
                                     double* site_out, double* nbr_out, bool renormalize) {
  const int nq = left.nq;
  const int ml = left.total, mr = right.total;
  const long n = (dir == D3S_L2R) ? (long)ml * d : (long)d * mr;     // Gram side
  const long rowlen = (dir == D3S_L2R) ? width : (long)d * mr;
  // ---- sector groups of the truncated bond
  std::vector<SecGroup> groups;
  std::unordered_map<long, int> gidx;
  std::vector<int> qq(nq);
  auto group_of = [&](const int* q) -> SecGroup& {
    long key = 0;
    for (int k = 0; k < nq; ++k) key = key * 2097152L + (q[k] + 1048576);
    auto it = gidx.find(key);
    if (it != gidx.end()) return groups[it->second];
    gidx[key] = (int)groups.size();
    groups.emplace_back();
    groups.back().q.assign(q, q + nq);
    return groups.back();
  };
  if (dir == D3S_L2R) {
    for (int i = 0; i < left.n; ++i)
      for (int s = 0; s < d; ++s) {
        for (int k = 0; k < nq; ++k) qq[k] = left.q[(size_t)i * nq + k] + pq[s * nq + k];
        SecGroup& g = group_of(qq.data());
        g.rows.push_back({(long)left.off[i] * d + s, (long)d, left.dim[i], g.nrows});
        g.nrows += left.dim[i];
      }
    for (SecGroup& g : groups) {
      const int j = right.find(g.q.data());
      if (j >= 0) {
        g.cols.push_back({(long)right.off[j], right.dim[j], g.ncols});
        g.ncols += right.dim[j];
      }
      for (int v = 0; v < wexp; ++v) {
        for (int k = 0; k < nq; ++k) qq[k] = g.q[k] - wq_exp[v * nq + k];
        const int jv = right.find(qq.data());
        if (jv < 0) continue;
        g.cols.push_back({(long)mr + (long)v * mr + right.off[jv], right.dim[jv], g.ncols});
        g.ncols += right.dim[jv];
      }
    }
  } else {
    for (int j = 0; j < right.n; ++j)
      for (int s = 0; s < d; ++s) {
        for (int k = 0; k < nq; ++k) qq[k] = right.q[(size_t)j * nq + k] - pq[s * nq + k];
        SecGroup& g = group_of(qq.data());
        g.cols.push_back({(long)s * mr + right.off[j], right.dim[j], g.ncols});
        g.ncols += right.dim[j];
      }
    for (SecGroup& g : groups) {
      const int i = left.find(g.q.data());
      if (i >= 0) {
        g.rows.push_back({(long)left.off[i], 1L, left.dim[i], g.nrows});
        g.nrows += left.dim[i];
      }
      for (int w = 0; w < wexp; ++w) {
        for (int k = 0; k < nq; ++k) qq[k] = g.q[k] - wq_exp[w * nq + k];
        const int iw = left.find(qq.data());
        if (iw < 0) continue;
        g.rows.push_back({(long)ml + (long)w * ml + left.off[iw], 1L, left.dim[iw], g.nrows});
        g.nrows += left.dim[iw];
      }
    }
  }
  // drop groups without entries; Gram dimension per group
  std::vector<SecGroup> gs;
  for (SecGroup& g : groups)
    if (g.nrows > 0 && g.ncols > 0) gs.push_back(std::move(g));
  if (gs.empty()) throw Error{D3S_ENUMERIC, "truncate: the expanded tensor has no symmetry-allowed block"};
  // ---- pack X_Q with its Gram side as rows (L2R: the (a,s) rows of the
  // sector; R2L: the transpose of its (s,b) columns)
  const bool l2r = (dir == D3S_L2R);
  long xtot = 0;
  std::vector<CopyDesc> gather;
  TruncMats tm;
  for (SecGroup& g : gs) {
    g.xoff = xtot;
    xtot += (long)g.nrows * g.ncols;
    const int nside = l2r ? g.nrows : g.ncols, nother = l2r ? g.ncols : g.nrows;
    tm.xoff.push_back(g.xoff);
    tm.nr.push_back(nside);
    tm.nc.push_back(nother);
    for (const RowGroup& rg : g.rows)
      for (const ColGroup& cg : g.cols) {
        if (l2r)
          gather.push_back(CopyDesc{rg.start * rowlen + cg.start, rg.stride * rowlen, 1,
                                    g.xoff + (long)rg.local * g.ncols + cg.local, (long)g.ncols, 1, rg.count,
                                    cg.count});
        else
          gather.push_back(CopyDesc{rg.start * rowlen + cg.start, rg.stride * rowlen, 1,
                                    g.xoff + (long)cg.local * g.nrows + rg.local, 1, (long)g.nrows, rg.count,
                                    cg.count});
      }
  }
  double* X = (double*)ws_get(c, WS_XPACK, sizeof(double) * (size_t)xtot);
  copy_blocks(c, Mt, X, gather);
  tm.X = X;
  TruncSel sel;
  trunc_solve(c, tm, kmax, eps, sel);
  if (!(sel.total > 0.0) || !std::isfinite(sel.total))
    throw Error{D3S_ENUMERIC, "truncate: the expanded tensor is zero or not finite"};
  const int k = sel.k;
  if (k <= 0) throw Error{D3S_ENUMERIC, "truncate: no singular value above the cutoff"};
  for (size_t gi = 0; gi < gs.size(); ++gi) gs[gi].keep = sel.keep[gi];
  // ---- new bond sectors (ordered by charge key)
  std::vector<int> order;
  for (int gi = 0; gi < (int)gs.size(); ++gi)
    if (gs[gi].keep > 0) order.push_back(gi);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return charge_lkey(gs[a].q.data(), nq) < charge_lkey(gs[b].q.data(), nq);
  });
  TruncBlocksResult res;
  res.k = k;
  res.total = sel.total;
  res.discarded = std::max(0.0, sel.total - sel.kept);
  int off = 0;
  for (int gi : order) {
    gs[gi].new_off = off;
    off += gs[gi].keep;
    res.q.insert(res.q.end(), gs[gi].q.begin(), gs[gi].q.end());
    res.dim.push_back(gs[gi].keep);
  }
  // ---- the new site tensor from the kept vectors of every sector
  std::map<const double*, std::vector<CopyDesc>> scatter;
  if (l2r) {
    zero_bytes(c, site_out, sizeof(double) * (size_t)n * k);
    for (int gi : order) {
      const SecGroup& g = gs[gi];
      for (const RowGroup& rg : g.rows)
        kept_copies(sel, gi, rg.local, rg.count, rg.start * k + g.new_off, 1, rg.stride * k, scatter);
    }
  } else {
    zero_bytes(c, site_out, sizeof(double) * (size_t)k * n);
    for (int gi : order) {
      const SecGroup& g = gs[gi];
      for (const ColGroup& cg : g.cols)
        kept_copies(sel, gi, cg.local, cg.count, (long)g.new_off * n + cg.start, n, 1, scatter);
    }
  }
  run_copies(c, scatter, site_out);
  // ---- neighbour (Sec. 5 step 5).  X = U^T M (L2R) or M U^T (R2L) couples a
  // kept sector only to the old bond's sector of the same charge, so X is
  // block diagonal and both products run sector by sector, one grouped
  // launch each (on the structured layout the dense products would spend
  // nearly all their flops on zero blocks).  X and the neighbour's output
  // are cleared first: blocks no sector writes stay zero.
  GroupedPlan px, pn;
  auto run = [&](GroupedPlan& gp, const double* A, const double* B, double* C) {
    if (gp.tasks.empty()) return;
    gp.table_slot = WS_TR_TAB;
    grouped_finalize(c, gp);
    grouped_gemm(c, D3S_F64, gp, A, B, C, 1.0, 0.0);
    grouped_release(gp);
  };
  if (dir == D3S_L2R) {
    double* Xn = (double*)ws_get(c, WS_X, sizeof(double) * (size_t)k * mr);
    zero_bytes(c, Xn, sizeof(double) * (size_t)k * mr);
    zero_bytes(c, nbr_out, sizeof(double) * (size_t)k * nbr_other);
    // X[new, b] = sum over the sector's (a, s) rows of U[(a, s), new] M[(a, s), b]
    px.a_kc = false;
    px.b_kc = false;
    // nbr_out[new, :] = X[new, b-block] B[b-block, :]
    pn.a_kc = true;
    pn.b_kc = false;
    for (int gi : order) {
      const SecGroup& g = gs[gi];
      const int j = right.find(g.q.data());
      if (j < 0) continue;
      const long oj = right.off[j];
      GTask t{g.keep, right.dim[j], (int)px.segs.size(), 0, 0, (long)g.new_off * mr + oj, (long)mr};
      for (const RowGroup& rg : g.rows) {
        px.segs.push_back(GSeg{rg.count, rg.start * k + g.new_off, rg.stride * k, rg.start * mr + oj, rg.stride * mr});
        ++t.nseg;
      }
      px.tasks.push_back(t);
      pn.tasks.push_back(GTask{g.keep, (int)nbr_other, (int)pn.segs.size(), 1, 0, (long)g.new_off * nbr_other,
                               nbr_other});
      pn.segs.push_back(GSeg{right.dim[j], (long)g.new_off * mr + oj, (long)mr, oj * nbr_other, nbr_other});
    }
    run(px, site_out, psi, Xn);
    run(pn, Xn, nbr, nbr_out);
  } else {
    double* Xn = (double*)ws_get(c, WS_X, sizeof(double) * (size_t)ml * k);
    zero_bytes(c, Xn, sizeof(double) * (size_t)ml * k);
    zero_bytes(c, nbr_out, sizeof(double) * (size_t)nbr_other * k);
    // X[a, new] = sum over the sector's (s, b) columns of M[a, (s, b)] U[new, (s, b)]
    px.a_kc = true;
    px.b_kc = true;
    // nbr_out[:, new] = A[:, a-block] X[a-block, new]
    pn.a_kc = true;
    pn.b_kc = false;
    for (int gi : order) {
      const SecGroup& g = gs[gi];
      const int i = left.find(g.q.data());
      if (i < 0) continue;
      const long oi = left.off[i];
      GTask t{left.dim[i], g.keep, (int)px.segs.size(), 0, 0, oi * k + g.new_off, (long)k};
      for (const ColGroup& cg : g.cols) {
        px.segs.push_back(GSeg{cg.count, oi * n + cg.start, n, (long)g.new_off * n + cg.start, n});
        ++t.nseg;
      }
      px.tasks.push_back(t);
      pn.tasks.push_back(GTask{(int)nbr_other, g.keep, (int)pn.segs.size(), 1, 0, (long)g.new_off, (long)k});
      pn.segs.push_back(GSeg{left.dim[i], oi, (long)ml, oi * k + g.new_off, (long)k});
    }
    run(px, psi, site_out, Xn);
    run(pn, nbr, Xn, nbr_out);
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
  return res;
}

namespace {

std::vector<int> state_keys(const Sectors& s) {
  std::vector<int> k;
  k.reserve(s.total);
  for (int i = 0; i < s.n; ++i)
    for (int r = 0; r < s.dim[i]; ++r) k.push_back(charge_lkey(&s.q[(size_t)i * s.nq], s.nq));
  return k;
}

void mask_to_bonds(Ctx* c, d3s_state* s, SymChain& sym, int i) {
  std::vector<int> ks(s->d);
  for (int t = 0; t < s->d; ++t) ks[t] = charge_lkey(&sym.phys[(size_t)t * sym.nq], sym.nq);
  mask_site(c, s->site[i], s->m[i], s->d, s->m[i + 1], state_keys(sym.bonds[i]), ks, state_keys(sym.bonds[i + 1]));
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void alpha_rule(d3s_sweep_params* p, double lam, double ef, double disc, double total) {
  if (!p->adaptive_alpha) return;
  const double dEO = lam - p->e_before, dET = ef - lam;
  if (disc <= 1e-12 * total) {
  } else if (std::fabs(dEO) < 1e-13 * std::fabs(lam)) {
    p->alpha *= 0.8;
  } else if (dET < 0.3 * std::fabs(dEO)) {
    p->alpha *= 1.25;
  } else {
    p->alpha *= 0.8;
  }
  p->alpha = std::min(1.0, std::max(1e-16, p->alpha));
}

}  // namespace

double op_energy_blocks(Ctx* c, BlockHeff& h, const double* L, const double* W, const double* R,
                        const double* psi) {
  const long n = h.packed ? h.npacked : (long)h.ml * h.d * h.mr;
  if (n <= 0) throw Error{D3S_ENUMERIC, "energy: the site has no symmetry-allowed block"};
  const double* x = psi;
  if (h.packed) {
    double* xp = (double*)ws_get(c, WS_PK, sizeof(double) * (size_t)n);
    pack_psi(c, h, psi, xp);
    x = xp;
  }
  double* hp = (double*)ws_get(c, WS_REF, sizeof(double) * (size_t)n);
  op_apply_heff_blocks(c, h, D3S_F64, L, W, R, x, hp, false);
  double* r = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 512);
  dot_f64(c, x, hp, n, r);
  dot_f64(c, x, x, n, r + 1);
  double v[2];
  D3S_HIP(hipMemcpyAsync(v, r, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  D3S_HIP(hipStreamSynchronize(c->stream));
  if (!(v[1] > 0.0)) throw Error{D3S_ENUMERIC, "energy: zero state"};
  const double e = v[0] / v[1];
  if (!std::isfinite(e)) throw Error{D3S_ENUMERIC, "energy: not finite"};
  return e;
}

namespace {

// plan of site i (bonds i, i+1) of a symmetric chain
// (environments are stored packed by the block sweeps)
void site_plan(Ctx* c, BlockHeff& h, const d3s_state* s, const SymChain& sym, int i, bool packed, bool with_g2) {
  build_block_heff(c, h, sym.bonds[i], sym.bonds[i + 1], s->d, s->w[i], s->w[i + 1], sym.phys.data(),
                   sym.wq[i].data(), sym.wq[i + 1].data(), packed, with_g2, true);
}

// the packed environment an update writes must fit the caller's buffers
void check_env_fits(const SymChain& sym, long need) {
  if (need > sym.env_cap)
    throw Error{D3S_EINVAL, "block sweep: a packed environment needs " + std::to_string(need) +
                                " elements, the environment buffers hold " + std::to_string(sym.env_cap)};
}

// owns a plan for the duration of a scope
struct PlanGuard {
  BlockHeff h;
  ~PlanGuard() { release_block_heff(h); }
};

}  // namespace

double op_prepare_blocks(Ctx* c, d3s_state* s, SymChain& sym, double eps) {
  const int l = s->l, d = s->d;
  for (int i = 0; i < l; ++i) mask_to_bonds(c, s, sym, i);
  const size_t cap = (size_t)s->mmax * d * s->mmax;
  double* tmpS = (double*)ws_get(c, WS_PSI, sizeof(double) * cap);
  double* tmpN = (double*)ws_get(c, WS_NBR, sizeof(double) * cap);
  for (int i = 0; i + 1 < l; ++i) {
    const int ml = s->m[i], mr = s->m[i + 1];
    const long other = (long)d * s->m[i + 2];
    TruncBlocksResult t = op_truncate_blocks(c, D3S_L2R, sym.bonds[i], sym.bonds[i + 1], d, sym.phys.data(), nullptr,
                                             0, mr, s->site[i], s->site[i], (int)budget_of(l, d, s->mmax, i + 1), eps,
                                             s->site[i + 1], other, tmpS, tmpN, false);
    copy_f64(c, tmpS, s->site[i], (long)ml * d * t.k);
    copy_f64(c, tmpN, s->site[i + 1], (long)t.k * other);
    s->m[i + 1] = t.k;
    sym.bonds[i + 1] = Sectors(sym.nq, (int)t.dim.size(), t.q.data(), t.dim.data());
  }
  const long n = (long)s->m[l - 1] * d * s->m[l];
  double* r = (double*)ws_get(c, WS_LZ_COEF, sizeof(double) * 512);
  dot_f64(c, s->site[l - 1], s->site[l - 1], n, r);
  const double nrm2 = read_scalar(c, r);
  if (!(nrm2 > 0.0) || !std::isfinite(nrm2)) throw Error{D3S_ENUMERIC, "prepare: zero state in the target sector"};
  scale_f64(c, s->site[l - 1], n, 1.0 / std::sqrt(nrm2));
  fill_f64(c, s->lenv[0], 1, 1.0);
  fill_f64(c, s->renv[l - 1], 1, 1.0);
  for (int i = 0; i + 1 < l; ++i) {
    PlanGuard e;
    site_plan(c, e.h, s, sym, i, false, false);
    check_env_fits(sym, e.h.epr.total);
    op_update_env_blocks(c, e.h, D3S_L2R, s->lenv[i], s->mpo[i], s->site[i], s->lenv[i + 1]);
  }
  s->center = l - 1;
  PlanGuard last;
  site_plan(c, last.h, s, sym, l - 1, true, true);
  return op_energy_blocks(c, last.h, s->lenv[l - 1], s->mpo[l - 1], s->renv[l - 1], s->site[l - 1]);
}

// One sweep with every contraction block-sparse: the eigensolver works on
// packed vectors with the grouped H_eff (graph-replayed), the expansion
// term and the environments are grouped contractions on the allowed
// blocks, and the plan built for the post-truncation energy of the next
// site is the one its eigensolver uses.
void op_sweep_blocks(Ctx* c, d3s_state* s, SymChain& sym, d3s_sweep_params* p, d3s_sweep_stats* st, bool use_graph) {
  const int mlim = (p->m_limit > 0 && p->m_limit < s->mmax) ? p->m_limit : s->mmax;
  const int l = s->l, d = s->d;
  if (s->center != l - 1) throw Error{D3S_EINVAL, "sweep: the orthogonality centre must be on site l-1"};
  int wmax = 1;
  for (int i = 0; i <= l; ++i) wmax = std::max(wmax, s->w[i]);
  const size_t cap = (size_t)s->mmax * d * s->mmax;
  double* tmpS = (double*)ws_get(c, WS_PSI, sizeof(double) * cap);
  double* tmpN = (double*)ws_get(c, WS_NBR, sizeof(double) * cap);
  double* Mt = (double*)ws_get(c, WS_MT, sizeof(double) * (size_t)(1 + wmax) * cap);
  const double t_start = now_s();
  st->count = 0;
  st->nonconverged = 0;
  double lam = p->e_before;
  PlanGuard cur, nxt;
  site_plan(c, cur.h, s, sym, l - 1, true, true);
  for (int pass = 0; pass < 2; ++pass) {
    const bool r2l = (pass == 0);
    const int i_first = r2l ? l - 1 : 0, i_last = r2l ? 1 : l - 2, step = r2l ? -1 : 1;
    for (int i = i_first; r2l ? (i >= i_last) : (i <= i_last); i += step) {
      d3s_site_record r{};
      r.site = i;
      r.dir = r2l ? D3S_R2L : D3S_L2R;
      r.e_before = p->e_before;
      const int ml = s->m[i], mr = s->m[i + 1], wl = s->w[i], wr = s->w[i + 1];
      const double t0 = now_s();
      double* xp = (double*)ws_get(c, WS_PK, sizeof(double) * (size_t)std::max<long>(1, cur.h.npacked));
      const d3s_prec prec = (cur.h.flops * 1e-9 >= p->mixed_min_gflop) ? p->prec : D3S_F64;
      LanczosResult lz = op_lanczos_blocks(c, prec, cur.h, s->lenv[i], s->mpo[i], s->renv[i], s->site[i],
                                           p->lanczos_tol, p->lanczos_kmax, p->lanczos_max_matvecs, use_graph, xp);
      lam = lz.theta;
      if (!lz.converged) st->nonconverged++;
      const double t1 = now_s();
      TruncBlocksResult t;
      double t2, t3, t4, ef;
      if (r2l) {
        op_expand_blocks(c, cur.h, D3S_R2L, s->renv[i], s->mpo[i], xp, p->alpha, Mt);
        D3S_HIP(hipStreamSynchronize(c->stream));
        t2 = now_s();
        c->stat_eig_s = 0.0;
        c->stat_passes = 0;
        const int mll = s->m[i - 1];
        t = op_truncate_blocks(c, D3S_R2L, sym.bonds[i], sym.bonds[i + 1], d, sym.phys.data(), sym.wq[i].data(), wl,
                               (long)(1 + wl) * ml, Mt, s->site[i], (int)budget_of(l, d, mlim, i), p->eps,
                               s->site[i - 1], (long)mll * d, tmpS, tmpN, true);
        copy_f64(c, tmpS, s->site[i], (long)t.k * d * mr);
        copy_f64(c, tmpN, s->site[i - 1], (long)mll * d * t.k);
        s->m[i] = t.k;
        sym.bonds[i] = Sectors(sym.nq, (int)t.dim.size(), t.q.data(), t.dim.data());
        t3 = now_s();
        r.t_trunc_eig = c->stat_eig_s;
        r.trunc_passes = c->stat_passes;
        {
          PlanGuard e;
          site_plan(c, e.h, s, sym, i, false, false);
          check_env_fits(sym, e.h.epl.total);
          op_update_env_blocks(c, e.h, D3S_R2L, s->renv[i], s->mpo[i], s->site[i], s->renv[i - 1]);
        }
        D3S_HIP(hipStreamSynchronize(c->stream));
        t4 = now_s();
        release_block_heff(nxt.h);
        site_plan(c, nxt.h, s, sym, i - 1, true, true);
        ef = op_energy_blocks(c, nxt.h, s->lenv[i - 1], s->mpo[i - 1], s->renv[i - 1], s->site[i - 1]);
        s->center = i - 1;
      } else {
        op_expand_blocks(c, cur.h, D3S_L2R, s->lenv[i], s->mpo[i], xp, p->alpha, Mt);
        D3S_HIP(hipStreamSynchronize(c->stream));
        t2 = now_s();
        c->stat_eig_s = 0.0;
        c->stat_passes = 0;
        const int mrr = s->m[i + 2];
        t = op_truncate_blocks(c, D3S_L2R, sym.bonds[i], sym.bonds[i + 1], d, sym.phys.data(), sym.wq[i + 1].data(),
                               wr, (long)(1 + wr) * mr, Mt, s->site[i], (int)budget_of(l, d, mlim, i + 1), p->eps,
                               s->site[i + 1], (long)d * mrr, tmpS, tmpN, true);
        copy_f64(c, tmpS, s->site[i], (long)ml * d * t.k);
        copy_f64(c, tmpN, s->site[i + 1], (long)t.k * d * mrr);
        s->m[i + 1] = t.k;
        sym.bonds[i + 1] = Sectors(sym.nq, (int)t.dim.size(), t.q.data(), t.dim.data());
        t3 = now_s();
        r.t_trunc_eig = c->stat_eig_s;
        r.trunc_passes = c->stat_passes;
        {
          PlanGuard e;
          site_plan(c, e.h, s, sym, i, false, false);
          check_env_fits(sym, e.h.epr.total);
          op_update_env_blocks(c, e.h, D3S_L2R, s->lenv[i], s->mpo[i], s->site[i], s->lenv[i + 1]);
        }
        D3S_HIP(hipStreamSynchronize(c->stream));
        t4 = now_s();
        release_block_heff(nxt.h);
        site_plan(c, nxt.h, s, sym, i + 1, true, true);
        ef = op_energy_blocks(c, nxt.h, s->lenv[i + 1], s->mpo[i + 1], s->renv[i + 1], s->site[i + 1]);
        s->center = i + 1;
      }
      std::swap(cur.h, nxt.h);
      const double t5 = now_s();
      r.k = t.k;
      r.matvecs = lz.matvecs;
      r.f64_matvecs = lz.f64_matvecs;
      r.lambda = lam;
      r.e_f = ef;
      r.alpha = p->alpha;
      r.discarded = t.discarded;
      r.t_eig = t1 - t0; r.t_expand = t2 - t1; r.t_trunc = t3 - t2; r.t_env = t4 - t3; r.t_energy = t5 - t4;
      if (st->count < st->capacity) st->records[st->count] = r;
      st->count++;
      alpha_rule(p, lam, ef, t.discarded, t.total);
      p->e_before = ef;
    }
  }
  st->energy = lam;
  st->seconds = now_s() - t_start;
}

}  // namespace d3s
