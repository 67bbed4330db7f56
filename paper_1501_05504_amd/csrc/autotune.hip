// Tile-configuration autotuner (host C++).
//
// Dense GEMMs: on the first product of a given shape class (precision,
// operand layouts, M, N, K, batch) every tile configuration is timed with
// HIP events on the context's stream and the fastest one is kept in the
// context's cache (and appended to an optional on-disk cache file of
// "key cfg" lines, loaded when autotuning is switched on).  Grouped block
// plans: both tile sizes of the grouped launch are timed on scratch buffers
// right after the plan is built (all six tile configurations).  Tuning is skipped while a stream is being
// captured into a graph and for products that accumulate into C (beta != 0).
#include <fstream>
#include <sstream>

#include "d3s_internal.h"

namespace d3s {

namespace {

std::string gemm_key(d3s_prec p, const GemmArgs& g) {
  std::ostringstream o;
  o << "gemm:" << (int)p << ':' << g.a_kc << ':' << g.b_kc << ':' << g.M << ':' << g.N << ':' << g.K << ':'
    << g.batch;
  return o.str();
}

bool capturing(Ctx* c) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return st != hipStreamCaptureStatusNone;
}

template <typename F>
double time_ms(Ctx* c, F&& launch, int reps) {
  hipEvent_t e0, e1;
  D3S_HIP(hipEventCreate(&e0));
  D3S_HIP(hipEventCreate(&e1));
  launch();   // warm-up
  D3S_HIP(hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r) launch();
  D3S_HIP(hipEventRecord(e1, c->stream));
  D3S_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  D3S_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

void remember(Ctx* c, const std::string& key, int cfg) {
  c->tune_cache[key] = cfg;
  if (!c->tune_path.empty()) {
    std::ofstream f(c->tune_path, std::ios::app);
    if (f) f << key << ' ' << cfg << '\n';
  }
}

}  // namespace

void autotune_load(Ctx* c) {
  if (c->tune_path.empty()) return;
  std::ifstream f(c->tune_path);
  std::string key;
  int cfg;
  while (f >> key >> cfg)
    if (cfg >= 0 && cfg <= 5) c->tune_cache[key] = cfg;
}

void tuned_gemm(Ctx* c, d3s_prec p, const GemmArgs& g) {
  if (!c->autotune || c->tile_config >= 0) {
    gemm(c, p, g);
    return;
  }
  const std::string key = gemm_key(p, g);
  auto it = c->tune_cache.find(key);
  int cfg = -1;
  if (it != c->tune_cache.end()) {
    cfg = it->second;
  } else if (g.beta == 0.0 && !capturing(c)) {
    double best = 1e300;
    for (int k = 0; k <= 4; ++k) {
      c->tile_config = k;
      const double ms = time_ms(c, [&] { gemm(c, p, g); }, 3);
      if (ms < best) {
        best = ms;
        cfg = k;
      }
    }
    c->tile_config = -1;
    remember(c, key, cfg);
  }
  c->tile_config = cfg;
  try {
    gemm(c, p, g);
  } catch (...) {
    c->tile_config = -1;
    throw;
  }
  c->tile_config = -1;
}

void tune_grouped(Ctx* c, GroupedPlan& g, const void* A, const void* B, void* C) {
  if (!c->autotune || g.ntasks == 0 || capturing(c)) return;
  double best = 1e300;
  int best_cfg = g.cfg;
  for (int cfg = 0; cfg <= 5; ++cfg) {
    g.cfg = cfg;
    grouped_retile(c, g);
    const double ms = time_ms(c, [&] { grouped_gemm(c, c->tune_prec, g, A, B, C, 1.0); }, 2);
    if (ms < best) {
      best = ms;
      best_cfg = cfg;
    }
  }
  if (g.cfg != best_cfg) {
    g.cfg = best_cfg;
    grouped_retile(c, g);
  }
}

}  // namespace d3s
