// Concurrent batched eigensolves for the truncation.
//
// rocSOLVER's divide-and-conquer eigensolver launches a short sequence of
// small kernels per matrix column, so a call costs about 24 us per column
// of its largest matrix whatever the batch, and the device sits mostly idle
// meanwhile (measured on MI355X).  The calls of one truncation (one per
// group of sector matrices of similar size) are independent, so they run
// side by side: a few host threads, each with its own HIP stream (default
// priority) and its own rocBLAS handle, each issue their calls' launch
// sequences at once, and the calling thread takes one share itself on the
// context's stream (so k concurrent shares use k streams: under HIP's
// default of four hardware queues per process a stream beyond them shares a
// queue and serialises behind it).  The caller's stream work before the
// solves is ordered before the workers' by an event; every worker
// synchronises its own stream before reporting, so the caller continues
// after all solves have completed.
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "d3s_internal.h"

namespace d3s {

struct EigPool {
  struct Worker {
    hipStream_t stream = nullptr;
    rocblas_handle handle = nullptr;
    std::thread th;
    std::function<void()> job;
    bool has_job = false;
    d3s_status code = D3S_OK;
    std::string msg;
  };
  int device = 0;
  std::vector<Worker> w;
  hipEvent_t start = nullptr;          // recorded on the caller's stream before the solves
  std::mutex m;
  std::condition_variable cv_job, cv_done;
  int pending = 0;
  bool stop = false;
};

namespace {

void worker_main(EigPool* P, int k) {
  EigPool::Worker& W = P->w[k];
  (void)hipSetDevice(P->device);
  for (;;) {
    std::function<void()> job;
    {
      std::unique_lock<std::mutex> lk(P->m);
      P->cv_job.wait(lk, [&] { return P->stop || W.has_job; });
      if (!W.has_job) return;          // stop requested and nothing left
      job = std::move(W.job);
      W.has_job = false;
    }
    d3s_status code = D3S_OK;
    std::string msg;
    try {
      job();
    } catch (const Error& e) {
      code = e.code;
      msg = e.msg;
    } catch (...) {
      code = D3S_EDEVICE;
      msg = "eigensolver worker: unexpected exception";
    }
    std::lock_guard<std::mutex> lk(P->m);
    W.code = code;
    W.msg = msg;
    if (--P->pending == 0) P->cv_done.notify_all();
  }
}

EigPool* pool_of(Ctx* c, int workers) {
  if (c->eig_pool && (int)c->eig_pool->w.size() == workers) return c->eig_pool;
  eig_pool_destroy(c);
  EigPool* P = new EigPool();
  P->device = c->device;
  P->w.resize(workers);
  try {
    D3S_HIP(hipEventCreateWithFlags(&P->start, hipEventDisableTiming));
    for (auto& W : P->w) {
      D3S_HIP(hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking));
      if (rocblas_create_handle(&W.handle) != rocblas_status_success)
        throw Error{D3S_EDEVICE, "rocblas_create_handle failed"};
      if (rocblas_set_stream(W.handle, W.stream) != rocblas_status_success)
        throw Error{D3S_EDEVICE, "rocblas_set_stream failed"};
    }
    for (int k = 0; k < workers; ++k) P->w[k].th = std::thread(worker_main, P, k);
  } catch (...) {
    c->eig_pool = P;
    eig_pool_destroy(c);
    throw;
  }
  c->eig_pool = P;
  return P;
}

}  // namespace

void eig_pool_destroy(Ctx* c) {
  EigPool* P = c->eig_pool;
  if (!P) return;
  {
    std::lock_guard<std::mutex> lk(P->m);
    P->stop = true;
  }
  P->cv_job.notify_all();
  for (auto& W : P->w)
    if (W.th.joinable()) W.th.join();
  for (auto& W : P->w) {
    if (W.handle) (void)rocblas_destroy_handle(W.handle);
    if (W.stream) (void)hipStreamDestroy(W.stream);
  }
  if (P->start) (void)hipEventDestroy(P->start);
  delete P;
  c->eig_pool = nullptr;
}

namespace {

// the calls `mine` of one share on stream s with handle h; throws on a
// failed or unconverged solve, and drains s before returning either way
void run_share(const std::vector<EigCall>& calls, const std::vector<int>& mine, hipStream_t s, rocblas_handle h,
               hipEvent_t start, char* scratch, const std::vector<size_t>& eo, const std::vector<size_t>& io,
               double* G, double* V) {
  std::vector<std::vector<rocblas_int>> info(mine.size());
  // whatever happens, the stream is drained before the share reports (and
  // before `info`, which copies may target, goes away)
  struct Drain {
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{s};
  if (start) D3S_HIP(hipStreamWaitEvent(s, start, 0));
  for (size_t j = 0; j < mine.size(); ++j) {
    const EigCall& e = calls[mine[j]];
    double* E = (double*)(scratch + eo[mine[j]]);
    rocblas_int* inf = (rocblas_int*)(scratch + io[mine[j]]);
    const rocblas_status st = rocsolver_dsyevd_strided_batched(
        h, rocblas_evect_original, rocblas_fill_upper, e.n, G + e.goff, e.n, (rocblas_stride)e.n * e.n, V + e.voff,
        e.n, E, e.n, inf, e.batch);
    if (st != rocblas_status_success)
      throw Error{D3S_EDEVICE, "rocsolver batched eigensolver failed (status " + std::to_string((int)st) + ")"};
    info[j].resize(e.batch);
    D3S_HIP(hipMemcpyAsync(info[j].data(), inf, sizeof(rocblas_int) * e.batch, hipMemcpyDeviceToHost, s));
  }
  D3S_HIP(hipStreamSynchronize(s));
  for (const auto& v : info)
    for (rocblas_int x : v)
      if (x != 0)
        throw Error{D3S_EDEVICE, "rocsolver batched eigensolver did not converge (info " + std::to_string(x) + ")"};
}

}  // namespace

void eig_calls_parallel(Ctx* c, const std::vector<EigCall>& calls, const std::vector<int>& worker, int workers,
                        double* G, double* V) {
  // share 0 runs here on the context's stream, shares 1.. on pool threads
  EigPool* P = pool_of(c, workers - 1);
  if (!c->solver) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{D3S_EDEVICE, "rocblas_create_handle failed"};
    c->solver = h;
  }
  rocblas_handle own = (rocblas_handle)c->solver;
  if (rocblas_set_stream(own, c->stream) != rocblas_status_success)
    throw Error{D3S_EDEVICE, "rocblas_set_stream failed"};
  // per call: the off-diagonal scratch of the tridiagonal form and the info flags
  std::vector<size_t> eo(calls.size()), io(calls.size());
  size_t bytes = 0;
  for (size_t i = 0; i < calls.size(); ++i) {
    eo[i] = bytes;
    bytes += ((sizeof(double) * (size_t)calls[i].n * calls[i].batch) + 255) & ~(size_t)255;
    io[i] = bytes;
    bytes += ((sizeof(rocblas_int) * (size_t)calls[i].batch) + 255) & ~(size_t)255;
  }
  char* scratch = (char*)ws_get(c, WS_EIG_PAR, bytes);
  D3S_HIP(hipEventRecord(P->start, c->stream));
  std::vector<int> mine0;
  {
    std::lock_guard<std::mutex> lk(P->m);
    P->pending = 0;
    for (int k = 0; k < workers; ++k) {
      std::vector<int> mine;
      for (size_t i = 0; i < calls.size(); ++i)
        if (worker[i] == k) mine.push_back((int)i);
      if (k == 0) {
        mine0 = mine;
        continue;
      }
      EigPool::Worker& W = P->w[k - 1];
      W.code = D3S_OK;
      W.msg.clear();
      if (mine.empty()) continue;
      W.job = [=, &calls, &W, &eo, &io]() {
        run_share(calls, mine, W.stream, W.handle, P->start, scratch, eo, io, G, V);
      };
      W.has_job = true;
      ++P->pending;
    }
  }
  P->cv_job.notify_all();
  d3s_status code = D3S_OK;
  std::string msg;
  try {
    run_share(calls, mine0, c->stream, own, nullptr, scratch, eo, io, G, V);
  } catch (const Error& e) {
    code = e.code;
    msg = e.msg;
  } catch (...) {
    code = D3S_EDEVICE;
    msg = "eigensolver: unexpected exception";
  }
  {
    std::unique_lock<std::mutex> lk(P->m);
    P->cv_done.wait(lk, [&] { return P->pending == 0; });
  }
  if (code != D3S_OK) throw Error{code, msg};
  for (auto& W : P->w)
    if (W.code != D3S_OK) throw Error{W.code, W.msg};
}

}  // namespace d3s
