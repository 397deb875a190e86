// Whole-path solve of a batch of problems (Alg. 1, steps 3-5 for every problem), split into
// parts that run concurrently: each part is built and solved by its own host thread on its own
// stream, so the host work and the short, latency-bound build launches of one part overlap the
// kernels of the others.  A part is an ordinary batch (stamp build, operator build, forcing,
// solve), and every problem's result is the one it gets alone.  The part threads are kept
// between calls (a new thread would pay its creation, the runtime's per-thread set-up and fresh
// pages for its reused host staging at the start of every batch).
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "ss_internal.h"

namespace ss {

namespace {

// Streams of the batch pipeline, created once per device and kept (default priority).
std::mutex g_stream_mu;
std::vector<std::vector<hipStream_t>> g_streams;

ss_status pipeline_streams(int device, int n, std::vector<hipStream_t>* out) {
  std::lock_guard<std::mutex> lk(g_stream_mu);
  if ((int)g_streams.size() <= device) g_streams.resize(device + 1);
  auto& v = g_streams[device];
  while ((int)v.size() < n) {
    hipStream_t s = nullptr;
    SS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    v.push_back(s);
  }
  out->assign(v.begin(), v.begin() + n);
  return SS_OK;
}

struct PartResult {
  ss_status status = SS_OK;
  std::string error;
};

// Worker threads that run queued jobs; they live as long as the process (never joined: a job
// never waits on another job, so a caller waiting for its own jobs cannot deadlock).
class PartPool {
 public:
  static PartPool& get() {
    static PartPool* p = new PartPool();   // never destroyed: workers may be blocked at exit
    return *p;
  }
  // run f(k) for k = 1 .. n - 1 on workers and f(0) on the caller; returns when all have ended
  void run(int n, const std::function<void(int)>& f) {
    struct Done {
      std::mutex mu;
      std::condition_variable cv;
      int left = 0;
    } done;
    done.left = n - 1;
    {
      std::lock_guard<std::mutex> g(mu_);
      while ((int)workers_ < n - 1 + busy_) {   // at least one idle worker per queued job
        std::thread(&PartPool::loop, this).detach();
        ++workers_;
      }
      for (int k = 1; k < n; ++k)
        jobs_.push_back([&f, &done, k]() {
          f(k);
          std::lock_guard<std::mutex> g(done.mu);
          if (--done.left == 0) done.cv.notify_all();
        });
      busy_ += n - 1;
    }
    cv_.notify_all();
    f(0);
    std::unique_lock<std::mutex> g(done.mu);
    done.cv.wait(g, [&]() { return done.left == 0; });
  }

 private:
  void loop() {
    for (;;) {
      std::function<void()> job;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&]() { return !jobs_.empty(); });
        job = std::move(jobs_.front());
        jobs_.pop_front();
      }
      job();
      std::lock_guard<std::mutex> g(mu_);
      --busy_;
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> jobs_;
  size_t workers_ = 0;
  int busy_ = 0;   // jobs queued or running
};

}  // namespace

void free_batch_impl(BatchImpl* b) {
  if (!b) return;
  for (auto& p : b->parts)
    if (p.u) pool_free(p.u);
  delete b;
}

ss_status batch_solve_impl(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                           const double* a_hat, const int32_t* n_f, const int16_t* f_freqs, const double* f_hat,
                           const int32_t* level, double tol, ss_precision prec, int32_t max_iter, uint32_t flags,
                           int32_t n_parts, ss_solve_info* info, BatchImpl** out) {
  *out = nullptr;
  if (n_prob < 1) return fail(SS_EINVAL, "n_prob must be >= 1");
  if (!n_a || !a_freqs || !a_hat || !n_f || !f_freqs || !f_hat || !level) return fail(SS_EINVAL, "null argument");
  if (n_parts < 1) return fail(SS_EINVAL, "n_parts must be >= 1");
  n_parts = std::min(n_parts, n_prob);
  int device = 0;
  SS_HIP(hipGetDevice(&device));
  std::vector<hipStream_t> streams;
  SS_TRY(pipeline_streams(device, n_parts, &streams));
  // entry offsets of every problem's a and f lists
  std::vector<int64_t> aoff(n_prob + 1, 0), foff(n_prob + 1, 0);
  for (int p = 0; p < n_prob; ++p) {
    if (n_a[p] < 0 || n_f[p] < 0) return fail(SS_EINVAL, "negative list length");
    aoff[p + 1] = aoff[p] + n_a[p];
    foff[p + 1] = foff[p] + n_f[p];
  }
  BatchImpl* b = new BatchImpl();
  std::unique_ptr<BatchImpl, void (*)(BatchImpl*)> guard(b, free_batch_impl);
  b->n_prob = n_prob;
  b->d = d;
  b->device = device;
  b->parts.resize(n_parts);
  for (int k = 0; k < n_parts; ++k) {
    b->parts[k].p0 = (int)((int64_t)n_prob * k / n_parts);
    b->parts[k].p1 = (int)((int64_t)n_prob * (k + 1) / n_parts);
  }
  std::vector<PartResult> res(n_parts);
  auto run = [&](int k) {
    BatchImpl::Part& part = b->parts[k];
    PartResult& r = res[k];
    const hipStream_t s = streams[k];
    const int p0 = part.p0, np = part.p1 - part.p0;
    auto failed = [&](ss_status st) {
      r.status = st;
      r.error = last_error_cstr();
    };
    if (hipSetDevice(device) != hipSuccess) {
      r.status = SS_EDEVICE;
      r.error = "hipSetDevice failed in a pipeline thread";
      return;
    }
    StampImpl* st = nullptr;
    ss_status e = build_stamp_impl(np, d, n_a + p0, a_freqs + aoff[p0] * d, n_f + p0, f_freqs + foff[p0] * d,
                                   level + p0, s, &st);
    if (e != SS_OK) return failed(e);
    std::unique_ptr<StampImpl, void (*)(StampImpl*)> stg(st, free_stamp_impl);
    OpImpl* op = nullptr;
    e = build_op_impl(st, n_a + p0, a_freqs + aoff[p0] * d, a_hat + 2 * aoff[p0], flags, s, &op);
    if (e != SS_OK) return failed(e);
    std::unique_ptr<OpImpl, void (*)(OpImpl*)> opg(op, free_op_impl);
    part.n = st->total;
    part.off = st->row_off;
    void* f = nullptr;
    if (pool_alloc(&f, (size_t)part.n * 16) != hipSuccess || pool_alloc((void**)&part.u, (size_t)part.n * 16) != hipSuccess) {
      if (f) pool_free(f);
      r.status = SS_ENOMEM;
      r.error = "device allocation failed";
      return;
    }
    e = stamp_forcing_impl(st, f_hat + 2 * foff[p0], f, s);
    if (e == SS_OK && hipMemsetAsync(part.u, 0, (size_t)part.n * 16, s) != hipSuccess) e = fail(SS_EDEVICE, "hipMemsetAsync failed");
    if (e == SS_OK) e = solve_op_impl(op, f, part.u, tol, prec, max_iter, s, info ? info + p0 : nullptr);
    (void)hipStreamSynchronize(s);   // the solve returns synchronised; this covers its error paths
    pool_free(f);
    if (e != SS_OK) failed(e);
  };
  PartPool::get().run(n_parts, run);
  // a build or device error wins over a solve that merely did not converge
  int worst = -1;
  for (int k = 0; k < n_parts; ++k) {
    if (res[k].status == SS_OK) continue;
    const bool solve_only = res[k].status == SS_ENOCONV || res[k].status == SS_EBREAKDOWN;
    if (worst < 0 || (!solve_only && (res[worst].status == SS_ENOCONV || res[worst].status == SS_EBREAKDOWN)))
      worst = k;
  }
  b->offsets.assign(n_prob + 1, 0);
  for (auto& part : b->parts)
    for (int q = 0; q < part.p1 - part.p0 && !part.off.empty(); ++q)
      b->offsets[part.p0 + q + 1] = part.off[q + 1] - part.off[q];
  for (int p = 0; p < n_prob; ++p) b->offsets[p + 1] += b->offsets[p];
  if (worst >= 0) {
    const ss_status st = res[worst].status;
    if (st != SS_ENOCONV && st != SS_EBREAKDOWN) return fail(st, res[worst].error);
    *out = guard.release();   // results are kept: the best iterates and the infos describe them
    return fail(st, res[worst].error);
  }
  *out = guard.release();
  return SS_OK;
}

ss_status batch_solution_impl(const BatchImpl* b, void* u, hipStream_t stream) {
  if (!u) return fail(SS_EINVAL, "null output");
  for (const auto& part : b->parts) {
    if (!part.u || part.n == 0) continue;
    double2* dst = static_cast<double2*>(u) + b->offsets[part.p0];
    SS_HIP(hipMemcpyAsync(dst, part.u, (size_t)part.n * 16, hipMemcpyDeviceToDevice, stream));
  }
  return SS_OK;
}

}  // namespace ss
