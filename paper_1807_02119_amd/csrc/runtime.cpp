// runtime.cpp -- host-side batch runtime: plan many knots on a pool of host
// threads, normalise many results (Eq. 4) in one call.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include <sched.h>
#include <unistd.h>

#include "internal.h"

namespace kn {

int32_t usable_cpus() {
  cpu_set_t set;
  CPU_ZERO(&set);
  if (sched_getaffinity(0, sizeof(set), &set) == 0) {
    const int c = CPU_COUNT(&set);
    if (c > 0) return c;
  }
  return (int32_t)std::max(1u, std::thread::hardware_concurrency());
}

namespace {

// Worker threads that sleep on a condition variable between calls.  A call
// publishes the job under a new generation number; each of the first
// `want` workers to wake runs it once.  The pool is never destroyed (its
// threads end with the process).
class Pool {
 public:
  explicit Pool(int32_t n) : pid_(getpid()) {
    for (int32_t i = 0; i < n; ++i) threads_.emplace_back([this] { loop(); });
  }
  pid_t pid() const { return pid_; }
  int32_t size() const { return (int32_t)threads_.size(); }
  std::mutex call_mu;  // one call at a time

  void run(int32_t helpers, const std::function<void()>& f) {
    {
      std::lock_guard<std::mutex> lock(mu_);
      job_ = &f;
      want_ = helpers;
      left_ = helpers;
      ++gen_;
    }
    cv_.notify_all();
    f();
    std::unique_lock<std::mutex> lock(mu_);
    done_cv_.wait(lock, [this] { return left_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lock(mu_);
    for (;;) {
      cv_.wait(lock, [&] { return gen_ != seen; });
      seen = gen_;
      if (want_ <= 0) continue;
      --want_;
      const std::function<void()>* f = job_;
      lock.unlock();
      (*f)();
      lock.lock();
      if (--left_ == 0) done_cv_.notify_all();
    }
  }
  pid_t pid_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void()>* job_ = nullptr;
  uint64_t gen_ = 0;
  int32_t want_ = 0, left_ = 0;
};

std::mutex g_pool_mu;
Pool* g_pool = nullptr;  // leaked on purpose, replaced in a forked child

Pool* pool() {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (!g_pool || g_pool->pid() != getpid()) g_pool = new Pool(std::min(usable_cpus(), 64) - 1);
  return g_pool;
}

}  // namespace

void parallel_run(int32_t n_threads, const std::function<void()>& f) {
  if (n_threads <= 1) {
    f();
    return;
  }
  Pool* pl = pool();
  std::unique_lock<std::mutex> lock(pl->call_mu, std::try_to_lock);
  if (lock.owns_lock() && pl->size() >= n_threads - 1) {
    pl->run(n_threads - 1, f);
    return;
  }
  std::vector<std::thread> extra;
  for (int32_t t = 1; t < n_threads; ++t) extra.emplace_back(f);
  f();
  for (auto& th : extra) th.join();
}

bool parallel_run_idle(int32_t n_threads, const std::function<void()>& f) {
  if (n_threads <= 1) return false;
  Pool* pl = pool();
  std::unique_lock<std::mutex> lock(pl->call_mu, std::try_to_lock);
  if (!lock.owns_lock()) return false;
  pl->run(std::min(n_threads, pl->size() + 1) - 1, f);
  return true;
}

}  // namespace kn

using kn::usable_cpus;

extern "C" kn_status kn_plan_many(int32_t n_knots, const int32_t* n_crossings, const int32_t* pd,
                                  const int8_t* signs, const int32_t* q, const kn_plan_opts* opts,
                                  int32_t n_threads, kn_tait** taits, kn_plan** plans,
                                  kn_status* status) {
  if (n_knots < 0 || (n_knots > 0 && (!n_crossings || !q || !taits || !plans))) return KN_E_INVALID;
  std::vector<int64_t> off(n_knots + 1, 0);
  for (int32_t i = 0; i < n_knots; ++i) {
    if (n_crossings[i] < 0) return KN_E_INVALID;
    off[i + 1] = off[i] + n_crossings[i];
  }
  if (off[n_knots] > 0 && !pd) return KN_E_INVALID;
  for (int32_t i = 0; i < n_knots; ++i) {
    taits[i] = nullptr;
    plans[i] = nullptr;
  }
  int32_t nt = n_threads > 0 ? n_threads : usable_cpus();
  nt = std::min(nt, std::max(1, n_knots));
  // largest knots first, so that the last ones handed out are short
  std::vector<int32_t> order(n_knots);
  for (int32_t i = 0; i < n_knots; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return n_crossings[a] > n_crossings[b]; });
  std::atomic<int32_t> next{0};
  std::vector<kn_status> st(n_knots, KN_OK);
  std::function<void()> worker = [&]() {
    for (;;) {
      const int32_t j = next.fetch_add(1);
      if (j >= n_knots) return;
      const int32_t i = order[j];
      kn_tait* g = nullptr;
      kn_status rc = kn_build_tait(n_crossings[i], pd ? pd + 4 * off[i] : nullptr,
                                   signs ? signs + off[i] : nullptr, -1, 0, &g);
      if (rc == KN_OK) {
        kn_plan* p = nullptr;
        rc = kn_plan_create(g, q[i], opts, &p);
        plans[i] = p;  // also kept on KN_E_BUDGET (statistics)
      }
      taits[i] = g;
      st[i] = rc;
    }
  };
  kn::parallel_run(nt, worker);
  kn_status first = KN_OK;
  for (int32_t i = 0; i < n_knots; ++i) {
    if (status) status[i] = st[i];
    if (first == KN_OK && st[i] != KN_OK) first = st[i];
  }
  return first;
}

extern "C" void kn_free_many(int32_t n, kn_tait** taits, kn_plan** plans) {
  for (int32_t i = 0; i < n; ++i) {
    if (plans && plans[i]) kn_plan_free(plans[i]);
    if (taits && taits[i]) kn_tait_free(taits[i]);
  }
}

extern "C" kn_status kn_jones_many(int32_t n, const int32_t* q, const kn_tait* const* g,
                                   const kn_scalar* z_host, double* v, double* log2_abs_v,
                                   double* arg_v) {
  if (n < 0 || (n > 0 && (!q || !g || !z_host))) return KN_E_INVALID;
  kn_status first = KN_OK;
  for (int32_t i = 0; i < n; ++i) {
    double re = 0, im = 0, l2 = 0, ar = 0;
    kn_status rc = kn_jones(q[i], g[i], &z_host[i], &re, &im, &l2, &ar);
    if (rc != KN_OK && first == KN_OK) first = rc;
    if (v) {
      v[2 * i] = re;
      v[2 * i + 1] = im;
    }
    if (log2_abs_v) log2_abs_v[i] = l2;
    if (arg_v) arg_v[i] = ar;
  }
  return first;
}
