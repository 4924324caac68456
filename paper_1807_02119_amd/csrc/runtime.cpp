// runtime.cpp -- host-side batch runtime: plan many knots on a pool of host
// threads, normalise many results (Eq. 4) in one call.
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include <sched.h>

#include "internal.h"

namespace {

// CPUs this process may run on (its affinity mask), at least 1.
int32_t usable_cpus() {
  cpu_set_t set;
  CPU_ZERO(&set);
  if (sched_getaffinity(0, sizeof(set), &set) == 0) {
    const int c = CPU_COUNT(&set);
    if (c > 0) return c;
  }
  return (int32_t)std::max(1u, std::thread::hardware_concurrency());
}

}  // namespace

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
  std::atomic<int32_t> next{0};
  std::vector<kn_status> st(n_knots, KN_OK);
  auto worker = [&]() {
    for (;;) {
      int32_t i = next.fetch_add(1);
      if (i >= n_knots) return;
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
  std::vector<std::thread> pool;
  for (int32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  kn_status first = KN_OK;
  for (int32_t i = 0; i < n_knots; ++i) {
    if (status) status[i] = st[i];
    if (first == KN_OK && st[i] != KN_OK) first = st[i];
  }
  return first;
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
