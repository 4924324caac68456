// Host-thread model of the persistent engine's task queue, for
// ThreadSanitizer (tests/test_queue_model.py builds it with
// -fsanitize=thread and runs it).
//
// The device program is a set of chains of task groups: group g + 1 of a
// chain starts when every task of group g has finished.  A workgroup of the
// engine is modelled by kWaves threads that meet at a barrier of their own
// (the workgroup barrier: a counter and a generation word of that workgroup,
// nothing shared with other workgroups -- std::barrier waits through a
// process-wide table of mutexes, which would order workgroups that the
// engine does not order and hide races from the sanitizer); the queue
// protocol is the engine's, operation for operation:
//   claim    thread 0: slot = head.fetch_add(1, relaxed); if slot < n_tasks,
//            wait until queue[slot] >= 0 (the engine: relaxed agent-scope loads,
//            then an agent-scope acquire fence; here the load itself is an
//            acquire, the form ThreadSanitizer understands: it does not model
//            stand-alone fences); the task id goes to the other threads through
//            shared memory and the barrier.
//   run      every thread reads the data words written by the tasks of the
//            previous group (plain loads) and writes its part of this task's
//            data (plain stores) -- the tensor entries of the engine.
//   publish  barrier (every thread's stores happen before it; the engine:
//            each wave's release fence, then the barrier); thread 0:
//            pending[next].fetch_sub(1, acq_rel); the last finisher reserves
//            n slots with tail.fetch_add(n, relaxed) and writes the next
//            group's task ids with release stores.
// Checks: every task runs exactly once, only after all tasks of its previous
// group finished and with their data visible; every chain's last group runs;
// the grid drains (every claimed slot is eventually filled) for any number of
// workgroups.  A data race on the plain words is reported by the sanitizer.
//
//   queue_model SEED N_WORKGROUPS   -> prints "ok <tasks>" or an error, exit 0/1
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr int kWaves = 2;           // threads per modelled workgroup
constexpr int kWordsPerTask = 4;    // data words a task writes (split over its waves)
constexpr long kSpinLimit = 200000000;  // bounded wait: a bug ends the run, not the test host

// Orders of the queue's publish store and claim load.  The tests also build
// the model with both relaxed (a planted mistake: nothing then orders a
// task's data before its successor's reads) to show that the sanitizer
// catches it.
#ifdef KN_MODEL_RELAXED_QUEUE
constexpr std::memory_order kPublish = std::memory_order_relaxed;
constexpr std::memory_order kClaim = std::memory_order_relaxed;
#else
constexpr std::memory_order kPublish = std::memory_order_release;
constexpr std::memory_order kClaim = std::memory_order_acquire;
#endif

struct Group {
  int first, n, next, n_pred;
};

// The barrier of one workgroup: the last of n arrivals (its acq_rel
// increment reads every earlier arrival's) advances the generation with a
// release store, which the waiters read with acquire loads.
struct WgBarrier {
  std::atomic<int> count{0}, gen{0};
  const int n;
  explicit WgBarrier(int n_) : n(n_) {}
  void arrive_and_wait() {
    const int g = gen.load(std::memory_order_acquire);
    if (count.fetch_add(1, std::memory_order_acq_rel) == n - 1) {
      count.store(0, std::memory_order_relaxed);
      gen.store(g + 1, std::memory_order_release);
    } else {
      while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
    }
  }
};

struct Program {
  std::vector<Group> groups;
  std::vector<int> task_group;  // group of every task
  std::vector<int> roots;       // first tasks of every chain's first group
  int n_tasks = 0;
};

Program make_program(unsigned seed) {
  std::mt19937 rng(seed);
  Program p;
  const int chains = 1 + (int)(rng() % 12);
  std::vector<int> first_groups;
  for (int c = 0; c < chains; ++c) {
    const int len = 1 + (int)(rng() % 8);
    int prev = -1;
    for (int j = 0; j < len; ++j) {
      const int n = 1 + (int)(rng() % 9);
      const int g = (int)p.groups.size();
      p.groups.push_back({p.n_tasks, n, -1, prev < 0 ? 0 : p.groups[prev].n});
      for (int i = 0; i < n; ++i) p.task_group.push_back(g);
      p.n_tasks += n;
      if (prev >= 0) p.groups[prev].next = g;
      else first_groups.push_back(g);
      prev = g;
    }
  }
  for (int g : first_groups)
    for (int i = 0; i < p.groups[g].n; ++i) p.roots.push_back(p.groups[g].first + i);
  return p;
}

struct State {
  std::atomic<int> head{0}, tail{0}, error{0};
  std::vector<std::atomic<int>> queue, pending, runs;
  std::vector<int> data;        // plain words: kWordsPerTask per task
  explicit State(const Program& p)
      : queue(p.n_tasks), pending(p.groups.size()), runs(p.n_tasks),
        data((size_t)p.n_tasks * kWordsPerTask, 0) {
    for (int i = 0; i < p.n_tasks; ++i) {
      queue[i].store(i < (int)p.roots.size() ? p.roots[i] : -1, std::memory_order_relaxed);
      runs[i].store(0, std::memory_order_relaxed);
    }
    for (size_t g = 0; g < p.groups.size(); ++g)
      pending[g].store(p.groups[g].n_pred, std::memory_order_relaxed);
    tail.store((int)p.roots.size(), std::memory_order_relaxed);
  }
};

void workgroup(const Program& p, State& s) {
  WgBarrier bar(kWaves);
  int shared_task = -1;  // the workgroup's LDS word
  auto wave = [&](int w) {
    for (;;) {
      if (w == 0) {
        int t = -1;
        const int slot = s.head.fetch_add(1, std::memory_order_relaxed);
        if (slot < p.n_tasks) {
          long spins = 0;
          while ((t = s.queue[slot].load(kClaim)) < 0) {
            std::this_thread::yield();
            if (++spins > kSpinLimit) {
              s.error.store(1, std::memory_order_relaxed);
              break;
            }
          }
        }
        shared_task = t;
      }
      bar.arrive_and_wait();
      const int t = shared_task;
      bar.arrive_and_wait();
      if (t < 0) return;
      // run: the previous group's data must be complete and visible
      const Group& g = p.groups[p.task_group[t]];
      if (w == 0 && s.runs[t].fetch_add(1, std::memory_order_relaxed) != 0)
        s.error.store(2, std::memory_order_relaxed);
      int prev = -1;
      for (size_t k = 0; k < p.groups.size(); ++k)
        if (p.groups[k].next == p.task_group[t]) prev = (int)k;
      if (prev >= 0) {
        const Group& pg = p.groups[prev];
        for (int u = pg.first; u < pg.first + pg.n; ++u)
          for (int j = w; j < kWordsPerTask; j += kWaves)
            if (s.data[(size_t)u * kWordsPerTask + j] != 1 + u * kWordsPerTask + j)
              s.error.store(3, std::memory_order_relaxed);
      }
      for (int j = w; j < kWordsPerTask; j += kWaves)
        s.data[(size_t)t * kWordsPerTask + j] = 1 + t * kWordsPerTask + j;
      // publish
      bar.arrive_and_wait();
      if (w == 0 && g.next >= 0 &&
          s.pending[g.next].fetch_sub(1, std::memory_order_acq_rel) == 1) {
        const Group& ng = p.groups[g.next];
        const int base = s.tail.fetch_add(ng.n, std::memory_order_relaxed);
        for (int i = 0; i < ng.n; ++i)
          s.queue[base + i].store(ng.first + i, kPublish);
      }
      bar.arrive_and_wait();
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < kWaves; ++w) th.emplace_back(wave, w);
  wave(0);
  for (auto& x : th) x.join();
}

}  // namespace

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1;
  const int grid = argc > 2 ? std::atoi(argv[2]) : 4;
  const Program p = make_program(seed);
  State s(p);
  std::vector<std::thread> wgs;
  for (int i = 0; i < grid; ++i) wgs.emplace_back(workgroup, std::cref(p), std::ref(s));
  for (auto& x : wgs) x.join();
  int bad = s.error.load();
  for (int t = 0; t < p.n_tasks && !bad; ++t)
    if (s.runs[t].load() != 1) bad = 4;
  if (!bad && s.tail.load() != p.n_tasks) bad = 5;
  if (bad) {
    std::printf("error %d (seed %u, grid %d, %d tasks)\n", bad, seed, grid, p.n_tasks);
    return 1;
  }
  std::printf("ok %d\n", p.n_tasks);
  return 0;
}
