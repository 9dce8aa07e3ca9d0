// Host scheduler of the uneven batch (header only, no HIP: it is also built
// on the host alone for the sanitizer tests).
//
// n jobs with device-memory estimates est[i] run on ns host threads ("slots"),
// largest estimate first.  A job is admitted while the estimates of the jobs
// running plus its own stay within `budget`, or when nothing else runs (a
// job larger than the budget still runs, alone).  Every slot thread gets an
// explicit stack of stack_bytes: the solver threads call into the HIP
// runtime, the host eigensolver and the profiler's callbacks, and the
// platform's default thread stack is not something to rely on.
#pragma once
#include <pthread.h>

#include <algorithm>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <vector>

namespace bsex {

struct BatchHooks {
  std::function<void(int slot)> slot_begin;       // on the slot's thread, before any job
  std::function<void(int slot, int job)> run;     // one job
  std::function<void(int slot)> slot_end;         // on the slot's thread, after its last job
};

// Returns 0, or -1 when no slot thread could be started (then no job ran).
inline int schedule_batch(int n, const std::vector<double>& est, double budget, int ns,
                          size_t stack_bytes, const BatchHooks& hooks) {
  if (n <= 0) return 0;
  ns = std::max(1, std::min(ns, n));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return est[a] > est[b]; });
  struct Shared {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<char> started;
    double reserved = 0.0;
    int running = 0, left = 0;
  } sh;
  sh.started.assign(n, 0);
  sh.left = n;
  auto pick_next = [&]() -> int {
    std::unique_lock<std::mutex> lk(sh.mu);
    for (;;) {
      if (sh.left == 0) return -1;
      for (int i : order)
        if (!sh.started[i] && (sh.reserved + est[i] <= budget || sh.running == 0)) {
          sh.started[i] = 1;
          sh.reserved += est[i];
          ++sh.running;
          --sh.left;
          return i;
        }
      sh.cv.wait(lk);
    }
  };
  auto done = [&](int i) {
    {
      std::lock_guard<std::mutex> lk(sh.mu);
      sh.reserved -= est[i];
      --sh.running;
    }
    sh.cv.notify_all();
  };
  struct Arg {
    int slot;
    std::function<void(int)>* body;
  };
  std::function<void(int)> body = [&](int slot) {
    if (hooks.slot_begin) hooks.slot_begin(slot);
    for (int i; (i = pick_next()) >= 0; done(i)) hooks.run(slot, i);
    if (hooks.slot_end) hooks.slot_end(slot);
  };
  auto entry = [](void* p) -> void* {
    Arg* a = static_cast<Arg*>(p);
    (*a->body)(a->slot);
    return nullptr;
  };
  std::vector<Arg> args(ns);
  std::vector<pthread_t> th;
  pthread_attr_t attr;
  pthread_attr_init(&attr);
  pthread_attr_setstacksize(&attr, stack_bytes);
  for (int s = 0; s < ns; ++s) {
    args[s] = Arg{s, &body};
    pthread_t t;
    if (pthread_create(&t, &attr, entry, &args[s]) == 0) th.push_back(t);
  }
  pthread_attr_destroy(&attr);
  if (th.empty()) return -1;
  for (pthread_t t : th) pthread_join(t, nullptr);
  return 0;
}

}  // namespace bsex
