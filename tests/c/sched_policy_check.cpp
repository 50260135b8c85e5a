// Checks of the request server's scheduling policy (host functions only),
// built and run on the CPU by tests/test_sanitizers.py under the address and
// undefined-behaviour sanitizers.  Prints "sched policy OK" on success.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <vector>

#include "sched_policy.h"

using namespace gpe_sched;

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                               \
    }                                                             \
  } while (0)

struct Q {
  int id;
  bool heavy;
  uint64_t bytes;
};

// The server's admission walk over a queue: requests start in arrival order;
// a heavy one waiting for its tier is passed by those behind it.
std::vector<int> admit_walk(std::deque<Q> &queue, int &running, int &running_heavy,
                            uint64_t &used, uint64_t budget, int max_active, int heavy_active) {
  std::vector<int> started;
  size_t at = 0;
  while (at < queue.size()) {
    const Q &q = queue[at];
    AdmitInput in{q.heavy, running, max_active, running_heavy, heavy_active, true, q.bytes,
                  used, budget};
    const Admit d = admit_decision(in);
    if (d == kSkip) {
      ++at;
      continue;
    }
    if (d == kStop) break;
    started.push_back(q.id);
    ++running;
    if (q.heavy) ++running_heavy;
    used += q.bytes;
    queue.erase(queue.begin() + (long)at);
  }
  return started;
}

int main() {
  // tiers
  CHECK(is_heavy(1LL << 24, 1LL << 23));
  CHECK(is_heavy(1LL << 23, 1LL << 23));
  CHECK(!is_heavy((1LL << 23) - 1, 1LL << 23));
  CHECK(!is_heavy(1LL << 30, 0));

  // single decisions
  AdmitInput base{false, 0, 0, 0, 1, true, 100, 0, 1000};
  CHECK(admit_decision(base) == kAdmit);
  AdmitInput a = base;
  a.max_active = 2;
  a.running = 2;
  CHECK(admit_decision(a) == kStop);
  a = base;
  a.heavy = true;
  a.running_heavy = 1;
  CHECK(admit_decision(a) == kSkip);
  a.heavy_active = 0;  // no tier cap
  CHECK(admit_decision(a) == kAdmit);
  a = base;
  a.free_slot = false;
  CHECK(admit_decision(a) == kStop);
  a = base;
  a.used = 950;
  CHECK(admit_decision(a) == kStop);
  a.used = 900;
  CHECK(admit_decision(a) == kAdmit);
  a.need = 2000;  // more than the whole budget: no unsigned wrap
  a.used = 0;
  CHECK(admit_decision(a) == kStop);

  // a walk: H1 runs, H2 waits for the tier, lights behind it pass
  {
    std::deque<Q> queue = {{1, true, 100}, {2, true, 100}, {3, false, 10}, {4, false, 10},
                           {5, true, 100}, {6, false, 10}};
    int running = 0, rh = 0;
    uint64_t used = 0;
    std::vector<int> s = admit_walk(queue, running, rh, used, 10000, 0, 1);
    CHECK((s == std::vector<int>{1, 3, 4, 6}));
    CHECK(queue.size() == 2 && queue[0].id == 2 && queue[1].id == 5);
    // H1 finishes: H2 (not H5) starts next
    --running;
    --rh;
    used -= 100;
    s = admit_walk(queue, running, rh, used, 10000, 0, 1);
    CHECK((s == std::vector<int>{2}));
    CHECK(queue.size() == 1 && queue[0].id == 5);
  }
  // memory keeps arrival order: a light request that does not fit stops the walk
  {
    std::deque<Q> queue = {{1, false, 600}, {2, false, 600}, {3, false, 10}};
    int running = 0, rh = 0;
    uint64_t used = 0;
    std::vector<int> s = admit_walk(queue, running, rh, used, 1000, 0, 1);
    CHECK((s == std::vector<int>{1}));
    CHECK(queue.front().id == 2);
  }
  // max_active = 1 is one at a time over every tier
  {
    std::deque<Q> queue = {{1, false, 1}, {2, true, 1}, {3, false, 1}};
    int running = 0, rh = 0;
    uint64_t used = 0;
    std::vector<int> s = admit_walk(queue, running, rh, used, 1000, 1, 1);
    CHECK((s == std::vector<int>{1}));
  }

  // chunk sizes: about quantum_ms of GPU time per running request
  ChunkInput c{};
  c.running = 4;
  c.step_ms = 0.5;
  c.step_running = 4;
  c.use_graph = false;
  c.paced = false;
  c.chunk = 16;
  c.quantum_ms = 1.0;
  c.sites = 1 << 24;
  c.esize = 16;
  CHECK(chunk_steps(c) == 8);  // 4 x 1 ms / 0.5 ms
  c.step_running = 2;          // measured with half the slots: twice the time now
  CHECK(chunk_steps(c) == 4);
  c.step_ms = 1e-9;            // capped
  CHECK(chunk_steps(c) == 4096);
  c.step_ms = 0;               // unmeasured: estimate from the bytes
  const int est = chunk_steps(c);
  CHECK(est >= 1 && est <= 4096);
  c.use_graph = true;          // whole graph replays
  c.step_ms = 0.01;
  c.step_running = 4;
  CHECK(chunk_steps(c) % 16 == 0 && chunk_steps(c) >= 16);
  c.paced = true;              // paced to the main stream's round
  c.main_round_ms = 10.0;
  c.step_ms = 0.1;
  CHECK(chunk_steps(c) == 100);
  c.step_ms = 0;
  CHECK(chunk_steps(c) == 16);
  std::printf("sched policy OK\n");
  return 0;
}
