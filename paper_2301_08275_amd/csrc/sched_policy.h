// Scheduling policy of the request server, as pure host functions (no HIP):
// which queued request may start now, and how many steps a shape class gets
// in a round.  Kept apart from the GPU code so that it can be built and
// checked on the CPU alone (also under the address and undefined-behaviour
// sanitizers).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace gpe_sched {

// Requests of at least heavy_sites grid points form the heavy tier; 0 turns
// the tiers off.
inline bool is_heavy(long long sites, long long heavy_sites) {
  return heavy_sites > 0 && sites >= heavy_sites;
}

enum Admit {
  kAdmit = 0,  // start it now
  kStop = 1,   // it waits, and so does everything behind it (arrival order
               // decides who gets memory and slots)
  kSkip = 2,   // it waits for a heavy request to finish; requests behind it
               // may start meanwhile
};

struct AdmitInput {
  bool heavy;          // the request is in the heavy tier
  int running;         // requests running, all tiers
  int max_active;      // cap on running requests (0: none)
  int running_heavy;   // heavy requests running
  int heavy_active;    // cap on running heavy requests (0: none)
  bool free_slot;      // its shape class has a free slot (or does not exist yet)
  uint64_t need;       // device bytes it would add
  uint64_t used;       // device bytes held
  uint64_t budget;     // device bytes allowed
};

// Heavy requests run first come, first served among themselves (at most
// heavy_active at once), while lighter requests share the GPU beside them:
// a heavy request then waits only for the heavy requests that arrived before
// it, not for every request in between, and light requests never queue
// behind a heavy one.  A budget refusal is kStop: the caller may free idle
// memory and ask again.
inline Admit admit_decision(const AdmitInput &in) {
  if (in.max_active > 0 && in.running >= in.max_active) return kStop;
  if (in.heavy && in.heavy_active > 0 && in.running_heavy >= in.heavy_active) return kSkip;
  if (!in.free_slot) return kStop;
  if (in.need > in.budget || in.used > in.budget - in.need) return kStop;
  return kAdmit;
}

struct ChunkInput {
  int running;             // running slots of the class
  double step_ms;          // measured GPU ms per batched step (<= 0: unknown)
  int step_running;        // running slots when step_ms was measured
  bool use_graph;          // chunks are whole replays of a chunk_steps graph
  bool paced;              // the class runs beside the main stream (on-chip or heavy)
  int chunk;               // steps per graph replay
  double quantum_ms;       // GPU time per running request per round
  double main_round_ms;    // the main stream's last round (pacing)
  double sites, esize;     // grid points and bytes per point of the class
};

// Steps for a class in one round: about quantum_ms of GPU time per running
// request.  Large grids are bandwidth-bound (a step's time grows with the
// running slots); small ones are launch-bound (it does not), and run whole
// graph replays.  Classes beside the main stream (on-chip classes on a few
// CUs, heavy classes on a stream of their own) are paced to last about as
// long as the main stream's last round.  An
// unmeasured class assumes about 4 TB/s over three passes of reads and writes.
inline int chunk_steps(const ChunkInput &in) {
  const int run = std::max(1, in.running);
  double ms = in.step_ms;
  if (in.paced) {
    if (!(ms > 0)) return in.chunk;
    const double target = std::max(in.quantum_ms * run, in.main_round_ms);
    return (int)std::max(1LL, std::min(65536LL, std::llround(target / ms)));
  }
  if (!(ms > 0)) {
    if (in.use_graph) return in.chunk;
    const double bytes = 6.0 * (double)run * in.sites * in.esize;
    ms = 0.02 + bytes / 4.0e9;
  } else if (!in.use_graph && in.step_running > 0) {
    ms *= (double)run / (double)in.step_running;
  }
  const double k = in.quantum_ms * run / ms;
  if (in.use_graph) {
    const long long reps = std::max(1LL, std::min(256LL, std::llround(k / in.chunk)));
    return (int)(reps * in.chunk);
  }
  return (int)std::max(1LL, std::min(4096LL, std::llround(k)));
}

}  // namespace gpe_sched
