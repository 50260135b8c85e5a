// Serving scheduler behind the gpe_server_* calls of include/gpe.h.
//
// One scheduler thread owns every GPU call and works in rounds.  A round
//  1. admits queued requests in arrival order while the HBM budget allows and
//     a slot of their shape class (dim, n, precision, box, dt, mode) is free: the
//     state upload goes to a side stream while the GPU still runs the previous
//     round, and the slot-table entry is written on the main stream after it;
//  2. enqueues one chunk of batched steps per shape class with requests in it
//     (the fused axis passes in slot mode; imaginary-time classes add a
//     renormalisation kernel per step; step counts advance once per chunk).  Small
//     classes replay a captured graph over all slots, large ones launch rows
//     for their owned slots only.  Chunks are sized from the measured GPU time
//     per step so that every running request receives about the same GPU time
//     per round, whatever its grid: small solves finish in few rounds instead
//     of advancing at the pace of the largest grid.  Small square 2D grids
//     form on-chip classes instead: one workgroup per request holds the whole
//     grid in LDS and runs the chunk's steps in one launch, on a side stream,
//     so they occupy a few CUs beside the large classes and are paced to
//     last about as long as the main stream's round.  Heavy-tier classes
//     (the largest grids, first come, first served) run on a stream of their
//     own in the same way: concurrently with the lighter classes, so a
//     heavy solve is not held to one quantum per round beside them;
//  3. copies the slot tables back and only then waits for the previous
//     round's chunk, and finishes the requests that chunk completed (final
//     imaginary-time scaling, observables, optional state download, all on the
//     side stream) while the GPU runs the chunk just enqueued.
// A finished or free slot costs its rows an early return, so a request that
// completes inside a chunk never changes the launches, and its state is left
// alone by the chunk that follows; that is what lets the host finish it one
// round late without stalling the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gpe_ctx.h"
#include "sched_policy.h"

using namespace gpe_host;

namespace {

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Req {
  uint64_t id = 0;
  gpe_request r{};
  std::vector<double> psi0_d;  // FP64 classes: the initial state as given
  std::vector<float> psi0_f;   // FP32 classes: rounded once at submit
  ReqState state = RQ_QUEUED;
  gpe_status status = GPE_EBUSY;
  gpe_obs obs{};
  double t_submit = 0, t_start = 0, t_done = 0;
  int64_t steps_done = 0;
  std::vector<double> psi_out;
  bool cancel = false;
  uint64_t need = 0;        // device bytes a fresh slot context takes
  uint64_t need_class = 0;  // device bytes a new shape class takes
  bool heavy = false;       // in the heavy tier (first come, first served)
};

struct ClassKey {
  int dim, n[3], prec, mode;
  double lo[3], hi[3], dt;
  bool operator==(const ClassKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

ClassKey key_of(const gpe_request &r) {
  ClassKey k;
  std::memset(&k, 0, sizeof(k));
  k.dim = r.desc.dim;
  k.prec = r.desc.precision;
  for (int j = 0; j < r.desc.dim; ++j) {
    k.n[j] = r.desc.n[j];
    k.lo[j] = r.desc.lo[j];
    k.hi[j] = r.desc.hi[j];
  }
  k.dt = r.dt;
  k.mode = r.mode;
  return k;
}

// Slot life: free -> running -> (finished and released) or draining -> free.
// A draining slot (cancelled, or its chunk failed) has had its table entry
// cleared on the main stream but may still be touched by a chunk already in
// flight; it is released once that chunk is known to be done.
enum SlotState { SS_FREE = 0, SS_RUN = 1, SS_DRAIN = 2 };

struct ShapeClass {
  ClassKey key{};
  int S = 0;
  gpe_ctx *proto = nullptr;             // geometry, twiddles, weights; no state
  std::vector<gpe_ctx *> ctx;           // per slot, kept for reuse while memory allows
  std::vector<uint64_t> owner;          // request id per slot (0: none)
  std::vector<int> sstate;              // SlotState
  std::vector<int> steps_total;
  std::vector<long long> admit_round;   // round whose chunk first ran the slot
  std::vector<long long> drain_until;   // draining: last round whose chunk may touch it
  std::vector<gpe_status> drain_status;
  gpe::Slot *d = nullptr;               // device slot table
  gpe::Slot *hp[2] = {nullptr, nullptr};  // pinned read-backs, by round parity
  bool hp_valid[2] = {false, false};
  bool failed[2] = {false, false};
  double *partial = nullptr;            // norm partials, S x blocks of the last pass
  long long bpg_last = 0;
  void *kreal[3] = {nullptr, nullptr, nullptr}, *kimag[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t graph = nullptr;
  bool use_graph = false;               // small grids: replay a chunk graph over all slots
  bool onchip = false;                  // square 2D grid held in LDS, steps looped in-kernel
  bool paced = false;                   // beside the main stream, paced to its round
  hipStream_t strm = nullptr;           // stream of the class's launches and table writes
  int *d_map = nullptr;                 // large grids: rows for the owned slots only
  int rows = 0;
  bool map_dirty = true;
  int owned = 0;                        // slots running or draining
  int running = 0;                      // slots running
  hipEvent_t ev0[2] = {nullptr, nullptr}, ev1[2] = {nullptr, nullptr};
  int timed_steps[2] = {0, 0}, timed_running[2] = {0, 0};
  double step_ms = 0;                   // measured GPU ms per batched step (0: unknown)
  int step_running = 0;                 // running slots when it was measured
  uint64_t fixed_bytes = 0;             // table holder + slot table + map + partials
};

}  // namespace

struct gpe_server {
  hipStream_t stream = nullptr;  // batched steps and slot-table writes
  hipStream_t aux = nullptr;     // uploads, final scaling, observables, downloads
  hipStream_t side = nullptr;    // on-chip classes (beside the main stream)
  hipStream_t heavy = nullptr;   // heavy-tier classes (beside the main stream)
  hipEvent_t done[2] = {nullptr, nullptr};        // end of a round's main-stream work
  hipEvent_t done_side[2] = {nullptr, nullptr};   // end of a round's side-stream work
  hipEvent_t done_heavy[2] = {nullptr, nullptr};  // end of a round's heavy-stream work
  bool used_main[2] = {false, false}, used_side[2] = {false, false};
  bool used_heavy[2] = {false, false};
  double main_round_ms = 0;      // GPU time of the main stream's last retired round
  hipEvent_t ev_up = nullptr;
  int device = 0;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  int max_slots = 1, max_active = 0, chunk = 16;
  bool use_graph = true;
  bool use_onchip = true;
  // Largest edge routed to the on-chip class.  One workgroup holds a whole
  // grid, so its step time grows with the grid on one CU: a lone 128^2 FP32
  // request took 48 us per step there against 12 us in the streaming
  // batched passes, while 64^2 grids run as fast or faster on chip.
  int onchip_max_n = 64;
  double quantum_ms = 1.0;  // GPU time per running request per round
  // Heavy tier: requests of at least heavy_sites points run first come,
  // first served, at most heavy_active at once, beside the lighter ones.
  long long heavy_sites = 1LL << 23;
  int heavy_active = 1;
  // GPU time per round of a running heavy request, in quanta (a running
  // light request gets one): at least heavy_weight, and at least
  // heavy_share / (1 - heavy_share) times the light requests' total, so that
  // the heavy tier keeps that fraction of each round (0: no such floor).
  double heavy_weight = 1.0;
  double heavy_share = 0.0;
  // Heavy classes run on a stream of their own, concurrently with the
  // lighter classes of the round and paced to last as long as the main
  // stream's round (else they take their quanta on the main stream).
  bool heavy_beside = true;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<ShapeClass *> classes;  // touched by the scheduler thread only
  uint64_t next_id = 1;
  int running = 0;
  int running_heavy = 0;
  bool stop = false;
  std::thread th;
  std::chrono::steady_clock::time_point t0;
  int64_t submitted = 0, completed = 0;
  double busy = 0, site_steps = 0;
};

namespace {

double now_s(const gpe_server *s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

long long sites_of(const gpe_desc &d) {
  long long n = 1;
  for (int j = 0; j < d.dim; ++j) n *= d.n[j];
  return n;
}

void destroy_class(gpe_server *s, ShapeClass *c) {
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->side);
  (void)hipStreamSynchronize(s->heavy);
  (void)hipStreamSynchronize(s->aux);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  for (gpe_ctx *x : c->ctx)
    if (x) gpe_destroy(x);
  if (c->proto) gpe_destroy(c->proto);
  if (c->d) (void)hipFree(c->d);
  if (c->partial) (void)hipFree(c->partial);
  if (c->d_map) (void)hipFree(c->d_map);
  for (int p = 0; p < 2; ++p) {
    if (c->hp[p]) (void)hipHostFree(c->hp[p]);
    if (c->ev0[p]) (void)hipEventDestroy(c->ev0[p]);
    if (c->ev1[p]) (void)hipEventDestroy(c->ev1[p]);
  }
  delete c;
}

// Device bytes a shape class holds besides its slot contexts: the table holder
// (geometry, twiddles, weights, its partials), two kinetic tables per axis,
// the slot table, the slot map and the norm partials of every slot.
uint64_t class_bytes(const gpe_desc &d, int max_slots) {
  int n3[3] = {1, 1, 1};
  const int off = 3 - d.dim;
  for (int j = 0; j < d.dim; ++j) n3[j + off] = d.n[j];
  uint64_t ktabs = 0;
  for (int ax = off; ax < 3; ++ax) ktabs += 2 * (uint64_t)n3[ax] * 16;
  // blocks of the last pass of a step, with the launch shapes the class will use
  int wreq[3], xcd[3], order[3], plan[3], stream[3];
  effective_tuning(d, wreq, xcd, order, plan, stream);
  int last = -1;
  for (int j = 0; j < 3; ++j)
    if (order[j] >= off) last = order[j];
  // (the batched slot passes are register-heavy: narrow shapes)
  const long long bpg = gpe::pass_shape(d.precision, n3, last, wreq[last], plan[last], true).blocks;
  return context_bytes(d, false) + ktabs +
         (uint64_t)max_slots * (sizeof(gpe::Slot) + sizeof(int)) +
         (uint64_t)max_slots * bpg * gpe::kRedSlots * sizeof(double);
}

ShapeClass *find_class(gpe_server *s, const ClassKey &k) {
  for (ShapeClass *c : s->classes)
    if (c->key == k) return c;
  return nullptr;
}

// Step k of a chunk of class c on the class stream (slot step = steps_done + k).
gpe_status enqueue_step(gpe_server *s, ShapeClass *c, int k) {
  gpe_ctx *p = c->proto;
  const int na = n_axes(p);
  const int rows = c->use_graph ? c->S : c->rows;
  if (rows == 0) return GPE_OK;
  for (int i = 0; i < na; ++i) {
    const int ax = order_axis(p, i);
    gpe::PassArgs a = base_args(p, ax);
    a.mid = gpe::MID_TABLE;
    a.slots = c->d;
    a.slot_map = c->use_graph ? nullptr : c->d_map;
    a.nslots = rows;
    a.slot_pass = (i == 0 ? gpe::SLOT_PASS_FIRST : 0) | (i == na - 1 ? gpe::SLOT_PASS_LAST : 0);
    a.dt = c->key.dt;
    a.mtab = c->kreal[ax];
    a.mtab_imag = c->kimag[ax];
    a.partial = c->partial;
    a.slot_step = k;
    a.slot_imag = c->key.mode == 1;
    if (gpe::launch_axis_pass(p->prec, a, c->strm) != hipSuccess) return GPE_EDEVICE;
  }
  if (c->key.mode != 1) return GPE_OK;  // real time: nothing to renormalise
  return gpe::launch_slot_update(c->d, c->S, c->partial, c->bpg_last, p->dV, k, c->strm) ==
                 hipSuccess
             ? GPE_OK
             : GPE_EDEVICE;
}

// Steps to give class c in this scheduling pass (gpe_sched::chunk_steps).
int steps_for(gpe_server *s, ShapeClass *c) {
  gpe_sched::ChunkInput in;
  in.running = c->running;
  in.step_ms = c->step_ms;
  in.step_running = c->step_running;
  in.use_graph = c->use_graph;
  in.paced = c->paced;
  in.chunk = s->chunk;
  in.quantum_ms = s->quantum_ms;
  if (gpe_sched::is_heavy(c->proto->sites, s->heavy_sites)) {
    double w = s->heavy_weight;
    if (s->heavy_share > 0 && s->heavy_share < 1) {
      const int lights = s->running - s->running_heavy;
      w = std::max(w, s->heavy_share / (1 - s->heavy_share) * lights);
    }
    in.quantum_ms *= w;
  }
  in.main_round_ms = s->main_round_ms;
  in.sites = (double)c->proto->sites;
  in.esize = (double)c->proto->esize;
  return gpe_sched::chunk_steps(in);
}

gpe_status run_chunk(gpe_server *s, ShapeClass *c, int steps) {
  if (!c->use_graph) {
    if (c->map_dirty) {
      gpe::SlotMap m;
      m.n = 0;
      for (int i = 0; i < c->S; ++i)
        if (c->owner[i]) m.idx[m.n++] = i;
      if (m.n > 0 && gpe::launch_map_write(c->d_map, m, c->strm) != hipSuccess)
        return GPE_EDEVICE;
      c->rows = m.n;
      c->map_dirty = false;
    }
    if (c->onchip) {
      if (c->rows == 0) return GPE_OK;
      gpe_ctx *p = c->proto;
      gpe::OnchipArgs a{};
      a.slots = c->d;
      a.slot_map = c->d_map;
      a.steps = steps;
      a.rows_first = order_axis(p, 0) == 2 ? 1 : 0;
      a.n = p->n3[2];
      a.dt = c->key.dt;
      a.dV = p->dV;
      for (int j = 0; j < 3; ++j) {
        a.lo[j] = p->lo3[j];
        a.h[j] = p->h3[j];
      }
      a.tw_row = p->tw[2];
      a.tw_col = p->tw[1];
      a.kr_row = c->kreal[2];
      a.kr_col = c->kreal[1];
      a.ki_row = c->kimag[2];
      a.ki_col = c->kimag[1];
      return gpe::launch_onchip(p->prec, a, c->rows, c->strm) == hipSuccess ? GPE_OK
                                                                            : GPE_EDEVICE;
    }
    for (int k = 0; k < steps; ++k) {
      gpe_status st = enqueue_step(s, c, k);
      if (st != GPE_OK) return st;
    }
    return gpe::launch_slot_advance(c->d, c->S, steps, c->strm) == hipSuccess ? GPE_OK
                                                                              : GPE_EDEVICE;
  }
  if (!c->graph) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->strm, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return GPE_EDEVICE;
    gpe_status st = GPE_OK;
    for (int k = 0; k < s->chunk && st == GPE_OK; ++k) st = enqueue_step(s, c, k);
    if (st == GPE_OK && gpe::launch_slot_advance(c->d, c->S, s->chunk, c->strm) != hipSuccess)
      st = GPE_EDEVICE;
    if (hipStreamEndCapture(c->strm, &g) != hipSuccess || st != GPE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return GPE_EDEVICE;
    }
    const hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return GPE_EDEVICE;
    }
  }
  for (int k = 0; k < steps; k += s->chunk)
    if (hipGraphLaunch(c->graph, c->strm) != hipSuccess) return GPE_EDEVICE;
  return GPE_OK;
}

gpe_status create_class(gpe_server *s, const gpe_request &r, ShapeClass **out) {
  ShapeClass *c = new ShapeClass();
  c->key = key_of(r);
  c->S = s->max_slots;
  gpe_desc d = r.desc;
  gpe_status st = create_context(&d, nullptr, nullptr, s->stream, false, &c->proto);
  if (st != GPE_OK) {
    destroy_class(s, c);
    return st;
  }
  gpe_ctx *p = c->proto;
  for (int i = 0; i < n_axes(p); ++i) {
    const int ax = order_axis(p, i);
    if ((st = get_table(p, ax, TB_KREAL, r.dt, &c->kreal[ax])) != GPE_OK ||
        (st = get_table(p, ax, TB_KIMAG, r.dt, &c->kimag[ax])) != GPE_OK) {
      destroy_class(s, c);
      return st;
    }
  }
  const int last = order_axis(p, n_axes(p) - 1);
  c->bpg_last = gpe::pass_shape(p->prec, p->n3, last, p->wreq[last], p->plan[last], true).blocks;
  // Graph replay over all slots pays for the empty rows' dispatch, which is
  // negligible for small grids (where launch latency dominates) and not for
  // large ones.
  c->onchip = s->use_onchip && p->dim == 2 && p->n3[1] == p->n3[2] &&
              p->n3[2] <= s->onchip_max_n && gpe::onchip_supported(p->prec, p->n3[2]);
  c->use_graph = !c->onchip && s->use_graph && p->sites * c->S <= (1LL << 22);
  const bool heavy_beside = s->heavy_beside && gpe_sched::is_heavy(p->sites, s->heavy_sites);
  c->paced = c->onchip || heavy_beside;
  c->strm = c->onchip ? s->side : heavy_beside ? s->heavy : s->stream;
  c->owner.assign(c->S, 0);
  c->sstate.assign(c->S, SS_FREE);
  c->steps_total.assign(c->S, 0);
  c->admit_round.assign(c->S, 0);
  c->drain_until.assign(c->S, 0);
  c->drain_status.assign(c->S, GPE_OK);
  c->ctx.assign(c->S, nullptr);
  const size_t pbytes = (size_t)c->S * c->bpg_last * gpe::kRedSlots * sizeof(double);
  const size_t tbytes = (size_t)c->S * sizeof(gpe::Slot);
  std::vector<gpe::Slot> zero(c->S, gpe::Slot{});
  bool ok = hipMalloc(&c->d, tbytes) == hipSuccess &&
            hipMalloc(&c->partial, pbytes) == hipSuccess &&
            hipMalloc(&c->d_map, c->S * sizeof(int)) == hipSuccess &&
            hipHostMalloc((void **)&c->hp[0], tbytes, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&c->hp[1], tbytes, hipHostMallocDefault) == hipSuccess;
  for (int q = 0; ok && q < 2; ++q)
    ok = hipEventCreate(&c->ev0[q]) == hipSuccess && hipEventCreate(&c->ev1[q]) == hipSuccess;
  ok = ok && hipMemcpy(c->d, zero.data(), tbytes, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    destroy_class(s, c);
    return GPE_ENOMEM;
  }
  c->fixed_bytes = p->dev_bytes + c->S * (sizeof(gpe::Slot) + sizeof(int)) + pbytes;
  s->used += c->fixed_bytes;
  s->classes.push_back(c);
  *out = c;
  return GPE_OK;
}

// Make room for `need` more bytes: free idle slot contexts first, then whole
// idle shape classes other than `keep` (the requester's own).
void reclaim(gpe_server *s, uint64_t need, const ClassKey &keep) {
  for (ShapeClass *c : s->classes) {
    for (int i = 0; i < c->S && s->used + need > s->budget; ++i) {
      if (c->owner[i] == 0 && c->ctx[i]) {
        s->used -= c->ctx[i]->dev_bytes;
        gpe_destroy(c->ctx[i]);
        c->ctx[i] = nullptr;
      }
    }
  }
  for (size_t k = 0; k < s->classes.size() && s->used + need > s->budget;) {
    ShapeClass *c = s->classes[k];
    if (c->owned == 0 && !(c->key == keep)) {
      s->used -= c->fixed_bytes;
      destroy_class(s, c);
      s->classes.erase(s->classes.begin() + k);
    } else {
      ++k;
    }
  }
}

void finish(gpe_server *s, Req *r, gpe_status st) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->state = RQ_DONE;
  r->t_done = now_s(s);
  r->psi0_d.clear();
  r->psi0_d.shrink_to_fit();
  r->psi0_f.clear();
  r->psi0_f.shrink_to_fit();
  ++s->completed;
  if (st == GPE_OK) s->site_steps += (double)sites_of(r->r.desc) * (double)r->steps_done;
  s->cv_done.notify_all();
}

Req *req_of(gpe_server *s, uint64_t id) {
  std::lock_guard<std::mutex> lk(s->mu);
  return s->reqs[id].get();
}

// GPU setup of an admitted request: class, slot context, state, slot entry.
gpe_status admit(gpe_server *s, Req *r, long long round) {
  ShapeClass *c = find_class(s, key_of(r->r));
  gpe_status st = GPE_OK;
  if (!c && (st = create_class(s, r->r, &c)) != GPE_OK) return st;
  int i = -1;
  for (int j = 0; j < c->S; ++j)
    if (c->sstate[j] == SS_FREE && (i < 0 || (c->ctx[j] && !c->ctx[i]))) i = j;  // warm first
  if (i < 0) return GPE_EBUSY;
  if (!c->ctx[i]) {
    gpe_desc d = r->r.desc;
    if ((st = create_context(&d, nullptr, &r->r.trap, s->aux, true, &c->ctx[i])) != GPE_OK)
      return st;
    s->used += c->ctx[i]->dev_bytes;
  } else {
    c->ctx[i]->desc = r->r.desc;
    if ((st = set_potential(c->ctx[i], nullptr, &r->r.trap)) != GPE_OK) return st;
  }
  gpe_ctx *x = c->ctx[i];
  const void *src = gpe::state_f32(x->prec) ? (const void *)r->psi0_f.data()
                                        : (const void *)r->psi0_d.data();
  if (hipMemcpyAsync(x->psi, src, x->sites * x->esize, hipMemcpyHostToDevice, s->aux) !=
          hipSuccess ||
      hipEventRecord(s->ev_up, s->aux) != hipSuccess ||
      hipStreamWaitEvent(c->strm, s->ev_up, 0) != hipSuccess)
    return GPE_EDEVICE;
  gpe::Slot sl{};
  sl.psi = x->psi;
  sl.g = r->r.desc.g;
  for (int j = 0; j < 3; ++j) sl.hv[j] = x->hv[j];
  sl.mode = r->r.mode == 1 ? gpe::SLOT_IMAG : gpe::SLOT_REAL;
  sl.steps_total = (int)r->r.nsteps;
  sl.steps_done = 0;
  sl.scale = 1.0;
  sl.norm_target = r->r.desc.norm_target;
  if (gpe::launch_slot_write(c->d + i, sl, c->strm) != hipSuccess) return GPE_EDEVICE;
  c->owner[i] = r->id;
  c->sstate[i] = SS_RUN;
  c->steps_total[i] = sl.steps_total;
  c->admit_round[i] = round;
  ++c->owned;
  ++c->running;
  c->map_dirty = true;
  return GPE_OK;
}

// Clear slot i's table entry on the main stream (after the chunks already
// enqueued; later chunks skip the slot).
void clear_entry(gpe_server *s, ShapeClass *c, int i) {
  gpe::Slot sl{};
  sl.mode = gpe::SLOT_FREE;
  (void)gpe::launch_slot_write(c->d + i, sl, c->strm);
}

void release(gpe_server *s, ShapeClass *c, int i, const Req *r) {
  if (c->sstate[i] == SS_RUN) --c->running;
  c->owner[i] = 0;
  c->sstate[i] = SS_FREE;
  --c->owned;
  c->map_dirty = true;
  std::lock_guard<std::mutex> lk(s->mu);
  --s->running;
  if (r->heavy) --s->running_heavy;
}

// Slot i finished its steps (seen in a read-back): final scaling, observables
// and state download on the side stream, then the slot is free.  The chunk
// now in flight skips the slot, so none of this races with it.
void complete(gpe_server *s, ShapeClass *c, int i, Req *r) {
  gpe_ctx *x = c->ctx[i];
  r->steps_done = c->steps_total[i];
  gpe_status st = GPE_OK;
  if (r->r.mode == 1 && r->steps_done > 0) {
    double *scale_dev = reinterpret_cast<double *>(reinterpret_cast<char *>(c->d + i) +
                                                   offsetof(gpe::Slot, scale));
    if (gpe::launch_scale(x->prec, x->psi, x->sites, scale_dev, s->aux) != hipSuccess)
      st = GPE_EDEVICE;
  }
  gpe_obs o{};
  if (st == GPE_OK) st = compute_obs(x, nullptr, &o);
  r->obs = o;
  if ((st == GPE_OK || st == GPE_ENONFINITE) && r->r.keep_state) {
    r->psi_out.resize(2 * (size_t)x->sites);
    if (gpe_get_state(x, r->psi_out.data()) != GPE_OK) st = GPE_EDEVICE;
  }
  clear_entry(s, c, i);
  release(s, c, i, r);
  finish(s, r, st);
}

// Start draining slot i: clear its entry now, release it once the chunk of
// round `until` (the last one that may still touch it) is known done.
void drain(gpe_server *s, ShapeClass *c, int i, long long until, gpe_status why) {
  clear_entry(s, c, i);
  if (c->sstate[i] == SS_RUN) --c->running;
  c->sstate[i] = SS_DRAIN;
  c->drain_until[i] = until;
  c->drain_status[i] = why;
}

// The chunk of round q is done and its slot tables are on the host: update
// the step-time estimates, finish completed requests, start or end drains.
// `now` is the round whose chunk is in flight.
void retire(gpe_server *s, long long q, long long now) {
  const int par = (int)(q & 1);
  double main_ms = 0;
  for (ShapeClass *c : s->classes) {
    if (!c->hp_valid[par]) continue;
    c->hp_valid[par] = false;
    float ms = 0;
    if (!c->failed[par] && c->timed_steps[par] > 0 &&
        hipEventElapsedTime(&ms, c->ev0[par], c->ev1[par]) == hipSuccess && ms > 0) {
      c->step_ms = ms / c->timed_steps[par];
      c->step_running = c->timed_running[par];
      if (c->strm == s->stream) main_ms += ms;
    }
    for (int i = 0; i < c->S; ++i) {
      if (!c->owner[i]) continue;
      Req *r = req_of(s, c->owner[i]);
      if (c->sstate[i] == SS_DRAIN) {
        if (q >= c->drain_until[i]) {
          const gpe_status why = c->drain_status[i];
          r->steps_done = std::min<int64_t>(r->steps_done, c->steps_total[i]);
          release(s, c, i, r);
          finish(s, r, why);
        }
        continue;
      }
      if (c->admit_round[i] > q) continue;  // the read-back predates this request
      r->steps_done = c->hp[par][i].steps_done;
      if (c->failed[par]) {
        drain(s, c, i, now, GPE_EDEVICE);
      } else if (r->cancel) {
        drain(s, c, i, now, GPE_ECANCELED);
      } else if (c->hp[par][i].steps_done >= c->steps_total[i]) {
        complete(s, c, i, r);
      }
    }
  }
  s->main_round_ms = main_ms;
}

// Admit queued requests in arrival order, one at a time, so that the bytes
// charged for each are known before the next decision (gpe_sched::admit_decision:
// a heavy request waiting for its tier lets the requests behind it pass).
void admit_queued(gpe_server *s, long long round) {
  size_t at = 0;  // queue position: entries before it wait for the heavy tier
  for (;;) {
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop || at >= s->queue.size()) return;
    Req *r = s->reqs[s->queue[at]].get();
    if (r->cancel) {
      s->queue.erase(s->queue.begin() + at);
      r->state = RQ_DONE;
      r->status = GPE_ECANCELED;
      r->t_done = now_s(s);
      ++s->completed;
      s->cv_done.notify_all();
      continue;
    }
    ShapeClass *c = find_class(s, key_of(r->r));
    bool warm = false, free_slot = c == nullptr;
    if (c)
      for (int j = 0; j < c->S; ++j)
        if (c->sstate[j] == SS_FREE) {
          free_slot = true;
          warm = warm || c->ctx[j] != nullptr;
        }
    gpe_sched::AdmitInput in;
    in.heavy = r->heavy;
    in.running = s->running;
    in.max_active = s->max_active;
    in.running_heavy = s->running_heavy;
    in.heavy_active = s->heavy_active;
    in.free_slot = free_slot;
    in.need = (warm ? 0 : r->need) + (c ? 0 : r->need_class);
    in.used = s->used;
    in.budget = s->budget;
    gpe_sched::Admit d = gpe_sched::admit_decision(in);
    if (d == gpe_sched::kStop && free_slot && in.used + in.need > in.budget) {
      reclaim(s, in.need, key_of(r->r));
      in.used = s->used;
      d = gpe_sched::admit_decision(in);
    }
    if (d == gpe_sched::kSkip) {
      ++at;
      continue;
    }
    if (d == gpe_sched::kStop) return;
    s->queue.erase(s->queue.begin() + at);
    r->state = RQ_RUNNING;
    r->t_start = now_s(s);
    ++s->running;
    if (r->heavy) ++s->running_heavy;
    lk.unlock();
    const gpe_status st = admit(s, r, round);
    if (st != GPE_OK) {
      {
        std::lock_guard<std::mutex> lk2(s->mu);
        --s->running;
        if (r->heavy) --s->running_heavy;
      }
      finish(s, r, st == GPE_EBUSY ? GPE_EDEVICE : st);
    }
  }
}

void scheduler(gpe_server *s) {
  (void)hipSetDevice(s->device);
  long long round = 0;
  bool pending = false;  // the previous round enqueued a chunk not yet retired
  for (;;) {
    const auto tb = std::chrono::steady_clock::now();
    admit_queued(s, round);
    const int par = (int)(round & 1);
    bool any = false;
    s->used_main[par] = s->used_side[par] = s->used_heavy[par] = false;
    for (ShapeClass *c : s->classes) {
      c->hp_valid[par] = false;
      if (!c->owned) continue;
      any = true;
      (c->strm == s->side ? s->used_side : c->strm == s->heavy ? s->used_heavy : s->used_main)[par] =
          true;
      const int steps = steps_for(s, c);
      (void)hipEventRecord(c->ev0[par], c->strm);
      c->failed[par] = run_chunk(s, c, steps) != GPE_OK;
      (void)hipEventRecord(c->ev1[par], c->strm);
      c->timed_steps[par] = steps;
      c->timed_running[par] = c->running;
      (void)hipMemcpyAsync(c->hp[par], c->d, c->S * sizeof(gpe::Slot), hipMemcpyDeviceToHost,
                           c->strm);
      c->hp_valid[par] = true;
    }
    if (s->used_main[par]) (void)hipEventRecord(s->done[par], s->stream);
    if (s->used_side[par]) (void)hipEventRecord(s->done_side[par], s->side);
    if (s->used_heavy[par]) (void)hipEventRecord(s->done_heavy[par], s->heavy);
    if (pending) {
      if (s->used_main[par ^ 1]) (void)hipEventSynchronize(s->done[par ^ 1]);
      if (s->used_side[par ^ 1]) (void)hipEventSynchronize(s->done_side[par ^ 1]);
      if (s->used_heavy[par ^ 1]) (void)hipEventSynchronize(s->done_heavy[par ^ 1]);
      retire(s, round - 1, round);
    }
    pending = any;
    ++round;
    std::unique_lock<std::mutex> lk(s->mu);
    if (any || s->running > 0)
      s->busy += std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
    if (s->stop) break;
    if (!pending && s->running == 0)
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    if (s->stop) break;
  }
  // Shutting down: let the GPU finish, then cancel whatever is still held.
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->side);
  (void)hipStreamSynchronize(s->heavy);
  (void)hipStreamSynchronize(s->aux);
  for (ShapeClass *c : s->classes)
    for (int i = 0; i < c->S; ++i)
      if (c->owner[i]) {
        Req *r = req_of(s, c->owner[i]);
        release(s, c, i, r);
        finish(s, r, GPE_ECANCELED);
      }
}

// Free everything the server holds (the scheduler thread has ended).
void release_server(gpe_server *s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->side) (void)hipStreamSynchronize(s->side);
  if (s->heavy) (void)hipStreamSynchronize(s->heavy);
  if (s->aux) (void)hipStreamSynchronize(s->aux);
  for (ShapeClass *c : s->classes) destroy_class(s, c);
  s->classes.clear();
  for (hipEvent_t e : {s->done[0], s->done[1], s->done_side[0], s->done_side[1],
                       s->done_heavy[0], s->done_heavy[1], s->ev_up})
    if (e) (void)hipEventDestroy(e);
  if (s->aux) (void)hipStreamDestroy(s->aux);
  if (s->heavy) (void)hipStreamDestroy(s->heavy);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

gpe_status gpe_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t max_active,
                             int32_t chunk_steps, gpe_server **out) {
  if (!out || max_slots < 1 || max_active < 0 || chunk_steps < 1) return GPE_EINVAL;
  *out = nullptr;
  if (max_slots > gpe::kMaxSlots) return GPE_EUNSUPPORTED;
  gpe_server *s = new gpe_server();
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->heavy, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->done_side[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->done_side[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->done_heavy[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->done_heavy[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->done[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->done[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_up, hipEventDisableTiming) != hipSuccess) {
    release_server(s);
    return GPE_EDEVICE;
  }
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  s->max_slots = max_slots;
  s->max_active = max_active;
  s->chunk = chunk_steps;
  // Experiment overrides: graph replay for small classes, on-chip classes,
  // GPU time per running request per round.
  if (const char *g = std::getenv("GPE_SERVER_GRAPH")) s->use_graph = std::atoi(g) != 0;
  if (const char *o = std::getenv("GPE_SERVER_ONCHIP")) s->use_onchip = std::atoi(o) != 0;
  if (const char *o = std::getenv("GPE_SERVER_ONCHIP_MAX_N")) {
    const int v = std::atoi(o);
    if (v > 0) s->onchip_max_n = v;
  }
  if (const char *q = std::getenv("GPE_SERVER_QUANTUM_MS")) {
    const double v = std::atof(q);
    if (v > 0) s->quantum_ms = v;
  }
  if (const char *h = std::getenv("GPE_SERVER_HEAVY_SITES")) s->heavy_sites = std::atoll(h);
  if (const char *h = std::getenv("GPE_SERVER_HEAVY_ACTIVE")) s->heavy_active = std::atoi(h);
  if (const char *h = std::getenv("GPE_SERVER_HEAVY_WEIGHT")) {
    const double v = std::atof(h);
    if (v > 0) s->heavy_weight = v;
  }
  if (const char *h = std::getenv("GPE_SERVER_HEAVY_SHARE")) {
    const double v = std::atof(h);
    if (v >= 0 && v < 1) s->heavy_share = v;
  }
  if (const char *h = std::getenv("GPE_SERVER_HEAVY_BESIDE")) s->heavy_beside = std::atoi(h) != 0;
  s->t0 = std::chrono::steady_clock::now();
  s->th = std::thread(scheduler, s);
  *out = s;
  return GPE_OK;
}

gpe_status gpe_server_submit(gpe_server *s, const gpe_request *req, uint64_t *id) {
  if (!s || !req || !id || !req->psi0) return GPE_EINVAL;
  const gpe_desc &d = req->desc;
  if (d.dim == 1) return GPE_EUNSUPPORTED;  // batched classes are 2D and 3D
  if (d.dim != 2 && d.dim != 3) return GPE_EINVAL;
  for (int j = 0; j < d.dim; ++j) {
    if (d.n[j] < 8 || d.n[j] > 1024 || (d.n[j] & (d.n[j] - 1))) return GPE_EUNSUPPORTED;
    if (!(d.hi[j] > d.lo[j])) return GPE_EINVAL;
  }
  if (!std::isfinite(d.g) ||
      (d.precision != GPE_FP64 && d.precision != GPE_FP32 && d.precision != GPE_FP32_STATE) ||
      !(d.norm_target > 0) || !(req->dt > 0) || !std::isfinite(req->dt) || req->nsteps < 0 ||
      req->nsteps > 2000000000 || (req->mode != 0 && req->mode != 1))
    return GPE_EINVAL;
  auto r = std::make_unique<Req>();
  r->r = *req;
  r->r.psi0 = nullptr;
  const size_t nreal = 2 * (size_t)sites_of(d);
  if (gpe::state_f32(d.precision)) {
    r->psi0_f.resize(nreal);
    for (size_t i = 0; i < nreal; ++i) r->psi0_f[i] = (float)req->psi0[i];
  } else {
    r->psi0_d.assign(req->psi0, req->psi0 + nreal);
  }
  r->need = context_bytes(d);
  r->need_class = class_bytes(d, s->max_slots);
  r->heavy = gpe_sched::is_heavy(sites_of(d), s->heavy_sites);
  if (r->need + r->need_class > s->budget) return GPE_ENOMEM;
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t_submit = now_s(s);
  *id = r->id;
  s->queue.push_back(r->id);
  s->reqs[r->id] = std::move(r);
  ++s->submitted;
  s->cv_work.notify_one();
  return GPE_OK;
}

gpe_status gpe_server_poll(gpe_server *s, uint64_t id, gpe_result *out, double *psi_out) {
  if (!s || !out) return GPE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return GPE_EINVAL;
  Req *r = it->second.get();
  if (r->state != RQ_DONE) return GPE_EBUSY;
  out->status = r->status;
  out->obs = r->obs;
  out->t_submit = r->t_submit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  out->steps_done = r->steps_done;
  if (psi_out) {
    if (r->psi_out.empty()) return GPE_EINVAL;
    std::memcpy(psi_out, r->psi_out.data(), r->psi_out.size() * sizeof(double));
  }
  return GPE_OK;
}

gpe_status gpe_server_cancel(gpe_server *s, uint64_t id) {
  if (!s) return GPE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return GPE_EINVAL;
  it->second->cancel = true;
  s->cv_work.notify_one();
  return GPE_OK;
}

gpe_status gpe_server_release(gpe_server *s, uint64_t id) {
  if (!s) return GPE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return GPE_EINVAL;
  if (it->second->state != RQ_DONE) return GPE_EBUSY;
  s->reqs.erase(it);
  return GPE_OK;
}

gpe_status gpe_server_wait_idle(gpe_server *s) {
  if (!s) return GPE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->completed >= s->submitted || s->stop; });
  return GPE_OK;
}

gpe_status gpe_request_bytes(const gpe_desc *desc, int32_t max_slots, uint64_t *class_b,
                             uint64_t *slot_b) {
  if (!desc || max_slots < 1 || desc->dim < 1 || desc->dim > 3) return GPE_EINVAL;
  if (desc->dim == 1) return GPE_EUNSUPPORTED;
  for (int j = 0; j < desc->dim; ++j)
    if (desc->n[j] < 8 || desc->n[j] > 1024 || (desc->n[j] & (desc->n[j] - 1)))
      return GPE_EUNSUPPORTED;
  if (class_b) *class_b = class_bytes(*desc, max_slots);
  if (slot_b) *slot_b = context_bytes(*desc);
  return GPE_OK;
}

gpe_status gpe_server_stats_read(gpe_server *s, gpe_server_stats *out) {
  if (!s || !out) return GPE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->running = s->running;
  out->queued = (int64_t)s->queue.size();
  out->busy_seconds = s->busy;
  out->site_steps = s->site_steps;
  out->bytes_in_use = s->used;
  return GPE_OK;
}

void gpe_server_destroy(gpe_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto &kv : s->reqs)
      if (kv.second->state != RQ_DONE) kv.second->cancel = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  release_server(s);
}

}  // extern "C"
