// Serving scheduler behind the gpe_server_* calls of include/gpe.h.
//
// One scheduler thread owns every GPU call.  Requests wait in arrival order;
// the head is admitted while the HBM budget allows and a slot of its shape
// class (dim, n, precision, box, dt) is free.  Every class keeps a
// device-resident slot table; one chunk of steps runs all active slots of a
// class in the same batched launches (the fused axis passes in slot mode, then
// a slot-update kernel), replayed from a HIP graph captured once per class.
// Slots that are free or finished return at once, so admissions and
// completions never change the launches.  After each chunk the scheduler reads
// the slot table back, finishes the requests whose steps are done (final
// imaginary-time scaling, observables, optional state copy) and frees their
// slots for the queue.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gpe_ctx.h"

using namespace gpe_host;

namespace {

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Req {
  uint64_t id = 0;
  gpe_request r{};
  std::vector<double> psi0;
  ReqState state = RQ_QUEUED;
  gpe_status status = GPE_EBUSY;
  gpe_obs obs{};
  double t_submit = 0, t_start = 0, t_done = 0;
  int64_t steps_done = 0;
  std::vector<double> psi_out;
  bool cancel = false;
  uint64_t need = 0;        // device bytes a fresh slot context takes
  uint64_t need_class = 0;  // device bytes a new shape class takes
  int cls = -1, slot = -1;
};

struct ClassKey {
  int dim, n[3], prec;
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
  return k;
}

struct ShapeClass {
  ClassKey key{};
  int S = 0;
  gpe_ctx *proto = nullptr;           // owns the class tables
  std::vector<gpe_ctx *> ctx;         // per slot, kept for reuse while memory allows
  std::vector<gpe::Slot> h;           // host mirror of the slot table
  gpe::Slot *d = nullptr;             // device slot table
  std::vector<uint64_t> owner;        // request id per slot (0: free)
  double *partial = nullptr;          // norm partials, S x blocks of the last pass
  long long bpg_last = 0;
  void *kreal[3] = {nullptr, nullptr, nullptr}, *kimag[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t graph = nullptr;
  bool use_graph = false;             // small grids: replay chunks from a graph over all slots
  int *d_map = nullptr;               // large grids: launch rows for the active slots only
  std::vector<int> h_map;
  bool map_dirty = true;
  int active = 0;
  bool failed = false;                // a chunk failed to launch this round
  uint64_t fixed_bytes = 0;           // proto context + slot table + partials
};

void destroy_class(ShapeClass *c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  for (gpe_ctx *x : c->ctx)
    if (x) gpe_destroy(x);
  if (c->proto) gpe_destroy(c->proto);
  if (c->d) (void)hipFree(c->d);
  if (c->partial) (void)hipFree(c->partial);
  if (c->d_map) (void)hipFree(c->d_map);
  delete c;
}

}  // namespace

struct gpe_server {
  hipStream_t stream = nullptr;
  int device = 0;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  int max_slots = 1, max_active = 0, chunk = 16;
  bool use_graph = true;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<ShapeClass *> classes;  // touched by the scheduler thread only
  uint64_t next_id = 1;
  int running = 0;
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

// Device bytes a shape class holds besides its slot contexts: the prototype
// context, its two kinetic tables per axis, the slot table and norm partials.
uint64_t class_bytes(const gpe_desc &d, int max_slots) {
  int n3[3] = {1, 1, 1};
  const int off = 3 - d.dim;
  for (int j = 0; j < d.dim; ++j) n3[j + off] = d.n[j];
  uint64_t ktabs = 0;
  for (int ax = off; ax < 3; ++ax) ktabs += 2 * (uint64_t)n3[ax] * 16;
  const int wlast = 16;  // the last pass of the default order is axis 0 (3D) or 1 (2D)
  const int last = off;
  const long long bpg =
      gpe::pass_shape(d.precision, n3, last, last == 0 ? wlast : (d.precision == GPE_FP32 ? 16 : 8))
          .blocks;
  return context_bytes(d) + ktabs + (uint64_t)max_slots * (sizeof(gpe::Slot) + sizeof(int)) +
         (uint64_t)max_slots * bpg * gpe::kRedSlots * sizeof(double);
}

ShapeClass *find_class(gpe_server *s, const ClassKey &k) {
  for (ShapeClass *c : s->classes)
    if (c->key == k) return c;
  return nullptr;
}

// Enqueue one batched step of class c on the server stream: graph classes
// launch a row per slot (free or finished rows return at once); the others a
// row per active slot through the slot map.
gpe_status enqueue_step(gpe_server *s, ShapeClass *c) {
  gpe_ctx *p = c->proto;
  const int na = n_axes(p);
  const int rows = c->use_graph ? c->S : (int)c->h_map.size();
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
    hipError_t e = gpe::launch_axis_pass(p->prec, a, s->stream);
    if (e != hipSuccess) return GPE_EDEVICE;
  }
  return gpe::launch_slot_update(c->d, c->S, c->partial, c->bpg_last, p->dV, s->stream) ==
                 hipSuccess
             ? GPE_OK
             : GPE_EDEVICE;
}

gpe_status run_chunk(gpe_server *s, ShapeClass *c) {
  if (!c->use_graph) {
    if (c->map_dirty) {
      c->h_map.clear();
      for (int i = 0; i < c->S; ++i)
        if (c->owner[i]) c->h_map.push_back(i);
      if (!c->h_map.empty() &&
          hipMemcpyAsync(c->d_map, c->h_map.data(), c->h_map.size() * sizeof(int),
                         hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return GPE_EDEVICE;
      c->map_dirty = false;
    }
    for (int k = 0; k < s->chunk; ++k) {
      gpe_status st = enqueue_step(s, c);
      if (st != GPE_OK) return st;
    }
    return GPE_OK;
  }
  if (!c->graph) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return GPE_EDEVICE;
    gpe_status st = GPE_OK;
    for (int k = 0; k < s->chunk && st == GPE_OK; ++k) st = enqueue_step(s, c);
    if (hipStreamEndCapture(s->stream, &g) != hipSuccess || st != GPE_OK) {
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
  return hipGraphLaunch(c->graph, s->stream) == hipSuccess ? GPE_OK : GPE_EDEVICE;
}

gpe_status create_class(gpe_server *s, const gpe_request &r, ShapeClass **out) {
  ShapeClass *c = new ShapeClass();
  c->key = key_of(r);
  c->S = s->max_slots;
  gpe_desc d = r.desc;
  gpe_status st = gpe_create(&d, nullptr, nullptr, s->stream, &c->proto);
  if (st != GPE_OK) {
    destroy_class(c);
    return st;
  }
  gpe_ctx *p = c->proto;
  for (int i = 0; i < n_axes(p); ++i) {
    const int ax = order_axis(p, i);
    if ((st = get_table(p, ax, TB_KREAL, r.dt, &c->kreal[ax])) != GPE_OK ||
        (st = get_table(p, ax, TB_KIMAG, r.dt, &c->kimag[ax])) != GPE_OK) {
      destroy_class(c);
      return st;
    }
  }
  const int last = order_axis(p, n_axes(p) - 1);
  c->bpg_last = gpe::pass_shape(p->prec, p->n3, last, p->wreq[last]).blocks;
  // Graph replay over all slots pays for the empty rows' dispatch, which is
  // negligible for small grids (where launch latency dominates) and not for
  // large ones.
  c->use_graph = s->use_graph && p->sites * c->S <= (1LL << 22);
  c->h.assign(c->S, gpe::Slot{});
  c->owner.assign(c->S, 0);
  c->ctx.assign(c->S, nullptr);
  const size_t pbytes = (size_t)c->S * c->bpg_last * gpe::kRedSlots * sizeof(double);
  if (hipMalloc(&c->d, c->S * sizeof(gpe::Slot)) != hipSuccess ||
      hipMalloc(&c->partial, pbytes) != hipSuccess ||
      hipMalloc(&c->d_map, c->S * sizeof(int)) != hipSuccess ||
      hipMemcpyAsync(c->d, c->h.data(), c->S * sizeof(gpe::Slot), hipMemcpyHostToDevice,
                     s->stream) != hipSuccess) {
    destroy_class(c);
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
    if (c->active == 0 && !(c->key == keep)) {
      s->used -= c->fixed_bytes;
      destroy_class(c);
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
  r->psi0.clear();
  r->psi0.shrink_to_fit();
  ++s->completed;
  if (st == GPE_OK) s->site_steps += (double)sites_of(r->r.desc) * (double)r->steps_done;
  s->cv_done.notify_all();
}

// GPU setup of an admitted request: class, slot context, state, slot entry.
gpe_status admit(gpe_server *s, Req *r) {
  ShapeClass *c = find_class(s, key_of(r->r));
  gpe_status st = GPE_OK;
  if (!c && (st = create_class(s, r->r, &c)) != GPE_OK) return st;
  int i = -1;
  for (int j = 0; j < c->S; ++j)
    if (c->owner[j] == 0 && (i < 0 || (c->ctx[j] && !c->ctx[i]))) i = j;  // prefer a warm slot
  if (i < 0) return GPE_EBUSY;
  if (!c->ctx[i]) {
    gpe_desc d = r->r.desc;
    if ((st = gpe_create(&d, nullptr, &r->r.trap, s->stream, &c->ctx[i])) != GPE_OK) return st;
    s->used += c->ctx[i]->dev_bytes;
  } else {
    c->ctx[i]->desc = r->r.desc;
    if ((st = set_potential(c->ctx[i], nullptr, &r->r.trap)) != GPE_OK) return st;
  }
  gpe_ctx *x = c->ctx[i];
  if ((st = gpe_set_state(x, r->psi0.data())) != GPE_OK) return st;
  gpe::Slot &sl = c->h[i];
  sl = gpe::Slot{};
  sl.psi = x->psi;
  sl.g = r->r.desc.g;
  for (int j = 0; j < 3; ++j) sl.hv[j] = x->hv[j];
  sl.mode = r->r.mode == 1 ? gpe::SLOT_IMAG : gpe::SLOT_REAL;
  sl.steps_total = (int)r->r.nsteps;
  sl.steps_done = 0;
  sl.scale = 1.0;
  sl.norm_target = r->r.desc.norm_target;
  if (hipMemcpyAsync(c->d + i, &sl, sizeof(gpe::Slot), hipMemcpyHostToDevice, s->stream) !=
      hipSuccess)
    return GPE_EDEVICE;
  c->owner[i] = r->id;
  ++c->active;
  c->map_dirty = true;
  r->cls = (int)(std::find(s->classes.begin(), s->classes.end(), c) - s->classes.begin());
  r->slot = i;
  return GPE_OK;
}

// Request in slot i of class c is done (or cancelled): finish and free the slot.
void complete(gpe_server *s, ShapeClass *c, int i, Req *r, bool cancelled) {
  gpe_ctx *x = c->ctx[i];
  r->steps_done = c->h[i].steps_done;
  gpe_status st = GPE_OK;
  if (c->h[i].mode == gpe::SLOT_IMAG && r->steps_done > 0) {
    double *scale_dev = reinterpret_cast<double *>(reinterpret_cast<char *>(c->d + i) +
                                                   offsetof(gpe::Slot, scale));
    if (gpe::launch_scale(x->prec, x->psi, x->sites, scale_dev, s->stream) != hipSuccess)
      st = GPE_EDEVICE;
  }
  gpe_obs o{};
  if (st == GPE_OK) st = compute_obs(x, nullptr, &o);
  r->obs = o;
  if ((st == GPE_OK || st == GPE_ENONFINITE) && r->r.keep_state) {
    r->psi_out.resize(2 * (size_t)x->sites);
    if (gpe_get_state(x, r->psi_out.data()) != GPE_OK) st = GPE_EDEVICE;
  }
  c->h[i].mode = gpe::SLOT_FREE;
  (void)hipMemcpyAsync(c->d + i, &c->h[i], sizeof(gpe::Slot), hipMemcpyHostToDevice, s->stream);
  c->owner[i] = 0;
  --c->active;
  c->map_dirty = true;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    --s->running;
  }
  finish(s, r, cancelled ? GPE_ECANCELED : st);
}

void scheduler(gpe_server *s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    // Admission, one request at a time and in arrival order, so that the bytes
    // charged for each admitted request are known before the next decision.
    bool admitted_any = false;
    const auto tb = std::chrono::steady_clock::now();
    for (;;) {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop || s->queue.empty()) break;
      Req *r = s->reqs[s->queue.front()].get();
      if (r->cancel) {
        s->queue.pop_front();
        r->state = RQ_DONE;
        r->status = GPE_ECANCELED;
        r->t_done = now_s(s);
        ++s->completed;
        s->cv_done.notify_all();
        continue;
      }
      if (s->max_active > 0 && s->running >= s->max_active) break;
      ShapeClass *c = find_class(s, key_of(r->r));
      if (c && c->active >= c->S) break;
      bool warm = false;
      if (c)
        for (int j = 0; j < c->S; ++j) warm = warm || (c->owner[j] == 0 && c->ctx[j]);
      const uint64_t need = (warm ? 0 : r->need) + (c ? 0 : r->need_class);
      if (s->used + need > s->budget) {
        reclaim(s, need, key_of(r->r));
        if (s->used + need > s->budget) break;
      }
      s->queue.pop_front();
      r->state = RQ_RUNNING;
      r->t_start = now_s(s);
      ++s->running;
      lk.unlock();
      const gpe_status st = admit(s, r);
      if (st != GPE_OK) {
        {
          std::lock_guard<std::mutex> lk2(s->mu);
          --s->running;
        }
        finish(s, r, st == GPE_EBUSY ? GPE_EDEVICE : st);
      }
      admitted_any = true;
    }
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop) break;
      if (!admitted_any && s->running == 0) {
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        continue;
      }
    }
    bool any = false;
    for (ShapeClass *c : s->classes) {
      if (!c->active) continue;
      any = true;
      c->failed = run_chunk(s, c) != GPE_OK;
    }
    for (ShapeClass *c : s->classes)
      if (c->active)
        (void)hipMemcpyAsync(c->h.data(), c->d, c->S * sizeof(gpe::Slot), hipMemcpyDeviceToHost,
                             s->stream);
    (void)hipStreamSynchronize(s->stream);
    for (ShapeClass *c : s->classes) {
      for (int i = 0; i < c->S; ++i) {
        if (!c->owner[i]) continue;
        Req *r;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          r = s->reqs[c->owner[i]].get();
        }
        if (c->failed) {
          c->owner[i] = 0;
          --c->active;
          c->map_dirty = true;
          c->h[i].mode = gpe::SLOT_FREE;
          (void)hipMemcpyAsync(c->d + i, &c->h[i], sizeof(gpe::Slot), hipMemcpyHostToDevice,
                               s->stream);
          {
            std::lock_guard<std::mutex> lk(s->mu);
            --s->running;
          }
          finish(s, r, GPE_EDEVICE);
        } else if (r->cancel || c->h[i].steps_done >= c->h[i].steps_total) {
          complete(s, c, i, r, r->cancel);
        }
      }
    }
    if (any || admitted_any) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->busy += std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
    }
  }
  // shutting down: cancel whatever is still held
  for (ShapeClass *c : s->classes)
    for (int i = 0; i < c->S; ++i)
      if (c->owner[i]) {
        Req *r;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          r = s->reqs[c->owner[i]].get();
        }
        complete(s, c, i, r, true);
      }
}

}  // namespace

extern "C" {

gpe_status gpe_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t max_active,
                             int32_t chunk_steps, gpe_server **out) {
  if (!out || max_slots < 1 || max_active < 0 || chunk_steps < 1) return GPE_EINVAL;
  *out = nullptr;
  gpe_server *s = new gpe_server();
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return GPE_EDEVICE;
  }
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  s->max_slots = max_slots;
  s->max_active = max_active;
  s->chunk = chunk_steps;
  if (const char *g = std::getenv("GPE_SERVER_GRAPH")) s->use_graph = std::atoi(g) != 0;
  s->t0 = std::chrono::steady_clock::now();
  s->th = std::thread(scheduler, s);
  *out = s;
  return GPE_OK;
}

gpe_status gpe_server_submit(gpe_server *s, const gpe_request *req, uint64_t *id) {
  if (!s || !req || !id || !req->psi0) return GPE_EINVAL;
  const gpe_desc &d = req->desc;
  if (d.dim != 2 && d.dim != 3) return GPE_EINVAL;
  for (int j = 0; j < d.dim; ++j) {
    if (d.n[j] < 8 || d.n[j] > 1024 || (d.n[j] & (d.n[j] - 1))) return GPE_EUNSUPPORTED;
    if (!(d.hi[j] > d.lo[j])) return GPE_EINVAL;
  }
  if (!std::isfinite(d.g) || (d.precision != GPE_FP64 && d.precision != GPE_FP32) ||
      !(d.norm_target > 0) || !(req->dt > 0) || !std::isfinite(req->dt) || req->nsteps < 0 ||
      req->nsteps > 2000000000 || (req->mode != 0 && req->mode != 1))
    return GPE_EINVAL;
  auto r = std::make_unique<Req>();
  r->r = *req;
  r->r.psi0 = nullptr;
  r->psi0.assign(req->psi0, req->psi0 + 2 * sites_of(d));
  r->need = context_bytes(d);
  r->need_class = class_bytes(d, s->max_slots);
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

gpe_status gpe_server_wait_idle(gpe_server *s) {
  if (!s) return GPE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->completed >= s->submitted || s->stop; });
  return GPE_OK;
}

gpe_status gpe_request_bytes(const gpe_desc *desc, int32_t max_slots, uint64_t *class_b,
                             uint64_t *slot_b) {
  if (!desc || max_slots < 1 || (desc->dim != 2 && desc->dim != 3)) return GPE_EINVAL;
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
  (void)hipStreamSynchronize(s->stream);
  for (ShapeClass *c : s->classes) destroy_class(c);
  (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
