// Launch-shape tuning per shape class (gpe_autotune and gpe_tuning_* calls).
//
// The fused axis passes have five run-time shape choices: the columns per
// workgroup of each strided axis (8 or 16, i.e. 128- or 256-byte rows in
// FP64), whether each XCD takes a contiguous run of tiles, and the order in
// which a step visits the axes (none changes the arithmetic of a line), the
// radix plan of a 1024-point axis (which changes the rounding only), and
// streaming (non-temporal) loads and stores per axis (cache policy only).
// gpe_autotune times the real-time step over these on the device for one
// shape class (dim, n, precision) by coordinate descent and records the
// fastest in a process-wide table; every context created afterwards for that
// class uses it.  The table is saved to and loaded from a small JSON file.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gpe_ctx.h"

namespace gpe_host {
namespace {

struct TuneKey {
  int dim, n[3], prec;
  bool operator<(const TuneKey &o) const {
    if (dim != o.dim) return dim < o.dim;
    if (prec != o.prec) return prec < o.prec;
    for (int j = 0; j < 3; ++j)
      if (n[j] != o.n[j]) return n[j] < o.n[j];
    return false;
  }
};

TuneKey key_of(const gpe_desc &d) {
  TuneKey k{};
  k.dim = d.dim;
  k.prec = d.precision;
  for (int j = 0; j < 3; ++j) k.n[j] = j < d.dim ? d.n[j] : 1;
  return k;
}

std::mutex g_mu;
std::map<TuneKey, gpe_tuning> g_table;

// Defaults (measured at 512^3 on MI355X): 256-byte rows on the slowest axis,
// 128-byte rows on the middle one in FP64 (64-byte rows of 16 columns in FP32),
// contiguous tile runs per XCD on the strided axes, slowest axis last.
void defaults(const gpe_desc &d, int wreq[3], int xcd[3], int order[3], int plan[3],
              int stream[3]) {
  plan[0] = plan[1] = plan[2] = 0;
  stream[0] = stream[1] = stream[2] = 0;
  wreq[0] = 16;
  wreq[1] = d.precision == GPE_FP64 ? 8 : 16;
  wreq[2] = 8;
  xcd[0] = xcd[1] = 1;
  xcd[2] = 0;
  order[0] = 2;
  order[1] = 1;
  order[2] = 0;
}

bool valid_tuning(int dim, const int *n, int precision, const gpe_tuning &t, std::string &msg) {
  for (int j = 0; j < dim; ++j)
    if (!gpe::plan_available(n[j], t.plan[j])) {
      msg = "plan 1 exists only for 1024-point axes";
      return false;
    }
  for (int j = 0; j < dim; ++j)
    if (t.stream[j] < 0 || t.stream[j] > 3) {
      msg = "stream must be 0..3";
      return false;
    }
  if (t.transpose != 0 && (t.transpose != 1 || dim != 3)) {
    msg = "transpose must be 0, or 1 on a 3D grid";
    return false;
  }
  const int tiled = t.transpose ? dim : dim - 1;  // axes with tile widths
  for (int j = 0; j < tiled; ++j) {
    // 32: two 16-column halves per tile, in-place passes with FP32 storage
    const bool halves = t.width[j] == 32 && !t.transpose && precision != GPE_FP64;
    const bool quad = t.width[j] == 4 && t.transpose;
    if (t.width[j] != 8 && t.width[j] != 16 && !halves && !quad) {
      msg = "width must be 8 or 16 (32: in-place, FP32 storage; 4: rotating passes)";
      return false;
    }
    if (t.xcd_remap[j] != 0 && t.xcd_remap[j] != 1) {
      msg = "xcd_remap must be 0 or 1";
      return false;
    }
  }
  bool seen[3] = {false, false, false};
  for (int i = 0; i < dim; ++i) {
    const int a = t.pass_order[i];
    if (a < 0 || a >= dim || seen[a]) {
      msg = "pass_order must be a permutation of the axes";
      return false;
    }
    seen[a] = true;
  }
  return true;
}

// ABI form (user axes) to the view-axis arrays of a context (3D view: 2D
// problems use view axes 1 and 2).  An entry of rotating step passes leaves
// the in-place shapes at their defaults (they then serve the read-only passes)
// and fills *rot instead.
void to_view(int dim, const gpe_tuning &t, int wreq[3], int xcd[3], int order[3],
             int plan[3], int stream[3], RotShape *rot) {
  const int off = 3 - dim;
  const bool tr = dim == 3 && t.transpose == 1;
  if (rot) *rot = RotShape{};
  for (int j = 0; j < dim; ++j) {
    plan[j + off] = t.plan[j];
    if (tr) {
      if (rot) {
        rot->on = 1;
        rot->wreq[j] = t.width[j];
        rot->xcd[j] = t.xcd_remap[j];
        rot->stream[j] = t.stream[j];
      }
      continue;
    }
    stream[j + off] = t.stream[j];
    if (j < dim - 1) {
      wreq[j + off] = t.width[j];
      xcd[j + off] = t.xcd_remap[j];
    }
  }
  // view order: the given axes first, then the axes that do not exist
  int k = 0;
  for (int i = 0; i < dim; ++i) order[k++] = t.pass_order[i] + off;
  for (int ax = 0; ax < off; ++ax) order[k++] = ax;
}

// The inverse of to_view: the in-place shapes, or the rotating ones when
// rot is on.
void from_view(int dim, const int wreq[3], const int xcd[3], const int order[3],
               const int plan[3], const int stream[3], const RotShape *rot, gpe_tuning *t) {
  const int off = 3 - dim;
  std::memset(t, 0, sizeof(*t));
  const bool tr = dim == 3 && rot && rot->on;
  t->transpose = tr ? 1 : 0;
  for (int j = 0; j < dim; ++j) {
    t->plan[j] = plan[j + off];
    t->stream[j] = tr ? rot->stream[j] : stream[j + off];
    t->width[j] = tr ? rot->wreq[j] : j < dim - 1 ? wreq[j + off] : 0;
    t->xcd_remap[j] = tr ? rot->xcd[j] : j < dim - 1 ? xcd[j + off] : 0;
  }
  int k = 0;
  for (int i = 0; i < 3 && k < dim; ++i)
    if (order[i] >= off) t->pass_order[k++] = order[i] - off;
}

// ---- a small JSON reader for the tuning file ------------------------------

struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal *get(const char *k) const {
    for (auto &kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char *p, *end;
  bool ok = true;
  void ws() {
    while (p < end && std::isspace((unsigned char)*p)) ++p;
  }
  bool lit(const char *s) {
    const size_t n = std::strlen(s);
    if ((size_t)(end - p) >= n && std::strncmp(p, s, n) == 0) {
      p += n;
      return true;
    }
    return false;
  }
  JVal value(int depth) {
    JVal v;
    ws();
    if (p >= end || depth > 32) {
      ok = false;
      return v;
    }
    if (*p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return v;
      }
      while (ok) {
        ws();
        JVal k = value(depth + 1);
        if (!ok || k.kind != JVal::STR) { ok = false; break; }
        ws();
        if (p >= end || *p != ':') { ok = false; break; }
        ++p;
        JVal x = value(depth + 1);
        v.obj.emplace_back(k.str, x);
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') { ++p; break; }
        ok = false;
      }
    } else if (*p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return v;
      }
      while (ok) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') { ++p; break; }
        ok = false;
      }
    } else if (*p == '"') {
      ++p;
      v.kind = JVal::STR;
      while (p < end && *p != '"') {
        if (*p == '\\') { ok = false; break; }  // the file never needs escapes
        v.str += *p++;
      }
      if (p >= end) ok = false;
      else ++p;
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
    } else if (lit("null")) {
      v.kind = JVal::NUL;
    } else {
      char *q = nullptr;
      v.num = std::strtod(p, &q);
      if (q == p) ok = false;
      else p = q;
      v.kind = JVal::NUM;
    }
    return v;
  }
};

bool int_array(const JVal *v, int n, int *out) {
  if (!v || v->kind != JVal::ARR || (int)v->arr.size() != n) return false;
  for (int i = 0; i < n; ++i) {
    if (v->arr[i].kind != JVal::NUM || v->arr[i].num != std::floor(v->arr[i].num)) return false;
    out[i] = (int)v->arr[i].num;
  }
  return true;
}

// Time `steps` real-time steps of ctx (min over two runs), in ms per step.
// A candidate replaces the incumbent only when it is faster by more than
// this fraction: run-to-run noise must not move a class off its defaults.
constexpr double kMargin = 0.01;

// Best of three timed runs of the steady-state real-time step (phase N(dt)
// and the kinetic factor; the opening and closing half-steps of a call are
// left out: they would weigh the last pass of the order), ms per step.
double time_steps(gpe_ctx *c, int steps, hipEvent_t e0, hipEvent_t e1) {
  const double dt = 1e-3;
  void *K[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < n_axes(c); ++i) {
    const int ax = order_axis(c, i);
    if (get_table(c, ax, TB_KREAL, dt, &K[ax]) != GPE_OK) return -1;
  }
  if (steady_steps(c, 0, dt, 2, 2, K) != GPE_OK) return -1;
  double best = -1;
  for (int r = 0; r < 3; ++r) {
    if (hipEventRecord(e0, c->stream) != hipSuccess) return -1;
    if (steady_steps(c, 0, dt, steps, kGraphSteps, K) != GPE_OK) return -1;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return -1;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1;
    const double per = ms / steps;
    if (best < 0 || per < best) best = per;
  }
  return best;
}

}  // namespace

void effective_tuning(const gpe_desc &d, int wreq[3], int xcd[3], int order[3], int plan[3],
                      int stream[3], RotShape *rot) {
  defaults(d, wreq, xcd, order, plan, stream);
  if (rot) *rot = RotShape{};
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key_of(d));
  if (it != g_table.end()) to_view(d.dim, it->second, wreq, xcd, order, plan, stream, rot);
}

}  // namespace gpe_host

using namespace gpe_host;

extern "C" {

gpe_status gpe_tuning_set(const gpe_desc *desc, const gpe_tuning *t) {
  std::string msg;
  gpe_status st = validate_desc(desc, msg);
  if (st != GPE_OK) return st;
  if (!t || !valid_tuning(desc->dim, desc->n, desc->precision, *t, msg)) return GPE_EINVAL;
  gpe_tuning v = *t;
  for (int j = v.transpose ? desc->dim : desc->dim - 1; j < 3; ++j) v.width[j] = v.xcd_remap[j] = 0;
  for (int i = desc->dim; i < 3; ++i) v.pass_order[i] = v.plan[i] = v.stream[i] = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key_of(*desc)] = v;
  return GPE_OK;
}

gpe_status gpe_tuning_get(const gpe_desc *desc, gpe_tuning *out, int32_t *found) {
  std::string msg;
  gpe_status st = validate_desc(desc, msg);
  if (st != GPE_OK) return st;
  if (!out) return GPE_EINVAL;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(key_of(*desc));
    if (it != g_table.end()) {
      *out = it->second;
      if (found) *found = 1;
      return GPE_OK;
    }
  }
  int w[3], x[3], o[3], pl[3], sm[3];
  defaults(*desc, w, x, o, pl, sm);
  from_view(desc->dim, w, x, o, pl, sm, nullptr, out);
  out->ms_per_step = 0;
  if (found) *found = 0;
  return GPE_OK;
}

void gpe_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

gpe_status gpe_tuning_save(const char *path) {
  if (!path) return GPE_EINVAL;
  std::string s = "{\n  \"format\": \"gpe-tuning-1\",\n  \"classes\": [";
  {
    std::lock_guard<std::mutex> lk(g_mu);
    bool first = true;
    char buf[512];
    for (auto &kv : g_table) {
      const TuneKey &k = kv.first;
      const gpe_tuning &t = kv.second;
      const int d = k.dim;
      auto arr = [&](const int *v) {
        std::string a = "[";
        for (int j = 0; j < d; ++j) a += (j ? ", " : "") + std::to_string(v[j]);
        return a + "]";
      };
      std::snprintf(buf, sizeof(buf),
                    "%s\n    {\"dim\": %d, \"n\": %s, \"precision\": \"%s\", \"width\": %s, "
                    "\"xcd_remap\": %s, \"pass_order\": %s, \"plan\": %s, \"stream\": %s, "
                    "\"transpose\": %d, \"ms_per_step\": %.6g}",
                    first ? "" : ",", d, arr(k.n).c_str(),
                    k.prec == GPE_FP32 ? "fp32" : k.prec == GPE_FP32_STATE ? "fp32s" : "fp64",
                    arr(t.width).c_str(), arr(t.xcd_remap).c_str(), arr(t.pass_order).c_str(),
                    arr(t.plan).c_str(), arr(t.stream).c_str(), (int)t.transpose, t.ms_per_step);
      s += buf;
      first = false;
    }
  }
  s += "\n  ]\n}\n";
  FILE *f = std::fopen(path, "wb");
  if (!f) return GPE_EINVAL;
  const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
  return std::fclose(f) == 0 && ok ? GPE_OK : GPE_EINVAL;
}

gpe_status gpe_tuning_load(const char *path) {
  if (!path) return GPE_EINVAL;
  FILE *f = std::fopen(path, "rb");
  if (!f) return GPE_EINVAL;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, n);
    if (text.size() > (1u << 22)) break;
  }
  std::fclose(f);
  JParser jp{text.data(), text.data() + text.size()};
  const JVal root = jp.value(0);
  jp.ws();
  if (!jp.ok || jp.p != jp.end || root.kind != JVal::OBJ) return GPE_EINVAL;
  const JVal *fmt = root.get("format");
  const JVal *cls = root.get("classes");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "gpe-tuning-1" || !cls ||
      cls->kind != JVal::ARR)
    return GPE_EINVAL;
  // validate everything before touching the table
  std::vector<std::pair<gpe_desc, gpe_tuning>> entries;
  for (const JVal &e : cls->arr) {
    if (e.kind != JVal::OBJ) return GPE_EINVAL;
    const JVal *dim = e.get("dim"), *prec = e.get("precision"), *ms = e.get("ms_per_step");
    if (!dim || dim->kind != JVal::NUM || (dim->num != 2 && dim->num != 3)) return GPE_EINVAL;
    const int d = (int)dim->num;
    gpe_desc desc{};
    desc.dim = d;
    gpe_tuning t{};
    if (!int_array(e.get("n"), d, desc.n) || !int_array(e.get("width"), d, t.width) ||
        !int_array(e.get("xcd_remap"), d, t.xcd_remap) ||
        !int_array(e.get("pass_order"), d, t.pass_order))
      return GPE_EINVAL;
    if (!prec || prec->kind != JVal::STR ||
        (prec->str != "fp64" && prec->str != "fp32" && prec->str != "fp32s"))
      return GPE_EINVAL;
    desc.precision = prec->str == "fp32" ? GPE_FP32 : prec->str == "fp32s" ? GPE_FP32_STATE : GPE_FP64;
    for (int j = 0; j < d; ++j) {
      desc.lo[j] = 0;
      desc.hi[j] = 1;
    }
    desc.norm_target = 1;
    std::string msg;
    const JVal *pl = e.get("plan");  // optional (files written before plans existed)
    if (pl && !int_array(pl, d, t.plan)) return GPE_EINVAL;
    const JVal *sm = e.get("stream");  // optional likewise
    if (sm && !int_array(sm, d, t.stream)) return GPE_EINVAL;
    const JVal *tp = e.get("transpose");  // optional likewise
    if (tp && (tp->kind != JVal::NUM || (tp->num != 0 && tp->num != 1))) return GPE_EINVAL;
    t.transpose = tp ? (int32_t)tp->num : 0;
    if (validate_desc(&desc, msg) != GPE_OK || !valid_tuning(d, desc.n, desc.precision, t, msg))
      return GPE_EINVAL;
    t.ms_per_step = ms && ms->kind == JVal::NUM ? ms->num : 0;
    entries.emplace_back(desc, t);
  }
  for (auto &e : entries) gpe_tuning_set(&e.first, &e.second);
  return GPE_OK;
}

gpe_status gpe_autotune(const gpe_desc *desc, int32_t steps, gpe_tuning *out) {
  std::string msg;
  gpe_status st = validate_desc(desc, msg);
  if (st != GPE_OK) return st;
  if (steps < 1) return GPE_EINVAL;
  gpe_desc d = *desc;
  d.g = 1.0;
  d.norm_target = 1.0;
  gpe_ctx *c = nullptr;
  // A scratch context of the class holding pseudo-random values (the passes
  // run the same instructions for any state, but a zero state draws less
  // power and would time faster than real data).  The real-time step uses no
  // partial sums, so the shapes tried need no other buffers.
  int w0[3], x0[3], o0[3], p0[3], s0[3];
  effective_tuning(d, w0, x0, o0, p0, s0);
  if ((st = create_context(&d, nullptr, nullptr, nullptr, true, &c)) != GPE_OK) return st;
  if (gpe::launch_fill_noise(c->prec, c->psi, c->sites, c->stream) != hipSuccess) {
    gpe_destroy(c);
    return GPE_EDEVICE;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    gpe_destroy(c);
    return GPE_EDEVICE;
  }
  int bs[3];  // streaming flags (the last coordinate tried)
  std::memcpy(bs, s0, sizeof(bs));
  int bt = 0;  // rotating step passes (tried last, from their own start)
  // GPE_TUNE_VERBOSE=1 prints every candidate and its time to stderr.
  const char *verbose_env = std::getenv("GPE_TUNE_VERBOSE");
  const bool verbose = verbose_env && *verbose_env == '1';
  auto report = [&](double t) {
    if (!verbose) return;
    const int *w = bt ? c->rot.wreq : c->wreq, *x = bt ? c->rot.xcd : c->xcd_remap;
    const int *sm = bt ? c->rot.stream : c->streaming;
    std::fprintf(stderr,
                 "tune %dx%dx%d p%d rot %d width %d %d %d xcd %d %d %d stream %d %d %d order %d %d %d "
                 "plan %d %d %d: %.4f ms\n",
                 c->n3[0], c->n3[1], c->n3[2], d.precision, bt, w[0], w[1], w[2], x[0], x[1], x[2],
                 sm[0], sm[1], sm[2], c->pass_order[0], c->pass_order[1], c->pass_order[2],
                 c->plan[0], c->plan[1], c->plan[2], t);
  };
  auto apply = [&](const int w[3], const int x[3], const int o[3], const int p[3]) {
    c->rot.on = bt;
    for (int j = 0; j < 3; ++j) {
      c->pass_order[j] = o[j];
      c->plan[j] = p[j];
      if (bt) {
        c->rot.wreq[j] = w[j];
        c->rot.xcd[j] = x[j];
        c->rot.stream[j] = bs[j];
      } else {
        c->wreq[j] = w[j];
        c->xcd_remap[j] = x[j];
        c->streaming[j] = bs[j];
      }
    }
    drop_step_graphs(c);  // cached step graphs hold the previous shapes
  };
  int bw[3], bx[3], bo[3], bp[3];
  std::memcpy(bw, w0, sizeof(bw));
  std::memcpy(bx, x0, sizeof(bx));
  std::memcpy(bo, o0, sizeof(bo));
  std::memcpy(bp, p0, sizeof(bp));
  apply(bw, bx, bo, bp);
  double best = time_steps(c, steps, e0, e1);
  report(best);
  const int off = 3 - d.dim;
  // Per axis, jointly: radix plan x width x tile order x streaming policy
  // (width and tile order on the strided axes only; a narrower tile may only
  // pay off with streaming loads, so the policy is not tried separately).
  auto axis_round = [&]() {
    for (int ax = off; ax < 3 && best > 0; ++ax) {
      for (int pl : {0, 1}) {
        if (!gpe::plan_available(c->n3[ax], pl)) continue;
        for (int w : {4, 8, 16, 32}) {
          // (a rotating pass has tiles on every axis, the in-place contiguous one none)
          const bool tiled = ax != 2 || bt;
          if (w == 32 && (bt || d.precision == GPE_FP64)) continue;
          if (w == 4 && !bt) continue;
          if (!tiled && w != bw[ax]) continue;
          if (tiled && gpe::pass_shape(d.precision, c->n3, ax, w, pl, false, bt).W != w) continue;
          for (int x : {0, 1}) {
            if (!tiled && x != bx[ax]) continue;
            for (int sm = 0; sm < 4; ++sm) {
              if (pl == bp[ax] && w == bw[ax] && x == bx[ax] && sm == bs[ax]) continue;
              int tw[3], tx[3], tp[3];
              std::memcpy(tw, bw, sizeof(tw));
              std::memcpy(tx, bx, sizeof(tx));
              std::memcpy(tp, bp, sizeof(tp));
              const int s_keep = bs[ax];
              tw[ax] = w;
              tx[ax] = x;
              tp[ax] = pl;
              bs[ax] = sm;
              apply(tw, tx, bo, tp);
              const double t = time_steps(c, steps, e0, e1);
              report(t);
              if (t > 0 && t < best * (1 - kMargin)) {
                best = t;
                std::memcpy(bw, tw, sizeof(bw));
                std::memcpy(bx, tx, sizeof(bx));
                std::memcpy(bp, tp, sizeof(bp));
              } else {
                bs[ax] = s_keep;
              }
            }
          }
        }
      }
    }
  };
  // In-place passes: 1. per-axis shapes; 2. the axis order of the step (it
  // decides which pass carries the phase); 3. per-axis shapes again for that
  // order.  Then, on large 3D grids, the rotating passes (their order is
  // fixed) from 8-column tiles, per-axis shapes twice; the faster form wins.
  axis_round();
  int perm[3] = {0, 1, 2};
  int axes[3], na = 0;
  for (int ax = off; ax < 3; ++ax) axes[na++] = ax;
  std::sort(perm, perm + na);
  do {
    int to[3];
    int k = 0;
    for (int i = 0; i < na; ++i) to[k++] = axes[perm[i]];
    for (int ax = 0; ax < off; ++ax) to[k++] = ax;
    if (std::equal(to, to + 3, bo) || best <= 0) continue;
    apply(bw, bx, to, bp);
    const double t = time_steps(c, steps, e0, e1);
    report(t);
    if (t > 0 && t < best * (1 - kMargin)) {
      best = t;
      std::memcpy(bo, to, sizeof(bo));
    }
  } while (std::next_permutation(perm, perm + na));
  axis_round();
  c->rot.on = 1;
  if (d.dim == 3 && use_trans(c) && best > 0) {
    int kw[3], kx[3], kp[3], ks[3];
    std::memcpy(kw, bw, sizeof(kw));
    std::memcpy(kx, bx, sizeof(kx));
    std::memcpy(kp, bp, sizeof(kp));
    std::memcpy(ks, bs, sizeof(ks));
    const double keep = best;
    bt = 1;
    for (int j = 0; j < 3; ++j) {
      bw[j] = 8;
      bx[j] = 1;
      bs[j] = 0;
    }
    apply(bw, bx, bo, bp);
    best = time_steps(c, steps, e0, e1);
    report(best);
    axis_round();
    axis_round();
    if (!(best > 0 && best < keep * (1 - kMargin))) {
      bt = 0;
      best = keep;
      std::memcpy(bw, kw, sizeof(bw));
      std::memcpy(bx, kx, sizeof(bx));
      std::memcpy(bp, kp, sizeof(bp));
      std::memcpy(bs, ks, sizeof(bs));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  gpe_destroy(c);
  if (!(best > 0)) return GPE_EDEVICE;
  gpe_tuning t{};
  RotShape rs;
  rs.on = bt;
  std::memcpy(rs.wreq, bw, sizeof(bw));
  std::memcpy(rs.xcd, bx, sizeof(bx));
  std::memcpy(rs.stream, bs, sizeof(bs));
  from_view(d.dim, bw, bx, bo, bp, bs, &rs, &t);
  t.ms_per_step = best;
  if ((st = gpe_tuning_set(&d, &t)) != GPE_OK) return st;
  if (out) *out = t;
  return GPE_OK;
}

}  // extern "C"
