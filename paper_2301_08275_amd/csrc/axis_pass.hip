// Launch geometry and operation-set dispatch of the fused axis pass.
#include "axis_pass.h"

namespace gpe {
namespace pass {

hipError_t launch_f64(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s);
hipError_t launch_f32(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s);
hipError_t launch_s32(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s);

int tpl_of(int N, int plan) {
  if (plan == 1 && N == 1024) return PlanAlt<1024>::type::TPL;
  switch (N) {
    case 8: return PlanFor<8>::type::TPL;
    case 16: return PlanFor<16>::type::TPL;
    case 32: return PlanFor<32>::type::TPL;
    case 64: return PlanFor<64>::type::TPL;
    case 128: return PlanFor<128>::type::TPL;
    case 256: return PlanFor<256>::type::TPL;
    case 512: return PlanFor<512>::type::TPL;
    case 1024: return PlanFor<1024>::type::TPL;
    default: return 0;
  }
}

namespace {

// The specialised kernels assume full tiles and one of the standard pass
// layouts (the step passes: forward, per-frequency table, inverse, store,
// with the opening or closing phase;
// forward-only transforms; the spectral-derivative pass; the observables'
// forward passes); anything else runs generic.
int stream_bits(const PassArgs &a) {
  return ((a.stream & 1) ? STREAM_LOAD : 0) | ((a.stream & 2) ? STREAM_STORE : 0);
}

int pick_mode(const PassArgs &a, const PassShape &sh) {
  if (a.slots)
    return (a.slot_imag ? MODE_SLOTS_IMAG : MODE_SLOTS_REAL) | SLOT_ROLE |
           ((a.slot_pass & SLOT_PASS_FIRST) ? SLOT_FIRST : 0) |
           ((a.slot_pass & SLOT_PASS_LAST) ? SLOT_LAST : 0);
  const bool full = sh.strided || ((long long)a.n[0] * a.n[1]) % sh.W == 0;
  if (!full || !a.forward) return MODE_GENERIC;
  if (!a.store) {
    const bool obs = !a.inverse && a.mid == MID_NONE && a.pre == PH_NONE &&
                     a.post == PH_NONE && !a.refwd;
    if (obs && a.red == RED_KIN) return MODE_OBS;
    if (obs && a.red == (RED_KIN | RED_REAL)) return MODE_OBS_REAL;
    return MODE_GENERIC;
  }
  const bool bare = !a.scale && a.pre == PH_NONE && a.red == RED_NONE;
  if (!a.inverse) {
    if (a.mid != MID_NONE || a.post != PH_NONE || a.refwd) return MODE_GENERIC;
    if (bare) return MODE_FWD;
    const bool real_sums = !a.scale && a.pre == PH_NONE && a.red == RED_REAL;
    return real_sums ? MODE_FWD_REAL : MODE_GENERIC;
  }
  if (a.mid != MID_TABLE) return MODE_GENERIC;
  if (a.refwd) return bare && a.post == PH_DERIV ? MODE_DERIV : MODE_GENERIC;
  if (a.pre == PH_NONE && a.post == PH_NONE && a.red == RED_NONE && !a.scale)
    return MODE_PLAIN | stream_bits(a);
  if (a.pre == PH_REAL && a.post == PH_NONE && a.red == RED_NONE && !a.scale)
    return MODE_PRE_REAL | stream_bits(a);
  if (a.pre == PH_NONE && a.post == PH_REAL && a.red == RED_NONE && !a.scale) return MODE_POST_REAL;
  const bool im_pre = a.pre == PH_IMAG || a.pre == PH_IMAG_EXACT;
  const bool im_post = a.post == PH_IMAG || a.post == PH_IMAG_EXACT;
  if (im_pre && a.post == PH_NONE && a.red == RED_NONE && a.scale)
    return a.pre == PH_IMAG ? MODE_PRE_IMAG : MODE_PRE_IMAG_EXACT;
  if (a.pre == PH_NONE && im_post && a.red == RED_NORM_OUT && !a.scale)
    return a.post == PH_IMAG ? MODE_POST_IMAG_RED : MODE_POST_IMAG_RED_EXACT;
  return MODE_GENERIC;
}

// Operation sets that need more than 128 VGPRs on a 1024-thread tile with
// FP64 arithmetic (compiler resource report at 512 points: 12-304 bytes of
// scratch per lane; the step passes, transforms and observables fit), and the
// exact imaginary-time pre pass, which fits but whose per-site exp, expm1 and
// sqrt make a lone 1024-thread tile per CU compute-bound (measured at 512^3:
// 3 % faster on 8-column tiles in FP64, 12 % with the FP32 state).
bool heavy_mode(int mode) {
  switch (base_mode(mode)) {
    case MODE_GENERIC:
    case MODE_PRE_IMAG:
    case MODE_PRE_IMAG_EXACT:
    case MODE_POST_IMAG_RED:
    case MODE_POST_IMAG_RED_EXACT:
    case MODE_POST_REAL:
    case MODE_SLOTS_REAL:
    case MODE_SLOTS_IMAG:
    case MODE_DERIV:
      return true;
    default:
      return false;
  }
}

}  // namespace
}  // namespace pass

PassShape pass_shape(int precision, const int n[3], int axis, int wreq, int plan, bool narrow,
                     bool trans) {
  using namespace pass;
  PassShape sh{};
  sh.N = n[axis];
  sh.strided = trans || axis != 2;
  const int tpl = tpl_of(sh.N, plan);
  if (tpl == 0) return sh;
  if (!sh.strided) {
    sh.W = tpl >= GPE_CONTIG_THREADS ? 1 : GPE_CONTIG_THREADS / tpl;
    sh.threads = tpl * sh.W;
    const long long lines = (long long)n[0] * n[1];
    sh.blocks = (lines + sh.W - 1) / sh.W;
  } else {
    // 32: tiles of two 16-column halves (in-place plain step passes with FP32
    // storage; launch_shape gives other passes 16)
    if (wreq == 32 && !narrow && !trans && state_f32(precision) && sh.N >= 256 &&
        fit_w(sh.N, math_f32(precision) ? 8 : 16, 16, tpl) == 16 && n[2] >= 32) {
      sh.W = 32;
      sh.threads = tpl * 16;
      const long long outer = axis == 1 ? n[0] : n[1];
      sh.blocks = outer * (n[2] / 32);
      return sh;
    }
    const int want = wreq >= 16 ? 16 : 8;
    int ws = fit_w(sh.N, math_f32(precision) ? 8 : 16, want, tpl);
    if (narrow && ws == 16 && tpl * 16 == 1024 && (!math_f32(precision) || sh.N / tpl == 16))
      ws = 8;
    if (trans) {
      // W lines at consecutive positions of the next axis, one tile per
      // (third-axis position, run of W); also 4 lines (N >= 128)
      const int nb = n[axis == 2 ? 0 : axis + 1], nc = n[3 - axis - (axis == 2 ? 0 : axis + 1)];
      if (wreq == 4 && !narrow && sh.N >= 128) ws = 4;
      sh.W = nb >= ws ? ws : 8;
      sh.threads = tpl * sh.W;
      sh.blocks = (long long)nc * (nb / sh.W);
      return sh;
    }
    sh.W = n[2] >= ws ? ws : 8;
    sh.threads = tpl * sh.W;
    const long long outer = axis == 1 ? n[0] : n[1];
    sh.blocks = outer * (n[2] / sh.W);
  }
  return sh;
}

PassShape launch_shape(int precision, const PassArgs &a) {
  const bool trans = a.trans && !a.slots;
  PassShape sh = pass_shape(precision, a.n, a.axis, a.wreq, a.plan, false, trans);
  if (sh.W == 32 && (a.slots || pass::base_mode(pass::pick_mode(a, sh)) != pass::MODE_PLAIN))
    sh = pass_shape(precision, a.n, a.axis, 16, a.plan, false, trans);
  // (narrowing changes strided tiles only, and the mode depends on the shape
  // only through the contiguous full-tile test, so the mode is unchanged)
  return pass::heavy_mode(pass::pick_mode(a, sh))
             ? pass_shape(precision, a.n, a.axis, a.wreq == 32 ? 16 : a.wreq, a.plan, true, trans)
             : sh;
}

hipError_t launch_axis_pass(int precision, const PassArgs &a, hipStream_t s) {
  const PassShape sh = launch_shape(precision, a);
  if (sh.threads == 0) return hipErrorInvalidValue;
  if (a.trans && !a.slots) {
    // a rotating pass reads whole lines and writes rows elsewhere: 3D grids,
    // distinct buffers, full tiles
    const int bx = a.axis == 2 ? 0 : a.axis + 1;
    if (a.n[0] < 2 || a.n[1] < 2 || a.n[2] < 2 || a.src == a.dst || a.n[bx] < sh.W ||
        a.n[bx] % sh.W != 0)
      return hipErrorInvalidValue;
  } else if (sh.strided && a.n[2] < sh.W) {
    return hipErrorInvalidValue;
  }
  const int mode = pass::pick_mode(a, sh);
  if (precision == 1) return pass::launch_f32(a, sh, mode, s);
  if (precision == 2) return pass::launch_s32(a, sh, mode, s);
  return pass::launch_f64(a, sh, mode, s);
}

}  // namespace gpe
