// Instantiations of the fused axis pass for an FP32 state with FP64
// arithmetic (templates in axis_pass.h): loads widen to FP64, the pass runs
// in FP64 like the FP64 form, and the store rounds once to FP32.
#include "axis_pass.h"

namespace gpe {
namespace pass {
hipError_t launch_s32(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  return launch_t<double, float>(a, sh, mode, s);
}
}  // namespace pass
}  // namespace gpe
