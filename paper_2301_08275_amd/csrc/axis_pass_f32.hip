// FP32 instantiations of the fused axis pass (templates in axis_pass.h).  The
// state, twiddles and butterflies are FP32; phases and sums stay FP64.
#include "axis_pass.h"

namespace gpe {
namespace pass {
hipError_t launch_f32(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  return launch_t<float>(a, sh, mode, s);
}
}  // namespace pass
}  // namespace gpe
