// FP64 instantiations of the fused axis pass (templates in axis_pass.h).
#include "axis_pass.h"

namespace gpe {
namespace pass {
hipError_t launch_f64(const PassArgs &a, const PassShape &sh, int mode, hipStream_t s) {
  return launch_t<double>(a, sh, mode, s);
}
}  // namespace pass
}  // namespace gpe
