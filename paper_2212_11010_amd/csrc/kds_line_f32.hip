// kds_line_f32.hip -- line-schedule kernels and launchers for FP32 state.
#include "kds_line.h"

namespace kds {

KDS_LINE_TU(float, f32)

}  // namespace kds
