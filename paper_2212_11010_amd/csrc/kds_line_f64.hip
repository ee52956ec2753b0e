// kds_line_f64.hip -- line-schedule kernels and launchers for FP64 state.
#include "kds_line.h"

namespace kds {

KDS_LINE_TU(double, f64)

}  // namespace kds
