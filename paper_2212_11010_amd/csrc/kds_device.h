// kds_device.h -- device helpers shared by the kernel translation units.
#pragma once

#include <algorithm>
#include <cstring>

#include "kds_internal.h"

namespace kds {

inline unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
__device__ __forceinline__ T powi(T x, int n) {
  T r = T(1);
  while (n > 0) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

// node offset inside a cell of the node with index 0 on axis a and the
// remaining indices given by the mixed-radix number `on` (x fastest)
__device__ __forceinline__ int other_node_offset(int on, int a, int P, int dim) {
  int off = 0, mul = 1;
  for (int ax = 0; ax < dim; ++ax) {
    if (ax != a) {
      off += (on % P) * mul;
      on /= P;
    }
    mul *= P;
  }
  return off;
}

}  // namespace kds
