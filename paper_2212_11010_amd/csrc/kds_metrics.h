// kds_metrics.h -- host entry points of the subdomain-iteration diagnostics
// (kds_metrics.hip).
#pragma once

#include "kds_internal.h"

namespace kds {

// The outflow traces of iterate 0 (the state f at t^{n-1}) at the end of
// every subdomain, into tr laid out as the plain sweep's traces ([k m + c]
// blocks of g.tr_stride entries: [subdomain][node line]).  Axis-aligned
// velocity sets (tab: the sweep table).
hipError_t launch_trace_iterate0(int prec, const Geom& g, const void* tab, const void* f,
                                 void* tr, hipStream_t s);

// out[0] = max |x - y| and out[1] = max |x| over n entries (run precision),
// as double bits combined with an unsigned atomic maximum: out must start at
// zero.  A NaN counts as +inf.
hipError_t launch_max_absdiff(int prec, const void* x, const void* y, int64_t n,
                              unsigned long long* out, hipStream_t s);

// The same over the nodes on the outflow faces of every subdomain (for
// velocity k the downwind faces along each axis with fp.sg[k][a] != 0), x and
// y full states [k m + c][cell][node]: any velocity set.
hipError_t launch_max_absdiff_outflow(int prec, const void* x, const void* y, const Geom& g,
                                      const FrontParams& fp, unsigned long long* out,
                                      hipStream_t s);

}  // namespace kds
