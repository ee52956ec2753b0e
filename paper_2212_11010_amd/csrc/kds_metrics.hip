// kds_metrics.hip -- diagnostics of the subdomain iteration (Sec. 5.1), off
// the step path: the outflow traces of iterate 0 (the state at t^{n-1}) in
// the layout the plain sweep writes its iterates' traces, and the largest
// difference between two trace sets.
#include "kds_device.h"
#include "kds_metrics.h"

namespace kds {

namespace {

// One thread per (node line, subdomain) of every (velocity, component): the
// value at the downwind face node of the subdomain's last cell, stored at
// [k m + c][subdomain][line] with the line numbering of the plain sweep
// (cells across the axis, then node combinations across the axis).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_trace_iterate0(const T* __restrict__ f,
                                                        T* __restrict__ tr, Geom g,
                                                        SweepTab<T> tab) {
  const int kc = blockIdx.y;
  const int k = kc / g.m;
  const int a = tab.axis[k];
  const int sg = tab.sign[k];
  const int Na = g.N[a];
  const int S = g.S[a];
  const int nseg = Na / S;
  const int per = g.nn / P;
  const int64_t nlines = (g.ncell / Na) * per;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nlines * nseg) return;
  const int seg = (int)(t / nlines);
  const int64_t line = t - (int64_t)seg * nlines;
  const int on = (int)(line % per);
  int64_t oc = line / per;
  int64_t cell0 = 0, cmul = 1, cs = 1;
  for (int ax = 0; ax < g.dim; ++ax) {
    if (ax == a) {
      cs = cmul;
    } else {
      cell0 += (oc % g.N[ax]) * cmul;
      oc /= g.N[ax];
    }
    cmul *= g.N[ax];
  }
  int ns = 1;
  for (int ax = 0; ax < a; ++ax) ns *= P;
  const int64_t base = ((int64_t)kc * g.ncell + cell0) * g.nn + other_node_offset(on, a, P, g.dim);
  // the subdomain's last cell in downwind order, and its downwind node
  const int j = seg * S + S - 1;
  const int r = sg > 0 ? j : Na - 1 - j;
  const int b = sg > 0 ? P - 1 : 0;
  tr[(int64_t)kc * g.tr_stride + (int64_t)seg * nlines + line] = f[base + r * cs * g.nn + b * ns];
}

// out[0] = max |x - y|, out[1] = max |x| over n entries, as the bits of
// non-negative doubles under an unsigned maximum (a NaN counts as +inf).
template <typename T>
__global__ __launch_bounds__(256) void k_max_absdiff(const T* __restrict__ x,
                                                     const T* __restrict__ y, int64_t n,
                                                     unsigned long long* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double d = 0.0, v = 0.0;
  for (; i < n; i += stride) {
    const double xi = (double)x[i], yi = (double)y[i];
    const double di = fabs(xi - yi), vi = fabs(xi);
    d = di == di ? fmax(d, di) : INFINITY;
    v = vi == vi ? fmax(v, vi) : INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o));
    v = fmax(v, __shfl_xor(v, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(d));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(v));
  }
}

// The same maximum over the nodes on the outflow faces of every subdomain:
// for velocity k, the faces on the downwind side along each axis where
// V^a != 0 (sg: the signs of V^a); x and y full states laid out
// [k m + c][cell][node], cells and nodes with axis 0 fastest.
template <typename T>
__global__ __launch_bounds__(256) void k_max_absdiff_outflow(const T* __restrict__ x,
                                                             const T* __restrict__ y, Geom g,
                                                             FrontParams fp,
                                                             unsigned long long* __restrict__ out) {
  const int64_t n = (int64_t)g.nv * g.m * g.ncell * g.nn;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double d = 0.0, v = 0.0;
  for (; i < n; i += stride) {
    int64_t r = i / g.nn;
    int nd = (int)(i - r * g.nn);
    int64_t cell = r % g.ncell;
    const int k = (int)(r / g.ncell) / g.m;
    bool on = false;
    for (int a = 0; a < g.dim; ++a) {
      const int ca = (int)(cell % g.N[a]);
      cell /= g.N[a];
      const int ba = nd % g.P;
      nd /= g.P;
      const int sa = fp.sg[k][a];
      if (sa > 0) on = on || (ca % g.S[a] == g.S[a] - 1 && ba == g.P - 1);
      if (sa < 0) on = on || (ca % g.S[a] == 0 && ba == 0);
    }
    if (!on) continue;
    const double xi = (double)x[i], yi = (double)y[i];
    const double di = fabs(xi - yi), vi = fabs(xi);
    d = di == di ? fmax(d, di) : INFINITY;
    v = vi == vi ? fmax(v, vi) : INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o));
    v = fmax(v, __shfl_xor(v, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(d));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(v));
  }
}

template <typename T>
hipError_t trace_iterate0_t(const Geom& g, const void* tab, const void* f, void* tr,
                            hipStream_t s) {
  const SweepTab<T>& t = *(const SweepTab<T>*)tab;
  int64_t most = 0;
  for (int k = 0; k < g.nv; ++k) {
    const int a = t.axis[k];
    most = std::max<int64_t>(most, (g.ncell / g.N[a]) * (g.nn / g.P) * (g.N[a] / g.S[a]));
  }
  const dim3 grid(blocks_for(most), g.nv * g.m);
  switch (g.P) {
#define KDS_TR0(PP)                                                                            \
  case PP:                                                                                     \
    hipLaunchKernelGGL((k_trace_iterate0<T, PP>), grid, dim3(256), 0, s, (const T*)f, (T*)tr, \
                       g, t);                                                                  \
    break;
    KDS_TR0(1)
    KDS_TR0(2)
    KDS_TR0(3)
    KDS_TR0(4)
#undef KDS_TR0
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trace_iterate0(int prec, const Geom& g, const void* tab, const void* f,
                                 void* tr, hipStream_t s) {
  return prec == KDS_FP64 ? trace_iterate0_t<double>(g, tab, f, tr, s)
                          : trace_iterate0_t<float>(g, tab, f, tr, s);
}

hipError_t launch_max_absdiff(int prec, const void* x, const void* y, int64_t n,
                              unsigned long long* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n), 1024));
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_max_absdiff<double>, dim3(nb), dim3(256), 0, s, (const double*)x,
                       (const double*)y, n, out);
  else
    hipLaunchKernelGGL(k_max_absdiff<float>, dim3(nb), dim3(256), 0, s, (const float*)x,
                       (const float*)y, n, out);
  return hipGetLastError();
}

hipError_t launch_max_absdiff_outflow(int prec, const void* x, const void* y, const Geom& g,
                                      const FrontParams& fp, unsigned long long* out,
                                      hipStream_t s) {
  const int64_t n = (int64_t)g.nv * g.m * g.ncell * g.nn;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n), 4096));
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_max_absdiff_outflow<double>, dim3(nb), dim3(256), 0, s, (const double*)x,
                       (const double*)y, g, fp, out);
  else
    hipLaunchKernelGGL(k_max_absdiff_outflow<float>, dim3(nb), dim3(256), 0, s, (const float*)x,
                       (const float*)y, g, fp, out);
  return hipGetLastError();
}

}  // namespace kds
