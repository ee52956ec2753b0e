// kds_kernels.hip -- gfx950 kernels of libkds: pointwise passes (init,
// relaxation, moments, checkpoint copies), the plain sweep, and the host-side
// dispatch of every launcher (the line schedule lives in kds_line.h, the front
// schedule in kds_front.hip).
//
// Kinetic state layout in HBM: f[k][c][cell][node] (velocity, component,
// cell x-fastest, node x-fastest), stored in T = double or float.  Every
// (velocity, component) pair is one contiguous plane of ncell * nn values, so
// the pointwise kernels (init, relaxation, moments) read one coalesced stream
// per (k, c) and the sweeps read whole cells.
//
// Transport of an axis-aligned velocity (Sec. 3.1 eq:dg_imp, Sec. 3.2,
// Sec. 5.1 eq:ibvp): the implicit upwind DG system splits exactly into
// independent 1-D problems along grid lines (faces with V.N = 0 carry no
// flux).  On one line, in downwind order, cell j obeys
//     f_j^n = C f_j^{n-1} + e1 t_j^{n-1} + eth t_j^n,
// t_j = outflow node of the upwind neighbour (node P-1 in downwind order),
// e1 = (1 - theta) e, eth = theta e.  Inside a subdomain t_j^n = f_{j-1}^n[P-1];
// at the first cell of a subdomain, iterate p takes t^n from the upwind
// subdomain's iterate p-1 (iterate 0 = the state at t^{n-1}), or the
// prescribed boundary value on a Dirichlet axis.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "kds_device.h"

namespace kds {

// ============================================================ equilibrium

// M_k(W) = a_k W + sum_i b_{k,i} Q^i(W) (moment conditions, eq:maxwell_def),
// evaluated in FP64.
template <int LAW, int D, int M, int NV>
__device__ __forceinline__ void flux(const EqTab<D, M, NV>& t, const double (&W)[M],
                                     double (&Q)[D][M]) {
  if constexpr (LAW == KDS_LAW_LINEAR) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) s += t.A[i][r][q] * W[q];
        Q[i][r] = s;
      }
  } else {
    static_assert(M == D + 2, "Euler needs m = d + 2");
    const double rho = W[0];
    const double E = W[D + 1];
    double u[D];
    double ke = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      u[i] = W[1 + i] / rho;
      ke += 0.5 * W[1 + i] * u[i];
    }
    const double pr = (t.gamma - 1.0) * (E - ke);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Q[i][0] = W[1 + i];
#pragma unroll
      for (int j = 0; j < D; ++j) Q[i][1 + j] = W[1 + i] * u[j] + (i == j ? pr : 0.0);
      Q[i][D + 1] = (E + pr) * u[i];
    }
  }
}

// Component r of M_k from W and Q(W).
template <int D, int M, int NV>
__device__ __forceinline__ double eq_comp(const EqTab<D, M, NV>& t, const double (&W)[M],
                                          const double (&Q)[D][M], int k, int r) {
  double s = t.a[k] * W[r];
#pragma unroll
  for (int i = 0; i < D; ++i) s += t.b[k][i] * Q[i][r];
  return s;
}

template <int LAW, int D, int M, int NV>
__device__ __forceinline__ void equilibrium(const EqTab<D, M, NV>& t, const double (&W)[M],
                                            double (&Mk)[NV][M]) {
  double Q[D][M];
  flux<LAW, D, M, NV>(t, W, Q);
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) Mk[k][r] = eq_comp(t, W, Q, k, r);
}

// ===================================================== pointwise kernels

// F_k = M_k(W) at every node (Sec. 2.2); W is [node][c] with node = cell*nn + i.
template <typename T, int LAW, int D, int M, int NV>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ W, T* __restrict__ f,
                                              int64_t plane, EqTab<D, M, NV> t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  double w[M];
#pragma unroll
  for (int r = 0; r < M; ++r) w[r] = W[i * M + r];
  double Mk[NV][M];
  equilibrium<LAW, D, M, NV>(t, w, Mk);
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) f[(int64_t)(k * M + r) * plane + i] = (T)Mk[k][r];
}

// Relaxation (eq:over_relaxation): W = sum_k f_k in FP64, M_k(W) in FP64,
// f_k <- f_k + omega (M_k - f_k), one rounding to T.  fin may equal fout.
template <typename T, int LAW, int D, int M, int NV>
__device__ __forceinline__ void relax_values(const EqTab<D, M, NV>& t, const T (&fr)[NV][M],
                                             T (&out)[NV][M]) {
  // the kinetic values stay in their storage type until used (registers);
  // W, Q(W) and every M_k component in FP64, one rounding per output
  double w[M];
#pragma unroll
  for (int r = 0; r < M; ++r) w[r] = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) w[r] += (double)fr[k][r];
  double Q[D][M];
  if (t.has_source) {
    // Crank-Nicolson source step on W; the kinetic data take the equilibrium
    // part of the change so that sum_k f_k = W+ before relaxing towards M(W+)
    double Qm[D][M], wp[M];
    flux<LAW, D, M, NV>(t, w, Qm);
#pragma unroll
    for (int r = 0; r < M; ++r) wp[r] = w[r] * t.mu[r];
    flux<LAW, D, M, NV>(t, wp, Q);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double mk = eq_comp(t, wp, Q, k, r);
        const double f = (double)fr[k][r] + (mk - eq_comp(t, w, Qm, k, r));
        out[k][r] = (T)(f + t.omega * (mk - f));
      }
  } else {
    flux<LAW, D, M, NV>(t, w, Q);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double mk = eq_comp(t, w, Q, k, r);
        const double f = (double)fr[k][r];
        out[k][r] = (T)(f + t.omega * (mk - f));
      }
  }
}

template <typename T, int LAW, int D, int M, int NV>
__device__ __forceinline__ void relax_node(const T* fin, T* fout, int64_t plane,
                                           const EqTab<D, M, NV>& t, int64_t i) {
  T fr[NV][M], out[NV][M];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) fr[k][r] = fin[(int64_t)(k * M + r) * plane + i];
  relax_values<T, LAW, D, M, NV>(t, fr, out);
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) fout[(int64_t)(k * M + r) * plane + i] = out[k][r];
}

template <typename T, int LAW, int D, int M, int NV>
// (the table is read from device memory where it is used: as a kernel
// argument its FP64 coefficients would be held in registers throughout)
__global__ __launch_bounds__(256) void k_relax(const T* fin, T* fout, int64_t plane,
                                               const EqTab<D, M, NV>* __restrict__ t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  relax_node<T, LAW, D, M, NV>(fin, fout, plane, *t, i);
}

// The same with VW consecutive nodes per thread: one 16-byte load and store
// per (velocity, component) plane (plane divisible by VW).
template <typename T, int LAW, int D, int M, int NV, int VW>
__global__ __launch_bounds__(256) void k_relax_vec(const T* fin, T* fout, int64_t plane,
                                                   const EqTab<D, M, NV>* __restrict__ tp) {
  const int64_t i0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * VW;
  if (i0 >= plane) return;
  struct alignas(16) V { T v[VW]; };
  V in[NV][M], out[NV][M];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r)
      in[k][r] = *reinterpret_cast<const V*>(fin + (int64_t)(k * M + r) * plane + i0);
#pragma unroll
  for (int u = 0; u < VW; ++u) {
    T fr[NV][M], o[NV][M];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) fr[k][r] = in[k][r].v[u];
    relax_values<T, LAW, D, M, NV>(*tp, fr, o);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) out[k][r].v[u] = o[k][r];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r)
      *reinterpret_cast<V*>(fout + (int64_t)(k * M + r) * plane + i0) = out[k][r];
}

// Relaxation of many problems of one (law, d, m, n_vel) in one launch; the
// blocks of all problems are numbered consecutively (start[] prefix).
template <typename T, int LAW, int D, int M, int NV>
__global__ __launch_bounds__(256) void k_relax_batch(const RelaxTask<D, M, NV>* __restrict__ tasks,
                                                     const int64_t* __restrict__ start, int ntask) {
  const int64_t gb = blockIdx.x;
  int pid = 0;
  while (gb >= start[pid + 1]) ++pid;
  const RelaxTask<D, M, NV>& t = tasks[pid];
  const int64_t i = (gb - start[pid]) * blockDim.x + threadIdx.x;
  if (i >= t.plane) return;
  relax_node<T, LAW, D, M, NV>((const T*)t.fin, (T*)t.fout, t.plane, t.t, i);
}

// W = sum_k f_k (FP64) at the nodes i0 .. i0 + n - 1, written W[(i - i0) m + r].
template <typename T>
__global__ __launch_bounds__(256) void k_moments(const T* __restrict__ f, double* __restrict__ W,
                                                 int64_t plane, int64_t i0, int64_t n, int m,
                                                 int nv) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = i0 + j;
  for (int r = 0; r < m; ++r) {
    double s = 0.0;
    for (int k = 0; k < nv; ++k) s += (double)f[(int64_t)(k * m + r) * plane + i];
    W[j * m + r] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_get_kinetic(const T* __restrict__ f, double* __restrict__ F,
                                                     int64_t plane, int m, int nv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  for (int k = 0; k < nv; ++k)
    for (int r = 0; r < m; ++r)
      F[((int64_t)k * plane + i) * m + r] = (double)f[(int64_t)(k * m + r) * plane + i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_set_kinetic(const double* __restrict__ F, T* __restrict__ f,
                                                     int64_t plane, int m, int nv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  for (int k = 0; k < nv; ++k)
    for (int r = 0; r < m; ++r)
      f[(int64_t)(k * m + r) * plane + i] = (T)F[((int64_t)k * plane + i) * m + r];
}

template <typename T>
__global__ __launch_bounds__(256) void k_check_finite(const T* __restrict__ f, int64_t n,
                                                      int* __restrict__ flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < n; i += stride) bad |= !isfinite((double)f[i]);
  if (bad) flag[0] = 1;  // every writer stores the same value
}

// Largest wave speed of a compressible Euler state W [node][d + 2] (FP64):
// max over nodes and axes of |u_i| + c, c = sqrt(gamma p / rho).  A node
// without a real wave speed (rho <= 0, p <= 0, NaN) counts as +inf.  The
// result is reduced as the bits of a non-negative double with an unsigned
// maximum, which orders non-negative doubles like their values.
__global__ __launch_bounds__(256) void k_euler_wave_speed(const double* __restrict__ W,
                                                          int64_t nodes, int dim, double gamma,
                                                          unsigned long long* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double best = 0.0;
  for (; i < nodes; i += stride) {
    const double* w = W + i * (dim + 2);
    const double rho = w[0], E = w[dim + 1];
    double ke = 0.0, umax = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double u = w[1 + a] / rho;
      ke += u * u;
      umax = fmax(umax, fabs(u));
    }
    const double pr = (gamma - 1.0) * (E - 0.5 * rho * ke);
    // (a NaN anywhere fails one of the comparisons: +inf)
    const double sp = (rho > 0.0 && pr > 0.0) ? umax + sqrt(gamma * pr / rho) : INFINITY;
    best = fmax(best, sp);
  }
  for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

// ====================================================== plain sweep

// One subdomain iteration p of the downwind sweep for every (velocity,
// component): one thread per (line, subdomain), walking the S cells of its
// subdomain in downwind order (the level loop of Sec. 3.2).  Inflow at the
// subdomain's first cell: tr_prev (the upwind subdomain's outflow of iterate
// p-1), or for p = 1 the state at t^{n-1} (eq:ibvp2/3).  Writes this iterate's
// outflow to tr_out and, when f_new is not null, the whole iterate.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_sweep_plain(const T* __restrict__ f_old,
                                                     T* __restrict__ f_new,
                                                     const T* __restrict__ tr_prev,
                                                     T* __restrict__ tr_out, Geom g,
                                                     SweepTab<T> tab, BndRef<T> bd) {
  const int kc = blockIdx.y;
  const int k = kc / g.m;
  const int a = tab.axis[k];
  const int sg = tab.sign[k];
  const int Na = g.N[a];
  const int S = g.S[a];
  const int nseg = Na / S;
  const int per = g.nn / P;                       // other-node combinations
  const int64_t nlines = (g.ncell / Na) * per;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nlines * nseg) return;
  const int seg = (int)(t / nlines);
  const int64_t line = t - (int64_t)seg * nlines;
  const int on = (int)(line % per);
  int64_t oc = line / per;
  // cell of the line with coordinate 0 along a
  int64_t cell0 = 0;
  int64_t cmul = 1;
  int64_t cs = 1;
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
  const int node0 = other_node_offset(on, a, P, g.dim);
  const int64_t base = ((int64_t)kc * g.ncell + cell0) * g.nn + node0;
  const int64_t cstride = cs * g.nn;
  auto phys = [&](int b) { return sg > 0 ? b : P - 1 - b; };

  T C[P][P], e1[P], eth[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    e1[r] = tab.e1[k][r];
    eth[r] = tab.eth[k][r];
#pragma unroll
    for (int c = 0; c < P; ++c) C[r][c] = tab.C[k][r * P + c];
  }

  T t_old, t_new;
  const int bside = sg > 0 ? 0 : 1;
  if (seg == 0 && bd.old != nullptr && bd.off[a][bside] >= 0) {
    // first subdomain on a Dirichlet axis: the prescribed inflow (the line
    // index is the boundary node's index on the face)
    const int64_t bi = (int64_t)kc * bd.nb + bd.off[a][bside] + line;
    t_old = bd.old[bi];
    t_new = bd.neu[bi];
  } else {
    const int j = seg * S;  // downwind index of the first cell
    const int r = sg > 0 ? j : Na - 1 - j;
    const int ru = sg > 0 ? (r == 0 ? Na - 1 : r - 1) : (r == Na - 1 ? 0 : r + 1);
    t_old = f_old[base + ru * cstride + phys(P - 1) * ns];
    if (tr_prev) {
      const int su = seg == 0 ? nseg - 1 : seg - 1;
      t_new = tr_prev[(int64_t)kc * g.tr_stride + (int64_t)su * nlines + line];
    } else {
      t_new = t_old;
    }
  }
  for (int jj = 0; jj < S; ++jj) {
    const int j = seg * S + jj;
    const int r = sg > 0 ? j : Na - 1 - j;
    T fo[P];
#pragma unroll
    for (int b = 0; b < P; ++b) fo[b] = f_old[base + r * cstride + phys(b) * ns];
    T fn[P];
#pragma unroll
    for (int b = 0; b < P; ++b) {
      T s = T(0);
#pragma unroll
      for (int c = 0; c < P; ++c) s += C[b][c] * fo[c];
      fn[b] = s + e1[b] * t_old + eth[b] * t_new;
    }
    if (f_new) {
#pragma unroll
      for (int b = 0; b < P; ++b) f_new[base + r * cstride + phys(b) * ns] = fn[b];
    }
    t_old = fo[P - 1];
    t_new = fn[P - 1];
  }
  tr_out[(int64_t)kc * g.tr_stride + (int64_t)seg * nlines + line] = t_new;
}

// ============================================================ launchers

namespace {

template <int LAW, int D, int M, int NV>
struct EqCombo {
  using Tab = EqTab<D, M, NV>;
  static bool build(const std::vector<double>& lp, const std::vector<double>& a,
                    const std::vector<double>& b, double omega, const std::vector<double>& mu,
                    std::vector<unsigned char>& blob) {
    Tab t{};
    if (LAW == KDS_LAW_LINEAR) {
      if ((int)lp.size() < D * M * M) return false;
      for (int i = 0; i < D; ++i)
        for (int r = 0; r < M; ++r)
          for (int q = 0; q < M; ++q) t.A[i][r][q] = lp[(i * M + r) * M + q];
    } else {
      if (lp.empty()) return false;
      t.gamma = lp[0];
    }
    for (int k = 0; k < NV; ++k) {
      t.a[k] = a[k];
      for (int i = 0; i < D; ++i) t.b[k][i] = b[k * D + i];
    }
    t.omega = omega;
    t.has_source = mu.empty() ? 0 : 1;
    for (int r = 0; r < M; ++r) t.mu[r] = mu.empty() ? 1.0 : mu[r];
    blob.resize(sizeof(Tab));
    std::memcpy(blob.data(), &t, sizeof(Tab));
    return true;
  }
  template <typename T>
  static hipError_t init(const Geom& g, const void* eq, const double* W, void* f, hipStream_t s) {
    const int64_t plane = g.ncell * g.nn;
    hipLaunchKernelGGL((k_init<T, LAW, D, M, NV>), dim3(blocks_for(plane)), dim3(256), 0, s, W,
                       (T*)f, plane, *(const Tab*)eq);
    return hipGetLastError();
  }
  static size_t task_bytes() { return sizeof(RelaxTask<D, M, NV>); }
  static void pack_task(const void* eq, const void* fin, void* fout, int64_t plane, void* out) {
    RelaxTask<D, M, NV> t;
    t.fin = fin;
    t.fout = fout;
    t.plane = plane;
    std::memcpy(&t.t, eq, sizeof(Tab));
    std::memcpy(out, &t, sizeof(t));
  }
  template <typename T>
  static hipError_t relax_batch(const void* tasks, const int64_t* start, int ntask, int64_t nblocks,
                                hipStream_t s) {
    hipLaunchKernelGGL((k_relax_batch<T, LAW, D, M, NV>), dim3((unsigned)nblocks), dim3(256), 0, s,
                       (const RelaxTask<D, M, NV>*)tasks, start, ntask);
    return hipGetLastError();
  }
  template <typename T>
  static hipError_t relax(const Geom& g, const void* eq, const void* fin, void* fout, bool vec,
                          hipStream_t s) {
    const int64_t plane = g.ncell * g.nn;
    constexpr int VW = 16 / sizeof(T);
    if (vec && plane % VW == 0)
      hipLaunchKernelGGL((k_relax_vec<T, LAW, D, M, NV, VW>), dim3(blocks_for(plane / VW)), dim3(256),
                         0, s, (const T*)fin, (T*)fout, plane, (const Tab*)eq);
    else
      hipLaunchKernelGGL((k_relax<T, LAW, D, M, NV>), dim3(blocks_for(plane)), dim3(256), 0, s,
                         (const T*)fin, (T*)fout, plane, (const Tab*)eq);
    return hipGetLastError();
  }
};

struct ComboEntry {
  int law, dim, m, nv;
  bool (*build)(const std::vector<double>&, const std::vector<double>&, const std::vector<double>&,
                double, const std::vector<double>&, std::vector<unsigned char>&);
  hipError_t (*init64)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*init32)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*relax64)(const Geom&, const void*, const void*, void*, bool, hipStream_t);
  hipError_t (*relax32)(const Geom&, const void*, const void*, void*, bool, hipStream_t);
  size_t (*task_bytes)();
  void (*pack_task)(const void*, const void*, void*, int64_t, void*);
  hipError_t (*batch64)(const void*, const int64_t*, int, int64_t, hipStream_t);
  hipError_t (*batch32)(const void*, const int64_t*, int, int64_t, hipStream_t);
};

#define KDS_COMBO(LAW, D, M, NV)                                                          \
  ComboEntry {                                                                            \
    LAW, D, M, NV, &EqCombo<LAW, D, M, NV>::build, &EqCombo<LAW, D, M, NV>::init<double>, \
        &EqCombo<LAW, D, M, NV>::init<float>, &EqCombo<LAW, D, M, NV>::relax<double>,     \
        &EqCombo<LAW, D, M, NV>::relax<float>, &EqCombo<LAW, D, M, NV>::task_bytes,       \
        &EqCombo<LAW, D, M, NV>::pack_task, &EqCombo<LAW, D, M, NV>::relax_batch<double>, \
        &EqCombo<LAW, D, M, NV>::relax_batch<float>                                       \
  }

// (law, dim, m, n_vel) combinations with compiled pointwise kernels
const ComboEntry kCombos[] = {
    KDS_COMBO(KDS_LAW_LINEAR, 1, 1, 2), KDS_COMBO(KDS_LAW_LINEAR, 1, 2, 2),
    KDS_COMBO(KDS_LAW_LINEAR, 2, 1, 4), KDS_COMBO(KDS_LAW_LINEAR, 2, 3, 4),
    KDS_COMBO(KDS_LAW_LINEAR, 3, 1, 6), KDS_COMBO(KDS_LAW_LINEAR, 3, 4, 6),
    KDS_COMBO(KDS_LAW_LINEAR, 3, 6, 6), KDS_COMBO(KDS_LAW_LINEAR, 3, 6, 4),
    KDS_COMBO(KDS_LAW_EULER, 1, 3, 2),
    KDS_COMBO(KDS_LAW_EULER, 2, 4, 4),  KDS_COMBO(KDS_LAW_EULER, 3, 5, 6),
};

const ComboEntry* find_combo(int law, int dim, int m, int nv) {
  for (const auto& c : kCombos)
    if (c.law == law && c.dim == dim && c.m == m && c.nv == nv) return &c;
  return nullptr;
}

template <typename T>
hipError_t sweep_plain_t(const Geom& g, const void* tab, const void* f_old, void* f_new,
                         const void* tr_prev, void* tr_out, const BndArgs& bnd, hipStream_t s) {
  const SweepTab<T>& t = *(const SweepTab<T>*)tab;
  int64_t maxthreads = 0;
  for (int k = 0; k < g.nv; ++k) {
    const int a = t.axis[k];
    const int64_t n = (g.ncell / g.N[a]) * (g.nn / g.P) * (g.N[a] / g.S[a]);
    if (n > maxthreads) maxthreads = n;
  }
  dim3 grid(blocks_for(maxthreads), g.nv * g.m);
  switch (g.P) {
#define KDS_PLAIN(PP)                                                                          \
  case PP:                                                                                     \
    hipLaunchKernelGGL((k_sweep_plain<T, PP>), grid, dim3(256), 0, s, (const T*)f_old, (T*)f_new, \
                       (const T*)tr_prev, (T*)tr_out, g, t, bnd_ref<T>(bnd));                  \
    break;
    KDS_PLAIN(1)
    KDS_PLAIN(2)
    KDS_PLAIN(3)
    KDS_PLAIN(4)
#undef KDS_PLAIN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool build_eq_blob(int law, int dim, int m, int nv, const std::vector<double>& law_params,
                   const std::vector<double>& a, const std::vector<double>& b, double omega,
                   const std::vector<double>& mu, std::vector<unsigned char>& blob) {
  const ComboEntry* c = find_combo(law, dim, m, nv);
  if (!c) return false;
  return c->build(law_params, a, b, omega, mu, blob);
}

// The combination was validated by build_eq_blob at create time.
static const ComboEntry* combo_of(int law, const Geom& g) { return find_combo(law, g.dim, g.m, g.nv); }

hipError_t launch_init(int prec, int law, const Geom& g, const void* eq, const double* W, void* f,
                       hipStream_t s) {
  const ComboEntry* c = combo_of(law, g);
  if (!c) return hipErrorInvalidValue;
  return prec == KDS_FP64 ? c->init64(g, eq, W, f, s) : c->init32(g, eq, W, f, s);
}

hipError_t launch_relax(int prec, int law, const Geom& g, const void* eq, const void* fin,
                        void* fout, bool vec, hipStream_t s) {
  const ComboEntry* c = combo_of(law, g);
  if (!c) return hipErrorInvalidValue;
  return prec == KDS_FP64 ? c->relax64(g, eq, fin, fout, vec, s)
                          : c->relax32(g, eq, fin, fout, vec, s);
}

hipError_t launch_moments_range(int prec, const Geom& g, const void* f, int64_t i0, int64_t n,
                                double* W, hipStream_t s) {
  const int64_t plane = g.ncell * g.nn;
  if (i0 < 0 || n < 0 || i0 + n > plane) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_moments<double>, dim3(blocks_for(n)), dim3(256), 0, s,
                       (const double*)f, W, plane, i0, n, g.m, g.nv);
  else
    hipLaunchKernelGGL(k_moments<float>, dim3(blocks_for(n)), dim3(256), 0, s,
                       (const float*)f, W, plane, i0, n, g.m, g.nv);
  return hipGetLastError();
}

hipError_t launch_moments(int prec, const Geom& g, const void* f, double* W, hipStream_t s) {
  return launch_moments_range(prec, g, f, 0, g.ncell * g.nn, W, s);
}

// ======================================================= static scratch
//
// Device memory of the entry points that allocate nothing (kds_moments_static):
// a fixed array in the code object, one copy per GPU, held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (on
// the host the name is not a device address): scratch_address() looks the
// array's device address up once per device, with that device current, and
// every use goes through that address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_get_kinetic(int prec, const Geom& g, const void* f, double* F, hipStream_t s) {
  const int64_t plane = g.ncell * g.nn;
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_get_kinetic<double>, dim3(blocks_for(plane)), dim3(256), 0, s,
                       (const double*)f, F, plane, g.m, g.nv);
  else
    hipLaunchKernelGGL(k_get_kinetic<float>, dim3(blocks_for(plane)), dim3(256), 0, s,
                       (const float*)f, F, plane, g.m, g.nv);
  return hipGetLastError();
}

hipError_t launch_set_kinetic(int prec, const Geom& g, const double* F, void* f, hipStream_t s) {
  const int64_t plane = g.ncell * g.nn;
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_set_kinetic<double>, dim3(blocks_for(plane)), dim3(256), 0, s, F,
                       (double*)f, plane, g.m, g.nv);
  else
    hipLaunchKernelGGL(k_set_kinetic<float>, dim3(blocks_for(plane)), dim3(256), 0, s, F,
                       (float*)f, plane, g.m, g.nv);
  return hipGetLastError();
}

hipError_t launch_check_finite(int prec, const Geom& g, const void* f, int* flag, hipStream_t s) {
  const int64_t n = g.ncell * g.nn * g.m * g.nv;
  const unsigned nb = (unsigned)std::min<int64_t>(blocks_for(n), 4096);
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_check_finite<double>, dim3(nb), dim3(256), 0, s, (const double*)f, n, flag);
  else
    hipLaunchKernelGGL(k_check_finite<float>, dim3(nb), dim3(256), 0, s, (const float*)f, n, flag);
  return hipGetLastError();
}

hipError_t launch_euler_wave_speed(const double* W, int64_t nodes, int dim, double gamma,
                                   unsigned long long* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(nodes), 1024));
  hipLaunchKernelGGL(k_euler_wave_speed, dim3(nb), dim3(256), 0, s, W, nodes, dim, gamma, out);
  return hipGetLastError();
}

hipError_t launch_sweep_plain(int prec, const Geom& g, const void* tab, const void* f_old,
                              void* f_new, const void* tr_prev, void* tr_out, const BndArgs& bnd,
                              hipStream_t s) {
  return prec == KDS_FP64 ? sweep_plain_t<double>(g, tab, f_old, f_new, tr_prev, tr_out, bnd, s)
                          : sweep_plain_t<float>(g, tab, f_old, f_new, tr_prev, tr_out, bnd, s);
}

hipError_t launch_sweep_line(int prec, const Geom& g, const void* tab, const LinePlan& plan,
                             void* f, const BndArgs& bnd, hipStream_t s) {
  return prec == KDS_FP64 ? sweep_line_f64(g, tab, plan, f, bnd, s)
                          : sweep_line_f32(g, tab, plan, f, bnd, s);
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, T* __restrict__ dst,
                                              int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(int prec, const void* src, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_copy<double>, dim3(blocks_for(n)), dim3(256), 0, s, (const double*)src,
                       (double*)dst, n);
  else
    hipLaunchKernelGGL(k_copy<float>, dim3(blocks_for(n)), dim3(256), 0, s, (const float*)src,
                       (float*)dst, n);
  return hipGetLastError();
}


size_t relax_task_bytes(int law, int dim, int m, int nv) {
  const ComboEntry* c = find_combo(law, dim, m, nv);
  return c ? c->task_bytes() : 0;
}

bool pack_relax_task(int law, int dim, int m, int nv, const void* eq, const void* fin, void* fout,
                     int64_t plane, void* out) {
  const ComboEntry* c = find_combo(law, dim, m, nv);
  if (!c) return false;
  c->pack_task(eq, fin, fout, plane, out);
  return true;
}

hipError_t launch_relax_batch(int prec, int law, int dim, int m, int nv, const void* tasks,
                              const int64_t* start, int ntask, int64_t nblocks, hipStream_t s) {
  const ComboEntry* c = find_combo(law, dim, m, nv);
  if (!c) return hipErrorInvalidValue;
  return prec == KDS_FP64 ? c->batch64(tasks, start, ntask, nblocks, s)
                          : c->batch32(tasks, start, ntask, nblocks, s);
}

size_t line_task_bytes(int prec) {
  return prec == KDS_FP64 ? line_task_bytes_f64() : line_task_bytes_f32();
}

void pack_line_task(int prec, void* f, const Geom& g, const void* tab, const LinePlan& pl,
                    const BndArgs& bnd, void* out) {
  if (prec == KDS_FP64)
    pack_line_task_f64(f, g, tab, pl, bnd, out);
  else
    pack_line_task_f32(f, g, tab, pl, bnd, out);
}

hipError_t launch_sweep_line_batch(int prec, int P, int dim, bool rounds, bool dir,
                                   const void* tasks, const int64_t* start, int ntask,
                                   int64_t nblocks, int threads, size_t lds_elems, hipStream_t s) {
  return prec == KDS_FP64 ? sweep_line_batch_f64(P, dim, rounds, dir, tasks, start, ntask,
                                                 nblocks, threads, lds_elems, s)
                          : sweep_line_batch_f32(P, dim, rounds, dir, tasks, start, ntask,
                                                 nblocks, threads, lds_elems, s);
}

// Allow the line kernels (single and batched) dynamic LDS up to `bytes`
// (workgroups above 64 KiB need the attribute).  Once per size and process.
hipError_t line_kernels_allow_lds(size_t bytes) {
  static size_t done = 0;
  if (bytes <= 64 * 1024 || bytes <= done) return hipSuccess;
  hipError_t e = line_allow_lds_f32(bytes);
  if (e == hipSuccess) e = line_allow_lds_f64(bytes);
  if (e == hipSuccess) done = bytes;
  else (void)hipGetLastError();
  return e;
}

}  // namespace kds
