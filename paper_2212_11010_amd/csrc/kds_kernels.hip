// kds_kernels.hip -- gfx950 kernels of libkds.
//
// Kinetic state layout in HBM: f[k][c][cell][node] (velocity, component,
// cell x-fastest, node x-fastest), stored in T = double or float.  Every
// (velocity, component) pair is one contiguous plane of ncell * nn values, so
// the pointwise kernels (init, relaxation, moments) read one coalesced stream
// per (k, c) and the sweeps read whole cells.
//
// Transport (Sec. 3.1 eq:dg_imp, Sec. 3.2, Sec. 5.1 eq:ibvp).  Every velocity
// here is parallel to a grid axis, so the implicit upwind DG system of one
// velocity splits exactly into independent 1-D problems along grid lines
// (faces with V.N = 0 carry no flux).  On one line, in downwind order, cell j
// obeys
//     f_j^n = C f_j^{n-1} + e1 t_j^{n-1} + eth t_j^n,
// t_j = outflow node of the upwind neighbour (node P-1 in downwind order),
// e1 = (1 - theta) e, eth = theta e.  Inside a subdomain t_j^n = f_{j-1}^n[P-1];
// at the first cell of a subdomain, iterate p takes t^n from the upwind
// subdomain's iterate p-1 (iterate 0 = the state at t^{n-1}).
#include <algorithm>
#include <cstring>

#include "kds_internal.h"

namespace kds {

// ================================================================ helpers

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

// ============================================================ equilibrium

// M_k(W) = a_k W + sum_i b_{k,i} Q^i(W) (moment conditions, eq:maxwell_def),
// evaluated in FP64.
template <int LAW, int D, int M, int NV>
__device__ __forceinline__ void equilibrium(const EqTab<D, M, NV>& t, const double (&W)[M],
                                            double (&Mk)[NV][M]) {
  double Q[D][M];
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
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double s = t.a[k] * W[r];
#pragma unroll
      for (int i = 0; i < D; ++i) s += t.b[k][i] * Q[i][r];
      Mk[k][r] = s;
    }
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
__device__ __forceinline__ void relax_node(const T* fin, T* fout, int64_t plane,
                                           const EqTab<D, M, NV>& t, int64_t i) {
  double fv[NV][M];
  double w[M];
#pragma unroll
  for (int r = 0; r < M; ++r) w[r] = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r) {
      fv[k][r] = (double)fin[(int64_t)(k * M + r) * plane + i];
      w[r] += fv[k][r];
    }
  double Mk[NV][M];
  if (t.has_source) {
    // Crank-Nicolson source step on W; the kinetic data take the equilibrium
    // part of the change so that sum_k f_k = W+ before relaxing towards M(W+)
    double Mm[NV][M];
    equilibrium<LAW, D, M, NV>(t, w, Mm);
#pragma unroll
    for (int r = 0; r < M; ++r) w[r] *= t.mu[r];
    equilibrium<LAW, D, M, NV>(t, w, Mk);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) fv[k][r] += Mk[k][r] - Mm[k][r];
  } else {
    equilibrium<LAW, D, M, NV>(t, w, Mk);
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r)
      fout[(int64_t)(k * M + r) * plane + i] = (T)(fv[k][r] + t.omega * (Mk[k][r] - fv[k][r]));
}

template <typename T, int LAW, int D, int M, int NV>
__global__ __launch_bounds__(256) void k_relax(const T* fin, T* fout, int64_t plane,
                                               EqTab<D, M, NV> t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  relax_node<T, LAW, D, M, NV>(fin, fout, plane, t, i);
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

template <typename T>
__global__ __launch_bounds__(256) void k_moments(const T* __restrict__ f, double* __restrict__ W,
                                                 int64_t plane, int m, int nv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
  for (int r = 0; r < m; ++r) {
    double s = 0.0;
    for (int k = 0; k < nv; ++k) s += (double)f[(int64_t)(k * m + r) * plane + i];
    W[i * m + r] = s;
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

// Value of the lane `OFF` places lower in the same 16-lane row (DPP
// row_shr); lanes without a source get 0.  Used only where every scan
// segment lies inside one row.
template <typename T, int OFF>
__device__ __forceinline__ T dpp_row_shr(T v);

template <>
__device__ __forceinline__ float dpp_row_shr<float, 1>(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
}
#define KDS_DPP_F32(OFF)                                                                        \
  template <>                                                                                   \
  __device__ __forceinline__ float dpp_row_shr<float, OFF>(float v) {                           \
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + (OFF), 0xf, \
                                                      0xf, true));                              \
  }                                                                                             \
  template <>                                                                                   \
  __device__ __forceinline__ double dpp_row_shr<double, OFF>(double v) {                        \
    const long long b = __double_as_longlong(v);                                                \
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x110 + (OFF), 0xf,  \
                                               0xf, true);                                      \
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + (OFF), 0xf, 0xf,      \
                                               true);                                           \
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);                      \
  }
KDS_DPP_F32(2)
KDS_DPP_F32(4)
KDS_DPP_F32(8)
#undef KDS_DPP_F32
template <>
__device__ __forceinline__ double dpp_row_shr<double, 1>(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x111, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Copy between a bundle of rows (R contiguous values each, rows rowstride
// apart, starting at rowbase) and the LDS tile (rows of R values, packed).
// Vectors of VW elements when the rows allow it; addresses advance
// incrementally (one division per thread) and U independent accesses are
// issued before any is consumed, so global latency overlaps.
template <typename T, int VW>
struct VecT;
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<float, 2> { using type = float2; };
template <> struct VecT<float, 4> { using type = float4; };
template <> struct VecT<double, 1> { using type = double; };
template <> struct VecT<double, 2> { using type = double2; };

template <typename T, int VW, bool LOAD>
__device__ __forceinline__ void copy_rows(T* __restrict__ f, T* tile, int64_t rowbase,
                                          int64_t rowstride, int R, int rows) {
  using VT = typename VecT<T, VW>::type;
  constexpr int U = 16;
  const int RV = R / VW;  // vectors per row
  const int total = rows * RV;
  const int bs = blockDim.x;
  const int64_t rs = rowstride / VW;
  VT* g = reinterpret_cast<VT*>(f + rowbase);
  VT* t = reinterpret_cast<VT*>(tile);
  int e = threadIdx.x;
  int r = e / RV;
  int q = e - r * RV;
  const int dr = bs / RV;
  const int dq = bs - dr * RV;
  int64_t go = (int64_t)r * rs + q;
  const int64_t gstep = (int64_t)dr * rs + dq;
  const int64_t gwrap = rs - RV;
  while (e < total) {
    int64_t ga[U];
    int ta[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ga[u] = go;
      ta[u] = e;
      e += bs;
      go += gstep;
      q += dq;
      if (q >= RV) {
        q -= RV;
        go += gwrap;
      }
    }
    if (LOAD) {
      // unconditional loads (slots past the end re-read element 0), so the
      // U loads stay in flight together
      VT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = g[ta[u] < total ? ga[u] : 0];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ta[u] < total) t[ta[u]] = v[u];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ta[u] < total) g[ga[u]] = t[ta[u]];
    }
  }
}

template <typename T, bool LOAD>
__device__ __forceinline__ void copy_tile(T* __restrict__ f, T* tile, int64_t rowbase,
                                          int64_t rowstride, int R, int rows) {
  // one contiguous block: treat as a single row
  if (rowstride == R) {
    R *= rows;
    rows = 1;
  }
  constexpr int VMAX = 16 / sizeof(T);
  if (VMAX >= 4 && R % 4 == 0 && rowbase % 4 == 0 && rowstride % 4 == 0) {
    copy_rows<T, (VMAX >= 4 ? 4 : 1), LOAD>(f, tile, rowbase, rowstride, R, rows);
  } else if (R % 2 == 0 && rowbase % 2 == 0 && rowstride % 2 == 0) {
    copy_rows<T, 2, LOAD>(f, tile, rowbase, rowstride, R, rows);
  } else {
    copy_rows<T, 1, LOAD>(f, tile, rowbase, rowstride, R, rows);
  }
}

// ======================================================= line sweep

// All K subdomain iterations of whole grid lines in one pass.
//
// A workgroup holds a bundle of complete columns of cells along the velocity
// axis (one (velocity, component) pair) in LDS, laid out [column][cell][node].
// Each lane owns Q consecutive cells of one column and ALL the 1-D lines
// through them (the (p+1)^(d-1) node rows parallel to the axis), so its cells
// are read from LDS as contiguous vectors and every node offset is a
// compile-time constant.  On a line, in downwind order, the outflow values
// obey the first-order recurrence
//     t_{j+1} = beta_j + g t_j,  beta_j = (C f_j^{n-1})[P-1] + e1[P-1] t_j^{n-1},
//     g = eth[P-1],
// restarted at every subdomain start.  A segmented scan over the lanes of a
// subdomain (DPP row shifts) gives each cell the inflow q_j it would receive
// with zero inflow at its subdomain start, and each subdomain s its
// zero-inflow outflow P_s.  With G = g^S, the outflow of subdomain s at
// iterate p is T_s^p = P_s + G T_{s-1}^{p-1} (T^0 = outflow of f^{n-1}), and the
// final iterate K has inflow t_in(s) = T_{s-1}^{K-1}, so
// t_j^n = q_j + g^{j - j_s} t_in(s).  This is the linear algebra of K literal
// sweeps (eq:ibvp), evaluated in another order; the state is read and
// written once per step.

// Copy between rows of a y/z bundle (row j = cell j along the axis: ncols
// adjacent cells, ncols*NN contiguous values at gbase + j*rowstride) and the
// LDS tile laid out [column][cell][node] (column stride CS).  Each thread
// owns one vector position of a row and walks the rows; U rows are in flight.
template <typename T, int NN, int VW, bool LOAD>
__device__ __forceinline__ void copy_cols_v(T* __restrict__ f, T* tile, int64_t gbase,
                                            int64_t rowstride, int ncols, int Na, int CS) {
  using VT = typename VecT<T, VW>::type;
  constexpr int U = 32 / VW;
  const int RWV = ncols * NN / VW;  // vectors per row
  const int rpi = blockDim.x / RWV; // rows per pass
  const int tid = threadIdx.x;
  if (rpi == 0 || tid >= rpi * RWV) return;
  const int jj = tid / RWV;
  const int ev = tid - jj * RWV;
  int tl[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) {
    const int e = ev * VW + i;
    const int c = e / NN;
    tl[i] = c * CS + jj * NN + (e - c * NN);
  }
  VT* g = reinterpret_cast<VT*>(f + gbase) + ev;
  const int64_t rs = rowstride / VW;
  for (int j0 = 0; j0 < Na; j0 += U * rpi) {
    if (LOAD) {
      VT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + jj + u * rpi;
        v[u] = g[(j < Na ? j : 0) * rs];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + jj + u * rpi;
        if (j < Na) {
          const T* vp = reinterpret_cast<const T*>(&v[u]);
#pragma unroll
          for (int i = 0; i < VW; ++i) tile[tl[i] + (j0 + u * rpi) * NN] = vp[i];
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + jj + u * rpi;
        if (j < Na) {
          VT v;
          T* vp = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int i = 0; i < VW; ++i) vp[i] = tile[tl[i] + (j0 + u * rpi) * NN];
          g[j * rs] = v;
        }
      }
    }
  }
}

template <typename T, int NN, bool LOAD>
__device__ __forceinline__ void copy_cols(T* __restrict__ f, T* tile, int64_t gbase,
                                          int64_t rowstride, int ncols, int Na, int CS) {
  const int RW = ncols * NN;
  constexpr int VMAX = 16 / sizeof(T);
  if (VMAX >= 4 && RW % 4 == 0 && gbase % 4 == 0 && rowstride % 4 == 0 && RW / 4 <= (int)blockDim.x)
    copy_cols_v<T, NN, (VMAX >= 4 ? 4 : 1), LOAD>(f, tile, gbase, rowstride, ncols, Na, CS);
  else if (RW % 2 == 0 && gbase % 2 == 0 && rowstride % 2 == 0 && RW / 2 <= (int)blockDim.x)
    copy_cols_v<T, NN, 2, LOAD>(f, tile, gbase, rowstride, ncols, Na, CS);
  else
    copy_cols_v<T, NN, 1, LOAD>(f, tile, gbase, rowstride, ncols, Na, CS);
}

template <int P, int DIM>
struct ColShape {
  static constexpr int NN = P * (DIM > 1 ? P : 1) * (DIM > 2 ? P : 1);
  static constexpr int PER = NN / P;  // lines through a cell along one axis
};

// offset inside a cell of the node with index b on `axis` and index `o` (a
// mixed-radix number over the other axes, x fastest)
template <int P, int DIM, int AXIS>
__device__ constexpr int node_of(int o, int b) {
  int off = 0, mul = 1;
  for (int ax = 0; ax < DIM; ++ax) {
    if (ax == AXIS) {
      off += b * mul;
    } else {
      off += (o % P) * mul;
      o /= P;
    }
    mul *= P;
  }
  return off;
}

struct LineLane {
  int Q, Ls, sl, end_up, src_prev;
  int nseg, s_me, lbase;
  bool dpp_ok;
  bool first;  // owns the first cells of the line in downwind order
};

// One lane's part of the line solve.  d[q][node]: my Q cells in downwind
// order (node indices physical); updated in place to the new state.
// Lines O0 .. O0+PER-1 of the cells (groups keep the live registers small).
template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, int O0, int PER>
__device__ __forceinline__ void line_group(T (&d)[QMAX][NN], const LineLane& ln,
                                           const T (&C)[P][P], const T (&e1)[P], const T (&eth)[P],
                                           T gg, T G, int K, const T* bo, const T* bn) {
  static_assert(NN == ColShape<P, DIM>::NN, "cell size");
  // Dirichlet axis: bo / bn point at this line's boundary values (inflow of
  // the first subdomain at the old / new time); nullptr on a periodic axis
  const bool dir = bo != nullptr;
  T bold[PER], bnew[PER];
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    bold[o] = dir ? bo[O0 + o] : T(0);
    bnew[o] = dir ? bn[O0 + o] : T(0);
  }
  // physical node of downwind node b along the axis, line O0 + o
#define KDS_ND(o, b) node_of<P, DIM, AXIS>(O0 + (o), SIGN > 0 ? (b) : P - 1 - (b))
  T last_old[PER], t_old0[PER], mB[PER];
  T beta[PER][QMAX];
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T lo = T(0);
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
      if (q == ln.Q - 1) lo = d[q][KDS_ND(o, P - 1)];
    last_old[o] = lo;
  }
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    t_old0[o] = __shfl(last_old[o], ln.src_prev, 64);
    if (dir && ln.first) t_old0[o] = bold[o];
  }
  // zero-inflow recurrence over my cells
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T to = t_old0[o], x = T(0);
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (q < ln.Q) {
        T bq = e1[P - 1] * to;
#pragma unroll
        for (int c = 0; c < P; ++c) bq += C[P - 1][c] * d[q][KDS_ND(o, c)];
        beta[o][q] = bq;
        x = gg * x + bq;
        to = d[q][KDS_ND(o, P - 1)];
      } else {
        beta[o][q] = T(0);
      }
    }
    mB[o] = x;
  }
  // segmented inclusive scan over the lanes of each subdomain
  {
    T gw = powi(gg, ln.Q);
    if (ln.dpp_ok) {
#define KDS_SCAN_STEP(OFF)                                   \
  if ((OFF) < ln.Ls) {                                       \
    _Pragma("unroll") for (int o = 0; o < PER; ++o) {        \
      const T pB = dpp_row_shr<T, (OFF)>(mB[o]);             \
      if (ln.sl >= (OFF)) mB[o] = gw * pB + mB[o];           \
    }                                                        \
    gw = gw * gw;                                            \
  }
      KDS_SCAN_STEP(1)
      KDS_SCAN_STEP(2)
      KDS_SCAN_STEP(4)
      KDS_SCAN_STEP(8)
#undef KDS_SCAN_STEP
    } else {
      for (int off = 1; off < ln.Ls; off <<= 1) {
#pragma unroll
        for (int o = 0; o < PER; ++o) {
          const T pB = __shfl_up(mB[o], off, 64);
          if (ln.sl >= off) mB[o] = gw * pB + mB[o];
        }
        gw = gw * gw;
      }
    }
  }
  // subdomain iteration on the outflows (meaningful on subdomain-end lanes):
  // T_s^p = P_s + G T_{s-1}^{p-1}, inflow of iterate K = T_{s-1}^{K-1}.
  // K = 0: the converged limit, T_s = sum_q G^q P_{s-q} / (1 - G^nseg)
  // (the fully implicit periodic line solve).  On a Dirichlet axis the first
  // subdomain's inflow is the boundary value b at every iterate, and the
  // limit is T_{s-1} = sum_{q<s} G^q P_{s-1-q} + G^s b.
  T t_in[PER];
  if (K > 0) {
    T Tv[PER];
#pragma unroll
    for (int o = 0; o < PER; ++o) Tv[o] = last_old[o];
    for (int it = 1; it < K; ++it) {
#pragma unroll
      for (int o = 0; o < PER; ++o) {
        T up = __shfl(Tv[o], ln.end_up, 64);
        if (dir && ln.s_me == 0) up = bnew[o];
        Tv[o] = mB[o] + G * up;
      }
    }
#pragma unroll
    for (int o = 0; o < PER; ++o) {
      t_in[o] = __shfl(Tv[o], ln.end_up, 64);
      if (dir && ln.s_me == 0) t_in[o] = bnew[o];
    }
  } else {
#pragma unroll
    for (int o = 0; o < PER; ++o) t_in[o] = T(0);
    T Gq = T(1);
    for (int q = 0; q < ln.nseg; ++q) {
      const int s_src = ((ln.s_me - 1 - q) % ln.nseg + ln.nseg) % ln.nseg;
      const int src = ln.lbase + (s_src + 1) * ln.Ls - 1;
#pragma unroll
      for (int o = 0; o < PER; ++o) {
        const T v = __shfl(mB[o], src, 64);
        if (!dir || q < ln.s_me) t_in[o] += Gq * v;
      }
      Gq *= G;
    }
    if (dir) {
      const T Gs = powi(G, ln.s_me);
#pragma unroll
      for (int o = 0; o < PER; ++o) t_in[o] += Gs * bnew[o];
    } else {
      const T inv = T(1) / (T(1) - Gq);
#pragma unroll
      for (int o = 0; o < PER; ++o) t_in[o] *= inv;
    }
  }
  const T g0 = powi(gg, ln.sl * ln.Q);
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T x = ln.dpp_ok ? dpp_row_shr<T, 1>(mB[o]) : __shfl_up(mB[o], 1, 64);
    if (ln.sl == 0) x = T(0);
    T gp = g0, to = t_old0[o];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (q < ln.Q) {
        const T tn = x + gp * t_in[o];
        const T to_next = d[q][KDS_ND(o, P - 1)];
        T fn[P];
#pragma unroll
        for (int b = 0; b < P; ++b) {
          T acc = e1[b] * to + eth[b] * tn;
#pragma unroll
          for (int c = 0; c < P; ++c) acc += C[b][c] * d[q][KDS_ND(o, c)];
          fn[b] = acc;
        }
#pragma unroll
        for (int b = 0; b < P; ++b) d[q][KDS_ND(o, b)] = fn[b];
        x = beta[o][q] + gg * x;
        to = to_next;
        gp *= gg;
      }
    }
  }
#undef KDS_ND
}

template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, int O0 = 0>
__device__ __forceinline__ void line_lanes(T (&d)[QMAX][NN], const LineLane& ln,
                                           const T (&C)[P][P], const T (&e1)[P], const T (&eth)[P],
                                           T gg, T G, int K, const T* bo, const T* bn) {
  constexpr int ALL = ColShape<P, DIM>::PER;
  constexpr int GS = ALL <= 4 ? ALL : (ALL % 3 == 0 ? 3 : 4);
  if constexpr (O0 < ALL) {
    constexpr int n = ALL - O0 < GS ? ALL - O0 : GS;
    line_group<T, P, DIM, AXIS, SIGN, QMAX, NN, O0, n>(d, ln, C, e1, eth, gg, G, K, bo, bn);
    line_lanes<T, P, DIM, AXIS, SIGN, QMAX, NN, O0 + n>(d, ln, C, e1, eth, gg, G, K, bo, bn);
  }
}

// Workgroups are dealt round-robin to the XCDs; give each XCD a contiguous
// range of the nb work items so that neighbouring bundles, which share cache
// lines at their edges, meet in the same L2.
__device__ __forceinline__ int64_t xcd_order(int64_t nb) {
  const int64_t xq = nb / kXcds, xr = nb % kXcds;
  const int64_t xcd = blockIdx.x % kXcds;
  return xcd * xq + min<int64_t>(xcd, xr) + blockIdx.x / kXcds;
}

// One bundle `bid` (numbered over all (velocity, component) pairs) of one
// problem; the body of the single-problem and the batched line kernels.
template <typename T, int P, int DIM>
__device__ __forceinline__ void line_bundle(T* __restrict__ f, const Geom& g,
                                            const SweepTab<T>& tab, const LinePlan& pl,
                                            const BndRef<T>& bd, int64_t bid, T* tile) {
  constexpr int NN = ColShape<P, DIM>::NN;
  constexpr int QMAX = line_qmax((int)sizeof(T), NN);
  int kc = 0;
  while (bid >= pl.block_start[kc + 1]) ++kc;
  const int64_t bundle = bid - pl.block_start[kc];
  const int k = kc / g.m;
  const int a = tab.axis[k];
  const int sg = tab.sign[k];
  const int Na = g.N[a];
  const int S = g.S[a];
  const int nseg = Na / S;
  const int Q = pl.Q[k];
  const int LPL2 = pl.lpl2[k];
  const int NL = Na / Q;
  const int bw = pl.bw[k];
  const int CS = Na * NN;  // LDS column stride
  const int64_t kc_base = (int64_t)kc * g.ncell * NN;

  // ------------------------------------------------------------ bundle
  int ncols;
  if (a == 0) {
    const int64_t nrows = g.ncell / Na;
    const int64_t col0 = bundle * bw;
    ncols = (int)min<int64_t>(bw, nrows - col0);
    // consecutive rows of cells are one contiguous block
    copy_tile<T, true>(f, tile, kc_base + col0 * CS, CS, CS, ncols);
  } else {
    const int nbx = (g.N[0] + bw - 1) / bw;
    const int bx = (int)(bundle % nbx);
    const int64_t other = bundle / nbx;
    const int x0 = bx * bw;
    ncols = min(bw, g.N[0] - x0);
    const int64_t gbase = a == 1 ? kc_base + (other * g.N[1] * g.N[0] + x0) * (int64_t)NN
                                 : kc_base + (other * g.N[0] + x0) * (int64_t)NN;
    const int64_t rowstride = a == 1 ? (int64_t)g.N[0] * NN : (int64_t)g.N[0] * g.N[1] * NN;
    copy_cols<T, NN, true>(f, tile, gbase, rowstride, ncols, Na, CS);
  }
  __syncthreads();

  // ----------------------------------------------------------- compute
  T C[P][P], e1[P], eth[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    e1[r] = tab.e1[k][r];
    eth[r] = tab.eth[k][r];
#pragma unroll
    for (int c = 0; c < P; ++c) C[r][c] = tab.C[k][r * P + c];
  }
  const T gg = eth[P - 1];
  const T G = powi(gg, S);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int LW = 64 / LPL2;
  const int lil = lane % LPL2;
  const int slot = lane / LPL2;
  const int lbase = slot * LPL2;
  LineLane ln;
  ln.Q = Q;
  ln.Ls = S / Q;
  ln.sl = lil % ln.Ls;
  ln.nseg = nseg;
  ln.lbase = lbase;
  ln.s_me = lil / ln.Ls;
  {
    const int s_up = ln.s_me == 0 ? nseg - 1 : ln.s_me - 1;
    ln.end_up = lbase + (s_up + 1) * ln.Ls - 1;
  }
  ln.src_prev = lbase + (lil == 0 ? NL - 1 : lil - 1);
  ln.dpp_ok = ln.Ls <= 16 && (16 % ln.Ls) == 0;
  ln.first = lil == 0;
  const int j0 = lil * Q;
  // Dirichlet axis: boundary values of this (k, c) on the inflow face
  constexpr int PER = ColShape<P, DIM>::PER;
  const int bside = sg > 0 ? 0 : 1;
  const int64_t boff = (bd.old != nullptr && bd.off[a][bside] >= 0)
                           ? (int64_t)kc * bd.nb + bd.off[a][bside] : -1;

  for (int cb = wave * LW; cb < ncols; cb += nwaves * LW) {
    const int c = cb + slot;
    const bool act = (c < ncols) && (lil < NL);
    const T* bo = nullptr;
    const T* bn = nullptr;
    if (boff >= 0 && act) {
      // the column's cell index on the face (cells over the other axes, lower fastest)
      int64_t fcell;
      if (a == 0) {
        fcell = bundle * bw + c;
      } else {
        const int nbx = (g.N[0] + bw - 1) / bw;
        fcell = (bundle % nbx) * bw + c + (int64_t)g.N[0] * (bundle / nbx);
      }
      bo = bd.old + boff + fcell * PER;
      bn = bd.neu + boff + fcell * PER;
    }
    // my cells in downwind order: physical cells j0.. (SIGN > 0) or
    // Na-1-j0 downwards (SIGN < 0)
    const int cbase = (act ? c : 0) * CS;
    // (lanes without a line and cells past Q re-read cell 0 of the column;
    // those values are never used)
    T d[QMAX][NN];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int row = (act && q < Q) ? (sg > 0 ? j0 + q : Na - 1 - j0 - q) : 0;
#pragma unroll
      for (int n = 0; n < NN; ++n) d[q][n] = tile[cbase + row * NN + n];
    }
    switch (a * 2 + (sg > 0 ? 1 : 0)) {
      case 0: line_lanes<T, P, DIM, 0, -1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
      case 1: line_lanes<T, P, DIM, 0, 1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
      case 2: if constexpr (DIM > 1) line_lanes<T, P, DIM, 1, -1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
      case 3: if constexpr (DIM > 1) line_lanes<T, P, DIM, 1, 1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
      case 4: if constexpr (DIM > 2) line_lanes<T, P, DIM, 2, -1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
      default: if constexpr (DIM > 2) line_lanes<T, P, DIM, 2, 1, QMAX, NN>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
    }
    if (act) {
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        if (q < Q) {
          const int row = sg > 0 ? j0 + q : Na - 1 - j0 - q;
#pragma unroll
          for (int n = 0; n < NN; ++n) tile[cbase + row * NN + n] = d[q][n];
        }
      }
    }
  }
  __syncthreads();

  // -------------------------------------------------------- write back
  if (a == 0) {
    const int64_t col0 = bundle * bw;
    copy_tile<T, false>(f, tile, kc_base + col0 * CS, CS, CS, ncols);
  } else {
    const int nbx = (g.N[0] + bw - 1) / bw;
    const int bx = (int)(bundle % nbx);
    const int64_t other = bundle / nbx;
    const int x0 = bx * bw;
    const int64_t gbase = a == 1 ? kc_base + (other * g.N[1] * g.N[0] + x0) * (int64_t)NN
                                 : kc_base + (other * g.N[0] + x0) * (int64_t)NN;
    const int64_t rowstride = a == 1 ? (int64_t)g.N[0] * NN : (int64_t)g.N[0] * g.N[1] * NN;
    copy_cols<T, NN, false>(f, tile, gbase, rowstride, ncols, Na, CS);
  }
}

template <typename T, int P, int DIM>
__global__ __launch_bounds__(256) void k_sweep_line(T* __restrict__ f, Geom g, SweepTab<T> tab,
                                                    LinePlan pl, BndRef<T> bd) {
  extern __shared__ unsigned char smem_raw[];
  line_bundle<T, P, DIM>(f, g, tab, pl, bd, xcd_order(pl.block_start[g.nv * g.m]),
                         reinterpret_cast<T*>(smem_raw));
}

// Many problems of one (precision, degree, dimension) in one launch: the
// bundles of all problems are numbered consecutively (start[] prefix).
template <typename T, int P, int DIM>
__global__ __launch_bounds__(256) void k_sweep_line_batch(const LineTask<T>* __restrict__ tasks,
                                                          const int64_t* __restrict__ start,
                                                          int ntask) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t gbid = xcd_order(start[ntask]);
  int pid = 0;
  while (gbid >= start[pid + 1]) ++pid;
  const LineTask<T>& t = tasks[pid];
  line_bundle<T, P, DIM>(t.f, t.g, t.tab, t.pl, t.bd, gbid - start[pid],
                         reinterpret_cast<T*>(smem_raw));
}

// ====================================================== front sweep

// Velocities with several nonzero components (the paper's D3Q4 set): the
// cell operator [C | E_x | E_y | E_z] is dense (nn x (nn + 3 nf)), and the
// cells of a subdomain are visited by levels (anti-diagonal fronts) of the
// V-oriented cell graph, l = sum over active axes of the downwind cell index:
// the topological order of Sec. 3.2 on a box.  All cells of a level, for all
// components, are independent, so their solves form one GEMM
//     Y[nn x cols] = W[nn x Kd] X[Kd x cols],
// X = [f^{n-1}(cell); theta t^n + (1-theta) t^{n-1} on the three inflow faces].
// t^n comes from the current iterate inside the subdomain (previous level)
// and from iterate p-1 across subdomain faces (eq:ibvp, Jacobi).  One
// workgroup per (velocity, subdomain); one launch per subdomain iteration.
//
// Products: FP64/FP32 FMA (kFrontFma), FP32 matrix cores
// (v_mfma_f32_16x16x4f32), or the split three-product forms on FP16/BF16
// matrix cores (x = hi + lo, W X ~ Wh Xh + Wh Xl + Wl Xh, FP32 accumulation;
// the FP16 low parts are scaled by 2^11 against underflow).

constexpr int kFrontMaxChunk = 64;  // GEMM columns per pass (col_chunk)

typedef float kds_f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 kds_f16x4 __attribute__((ext_vector_type(4)));
typedef short kds_i16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const unsigned int b = __float_as_uint(x);
  return (unsigned short)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_sweep_front(const T* __restrict__ f_old,
                                                     const T* __restrict__ f_prev,
                                                     T* __restrict__ f_cur, Geom g, FrontParams fp,
                                                     const T* __restrict__ Wop,
                                                     const int* __restrict__ lvl_start,
                                                     const int* __restrict__ lvl_cells,
                                                     BndRef<T> bd) {
  extern __shared__ unsigned char smem_raw[];
  const int nn = g.nn, nf = fp.nf, Kd = fp.Kd, P = g.P, m = g.m;
  const int Mpad = (nn + 15) & ~15;
  const int Kpad = (Kd + 15) & ~15;
  const int CH = fp.col_chunk;
  const int XS = CH + 1;  // odd row stride: conflict-free gathers
  T* Wt = reinterpret_cast<T*>(smem_raw);            // [Mpad][Kpad] (matrix-core modes)
  T* X = Wt + (MODE == kFrontFma ? 0 : Mpad * Kpad);  // [Kpad][XS]
  __shared__ int64_t col_base[kFrontMaxChunk];         // per column: state offset of the cell
  __shared__ int64_t col_nb[3][kFrontMaxChunk];        // ... of the upwind neighbour per face
  __shared__ unsigned char col_int[3][kFrontMaxChunk]; // 1: neighbour inside the subdomain,
                                                       // 2: face of the box on a Dirichlet axis
  __shared__ int face_node[3 * kMaxP * kMaxP * kMaxP]; // neighbour node of face row q
  const int nsd = fp.nsub[0] * fp.nsub[1] * fp.nsub[2];
  const int k = blockIdx.x / nsd;
  const int sd = blockIdx.x - k * nsd;
  int sdc[3] = {sd % fp.nsub[0], (sd / fp.nsub[0]) % fp.nsub[1], sd / (fp.nsub[0] * fp.nsub[1])};
  const int tid = threadIdx.x, bs = blockDim.x;
  const T th = (T)fp.theta;
  const T* Wk = Wop + (int64_t)k * nn * Kd;
  if (MODE != kFrontFma) {
    for (int e = tid; e < Mpad * Kpad; e += bs) {
      const int i = e / Kpad, r = e - i * Kpad;
      Wt[e] = (i < nn && r < Kd) ? Wk[i * Kd + r] : T(0);
    }
  }
  int sgn[3], outn[3];
  for (int a = 0; a < 3; ++a) {
    sgn[a] = a < g.dim ? fp.sg[k][a] : 0;
    outn[a] = sgn[a] > 0 ? P - 1 : 0;  // neighbour's node index on the shared face
  }
  const int pw[3] = {1, P, P * P};
  const int64_t plane = g.ncell * nn;
  const int nlev = fp.nlev[k];
  // node of the upwind neighbour matching face row (a, q): index outn[a] on
  // axis a, the other indices from q (x fastest)
  for (int t = tid; t < 3 * nf; t += bs) {
    const int a = t / nf, q = t - a * nf;
    int node = 0, rem = q;
    for (int o = 0; o < g.dim; ++o) {
      int io;
      if (o == a) io = outn[a];
      else { io = rem % P; rem /= P; }
      node += io * pw[o];
    }
    face_node[t] = a < g.dim ? node : 0;
  }
  __syncthreads();

  for (int lev = 0; lev < nlev; ++lev) {
    const int c0 = lvl_start[fp.lvl_off[k] + lev];
    const int c1 = lvl_start[fp.lvl_off[k] + lev + 1];
    const int ncol = (c1 - c0) * m;
    for (int j0 = 0; j0 < ncol; j0 += CH) {
      const int nc = min(CH, ncol - j0);
      // ---- column descriptors: state offset of the column's cell, and of the
      // upwind neighbour across each inflow face (flagged internal / interface)
      if (tid < nc) {
        const int j = j0 + tid;
        const int ci = c0 + j / m, c = j - (j / m) * m;
        const int pk = lvl_cells[ci];
        const int lc[3] = {pk & 1023, (pk >> 10) & 1023, (pk >> 20) & 1023};
        int gc[3];
        for (int a = 0; a < 3; ++a) {
          const int pl = sgn[a] < 0 ? g.S[a] - 1 - lc[a] : lc[a];
          gc[a] = sdc[a] * g.S[a] + pl;
        }
        const int64_t kc = (int64_t)(k * m + c) * plane;
        col_base[tid] = kc + (gc[0] + (int64_t)g.N[0] * (gc[1] + (int64_t)g.N[1] * gc[2])) * nn;
        for (int a = 0; a < 3; ++a) {
          int64_t nbo = -1;
          if (a < g.dim && sgn[a] != 0) {
            int nb[3] = {gc[0], gc[1], gc[2]};
            nb[a] -= sgn[a];
            const bool outside = nb[a] < 0 || nb[a] >= g.N[a];
            const int bside = sgn[a] > 0 ? 0 : 1;
            if (outside && bd.old != nullptr && bd.off[a][bside] >= 0) {
              // boundary values of the face cell (cells over the other axes)
              int64_t fcell = 0, mul = 1;
              for (int o = 0; o < g.dim; ++o)
                if (o != a) {
                  fcell += gc[o] * mul;
                  mul *= g.N[o];
                }
              nbo = (int64_t)(k * m + c) * bd.nb + bd.off[a][bside] + fcell * nf;
              col_int[a][tid] = 2;
            } else {
              if (nb[a] < 0) nb[a] += g.N[a];
              if (nb[a] >= g.N[a]) nb[a] -= g.N[a];
              nbo = kc + (nb[0] + (int64_t)g.N[0] * (nb[1] + (int64_t)g.N[1] * nb[2])) * nn;
              col_int[a][tid] = lc[a] > 0 ? 1 : 0;
            }
          }
          col_nb[a][tid] = nbo;
        }
      }
      __syncthreads();
      // ---- gather X[r][jj] (r fastest over threads: contiguous nodes); U
      // independent loads per thread are issued before any is used
      {
        constexpr int U = 4;
        const int total = Kpad * CH;
        for (int e0 = tid; e0 < total; e0 += U * bs) {
          T vo[U], vn[U];
          int rr[U], jq[U];
          int face[U];
          bool isb[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bs;
            const int jj = e / Kpad, r = e - jj * Kpad;
            rr[u] = r;
            jq[u] = jj;
            int64_t at = 0;
            int fa = -1;
            bool live = e < total && jj < nc && r < Kd;
            if (live) {
              if (r < nn) {
                at = col_base[jj] + r;
              } else {
                const int a = (r - nn) / nf;
                if (col_nb[a][jj] >= 0) {
                  fa = a;
                  // boundary values are numbered by face node (row q of face a)
                  at = col_nb[a][jj] +
                       (col_int[a][jj] == 2 ? (r - nn - a * nf) : face_node[r - nn]);
                } else {
                  live = false;
                }
              }
            }
            face[u] = live ? fa : -2;
            isb[u] = live && fa >= 0 && col_int[fa][jj] == 2;
            // inactive slots re-read element 0 of the state (never used)
            vo[u] = isb[u] ? bd.old[at] : f_old[live ? at : 0];
            vn[u] = isb[u] ? bd.neu[at]
                           : ((fa >= 0 && col_int[fa][jj]) ? f_cur[at] : f_prev[fa >= 0 ? at : 0]);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bs;
            if (e < total) {
              T v = T(0);
              if (face[u] == -1) v = vo[u];
              else if (face[u] >= 0) v = th * vn[u] + (T(1) - th) * vo[u];
              X[rr[u] * XS + jq[u]] = v;
            }
          }
        }
      }
      __syncthreads();
      // ---- Y = W X, written to the current iterate
      auto store = [&](int i, int jj, T y) { f_cur[col_base[jj] + i] = y; };
      if constexpr (MODE == kFrontFma) {
        for (int e = tid; e < nn * nc; e += bs) {
          const int jj = e / nn, i = e - jj * nn;
          T acc = T(0);
          for (int r = 0; r < Kd; ++r) acc += Wk[i * Kd + r] * X[r * XS + jj];
          store(i, jj, acc);
        }
      } else {
        const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
        const int li = lane & 15, lk = lane >> 4;
        const int mt_n = Mpad / 16, nt_n = (nc + 15) / 16;
        for (int t = wave; t < mt_n * nt_n; t += nw) {
          const int mt = t % mt_n, nt = t / mt_n;
          const int i0 = mt * 16, jb = nt * 16;
          kds_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          if constexpr (MODE == kFrontMfma) {
            for (int kk = 0; kk < Kpad; kk += 4) {
              const float av = (float)Wt[(i0 + li) * Kpad + kk + lk];
              const float bv = (float)X[(kk + lk) * XS + jb + li];
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
          } else {
            kds_f32x4 cor = {0.f, 0.f, 0.f, 0.f};
            for (int kk = 0; kk < Kpad; kk += 16) {
              float aw[4], bw[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                aw[u] = (float)Wt[(i0 + li) * Kpad + kk + 4 * lk + u];
                bw[u] = (float)X[(kk + 4 * lk + u) * XS + jb + li];
              }
              if constexpr (MODE == kFrontSplitF16) {
                kds_f16x4 ah, al, bh, bl;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const _Float16 ha = (_Float16)aw[u], hb = (_Float16)bw[u];
                  ah[u] = ha;
                  bh[u] = hb;
                  al[u] = (_Float16)((aw[u] - (float)ha) * 2048.0f);
                  bl[u] = (_Float16)((bw[u] - (float)hb) * 2048.0f);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, acc, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, cor, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, cor, 0, 0, 0);
              } else {
                kds_i16x4 ah, al, bh, bl;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const unsigned short ha = bf16_rne(aw[u]), hb = bf16_rne(bw[u]);
                  ah[u] = (short)ha;
                  bh[u] = (short)hb;
                  al[u] = (short)bf16_rne(aw[u] - bf16_to_f32(ha));
                  bl[u] = (short)bf16_rne(bw[u] - bf16_to_f32(hb));
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, cor, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, cor, 0, 0, 0);
              }
            }
            const float sc = MODE == kFrontSplitF16 ? 1.0f / 2048.0f : 1.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += sc * cor[v];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = i0 + 4 * lk + v, jj = jb + li;
            if (i < nn && jj < nc) store(i, jj, (T)acc[v]);
          }
        }
      }
      __syncthreads();
    }
  }
}

// ============================================================ launchers

namespace {

inline unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

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
  static hipError_t relax(const Geom& g, const void* eq, const void* fin, void* fout, hipStream_t s) {
    const int64_t plane = g.ncell * g.nn;
    hipLaunchKernelGGL((k_relax<T, LAW, D, M, NV>), dim3(blocks_for(plane)), dim3(256), 0, s,
                       (const T*)fin, (T*)fout, plane, *(const Tab*)eq);
    return hipGetLastError();
  }
};

struct ComboEntry {
  int law, dim, m, nv;
  bool (*build)(const std::vector<double>&, const std::vector<double>&, const std::vector<double>&,
                double, const std::vector<double>&, std::vector<unsigned char>&);
  hipError_t (*init64)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*init32)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*relax64)(const Geom&, const void*, const void*, void*, hipStream_t);
  hipError_t (*relax32)(const Geom&, const void*, const void*, void*, hipStream_t);
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

template <typename T>
hipError_t sweep_line_t(const Geom& g, const void* tab, const LinePlan& plan, void* f,
                        const BndArgs& bnd, hipStream_t s) {
  const BndRef<T> bd = bnd_ref<T>(bnd);
  const SweepTab<T>& t = *(const SweepTab<T>*)tab;
  const int64_t nblocks = plan.block_start[g.nv * g.m];
  const size_t lds = (size_t)plan.lds_elems * sizeof(T);
  const int key = g.P * 10 + g.dim;
  switch (key) {
#define KDS_LINE(PP, DD)                                                                        \
  case PP * 10 + DD:                                                                            \
    hipLaunchKernelGGL((k_sweep_line<T, PP, DD>), dim3((unsigned)nblocks), dim3(plan.threads),  \
                       lds, s, (T*)f, g, t, plan, bd);                                          \
    break;
    KDS_LINE(1, 1) KDS_LINE(2, 1) KDS_LINE(3, 1) KDS_LINE(4, 1)
    KDS_LINE(1, 2) KDS_LINE(2, 2) KDS_LINE(3, 2) KDS_LINE(4, 2)
    KDS_LINE(1, 3) KDS_LINE(2, 3) KDS_LINE(3, 3) KDS_LINE(4, 3)
#undef KDS_LINE
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
                        void* fout, hipStream_t s) {
  const ComboEntry* c = combo_of(law, g);
  if (!c) return hipErrorInvalidValue;
  return prec == KDS_FP64 ? c->relax64(g, eq, fin, fout, s) : c->relax32(g, eq, fin, fout, s);
}

hipError_t launch_moments(int prec, const Geom& g, const void* f, double* W, hipStream_t s) {
  const int64_t plane = g.ncell * g.nn;
  if (prec == KDS_FP64)
    hipLaunchKernelGGL(k_moments<double>, dim3(blocks_for(plane)), dim3(256), 0, s,
                       (const double*)f, W, plane, g.m, g.nv);
  else
    hipLaunchKernelGGL(k_moments<float>, dim3(blocks_for(plane)), dim3(256), 0, s,
                       (const float*)f, W, plane, g.m, g.nv);
  return hipGetLastError();
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

hipError_t launch_sweep_plain(int prec, const Geom& g, const void* tab, const void* f_old,
                              void* f_new, const void* tr_prev, void* tr_out, const BndArgs& bnd,
                              hipStream_t s) {
  return prec == KDS_FP64 ? sweep_plain_t<double>(g, tab, f_old, f_new, tr_prev, tr_out, bnd, s)
                          : sweep_plain_t<float>(g, tab, f_old, f_new, tr_prev, tr_out, bnd, s);
}

hipError_t launch_sweep_line(int prec, const Geom& g, const void* tab, const LinePlan& plan,
                             void* f, const BndArgs& bnd, hipStream_t s) {
  return prec == KDS_FP64 ? sweep_line_t<double>(g, tab, plan, f, bnd, s)
                          : sweep_line_t<float>(g, tab, plan, f, bnd, s);
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


size_t front_lds_bytes(int prec, int mode, const Geom& g, const FrontParams& fp) {
  const int Mpad = (g.nn + 15) & ~15, Kpad = (fp.Kd + 15) & ~15;
  const size_t el = prec == KDS_FP64 ? 8 : 4;
  return ((mode == kFrontFma ? 0 : (size_t)Mpad * Kpad) + (size_t)Kpad * (fp.col_chunk + 1)) * el;
}

hipError_t launch_sweep_front(int prec, int mode, const Geom& g, const FrontParams& fp,
                              const void* Wop, const int* lvl_start, const int* lvl_cells,
                              const void* f_old, const void* f_prev, void* f_cur,
                              const BndArgs& bnd, hipStream_t s) {
  const int nsd = fp.nsub[0] * fp.nsub[1] * fp.nsub[2];
  const dim3 grid((unsigned)(nsd * g.nv)), block(256);
  const size_t lds = front_lds_bytes(prec, mode, g, fp);
  if (prec == KDS_FP64) {
    if (mode != kFrontFma) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep_front<double, kFrontFma>), grid, block, lds, s, (const double*)f_old,
                       (const double*)f_prev, (double*)f_cur, g, fp, (const double*)Wop, lvl_start,
                       lvl_cells, bnd_ref<double>(bnd));
  } else {
    switch (mode) {
#define KDS_FRONT(MODE)                                                                         \
  case MODE:                                                                                    \
    hipLaunchKernelGGL((k_sweep_front<float, MODE>), grid, block, lds, s, (const float*)f_old,  \
                       (const float*)f_prev, (float*)f_cur, g, fp, (const float*)Wop, lvl_start, \
                       lvl_cells, bnd_ref<float>(bnd));                                         \
    break;
      KDS_FRONT(kFrontFma)
      KDS_FRONT(kFrontMfma)
      KDS_FRONT(kFrontSplitF16)
      KDS_FRONT(kFrontSplitBf16)
#undef KDS_FRONT
      default:
        return hipErrorInvalidValue;
    }
  }
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
  return prec == KDS_FP64 ? sizeof(LineTask<double>) : sizeof(LineTask<float>);
}

void pack_line_task(int prec, void* f, const Geom& g, const void* tab, const LinePlan& pl,
                    const BndArgs& bnd, void* out) {
  if (prec == KDS_FP64) {
    LineTask<double> t;
    t.f = (double*)f;
    t.g = g;
    std::memcpy(&t.tab, tab, sizeof(t.tab));
    t.pl = pl;
    t.bd = bnd_ref<double>(bnd);
    std::memcpy(out, &t, sizeof(t));
  } else {
    LineTask<float> t;
    t.f = (float*)f;
    t.g = g;
    std::memcpy(&t.tab, tab, sizeof(t.tab));
    t.pl = pl;
    t.bd = bnd_ref<float>(bnd);
    std::memcpy(out, &t, sizeof(t));
  }
}

hipError_t launch_sweep_line_batch(int prec, int P, int dim, const void* tasks, const int64_t* start,
                                   int ntask, int64_t nblocks, int threads, size_t lds_elems,
                                   hipStream_t s) {
  const size_t lds = lds_elems * (prec == KDS_FP64 ? 8 : 4);
  const int key = P * 10 + dim;
  if (prec == KDS_FP64) {
    switch (key) {
#define KDS_LB(PP, DD)                                                                            \
  case PP * 10 + DD:                                                                              \
    hipLaunchKernelGGL((k_sweep_line_batch<double, PP, DD>), dim3((unsigned)nblocks), dim3(threads), \
                       lds, s, (const LineTask<double>*)tasks, start, ntask);                    \
    break;
      KDS_LB(1, 1) KDS_LB(2, 1) KDS_LB(3, 1) KDS_LB(4, 1)
      KDS_LB(1, 2) KDS_LB(2, 2) KDS_LB(3, 2) KDS_LB(4, 2)
      KDS_LB(1, 3) KDS_LB(2, 3) KDS_LB(3, 3) KDS_LB(4, 3)
#undef KDS_LB
      default:
        return hipErrorInvalidValue;
    }
  } else {
    switch (key) {
#define KDS_LB(PP, DD)                                                                            \
  case PP * 10 + DD:                                                                              \
    hipLaunchKernelGGL((k_sweep_line_batch<float, PP, DD>), dim3((unsigned)nblocks), dim3(threads), \
                       lds, s, (const LineTask<float>*)tasks, start, ntask);                     \
    break;
      KDS_LB(1, 1) KDS_LB(2, 1) KDS_LB(3, 1) KDS_LB(4, 1)
      KDS_LB(1, 2) KDS_LB(2, 2) KDS_LB(3, 2) KDS_LB(4, 2)
      KDS_LB(1, 3) KDS_LB(2, 3) KDS_LB(3, 3) KDS_LB(4, 3)
#undef KDS_LB
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}


// Allow the line kernels (single and batched) dynamic LDS up to `bytes`
// (workgroups above 64 KiB need the attribute).  Once per size and process.
hipError_t line_kernels_allow_lds(size_t bytes) {
  static size_t done = 0;
  if (bytes <= 64 * 1024 || bytes <= done) return hipSuccess;
  hipError_t e = hipSuccess;
  auto set = [&](const void* k) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  };
#define KDS_ALLOW(PP, DD)                                                \
  set(reinterpret_cast<const void*>(&k_sweep_line<float, PP, DD>));        \
  set(reinterpret_cast<const void*>(&k_sweep_line<double, PP, DD>));       \
  set(reinterpret_cast<const void*>(&k_sweep_line_batch<float, PP, DD>));  \
  set(reinterpret_cast<const void*>(&k_sweep_line_batch<double, PP, DD>));
  KDS_ALLOW(1, 1) KDS_ALLOW(2, 1) KDS_ALLOW(3, 1) KDS_ALLOW(4, 1)
  KDS_ALLOW(1, 2) KDS_ALLOW(2, 2) KDS_ALLOW(3, 2) KDS_ALLOW(4, 2)
  KDS_ALLOW(1, 3) KDS_ALLOW(2, 3) KDS_ALLOW(3, 3) KDS_ALLOW(4, 3)
#undef KDS_ALLOW
  if (e == hipSuccess) done = bytes;
  return e;
}

}  // namespace kds
