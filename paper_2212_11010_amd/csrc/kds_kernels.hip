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
__global__ __launch_bounds__(256) void k_relax(const T* fin, T* fout, int64_t plane,
                                               EqTab<D, M, NV> t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= plane) return;
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
  equilibrium<LAW, D, M, NV>(t, w, Mk);
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int r = 0; r < M; ++r)
      fout[(int64_t)(k * M + r) * plane + i] = (T)(fv[k][r] + t.omega * (Mk[k][r] - fv[k][r]));
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
                                                     SweepTab<T> tab) {
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
  {
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
  constexpr int U = 8;
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
      VT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ta[u] < total) v[u] = g[ga[u]];
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

// All K subdomain iterations of whole grid lines in one pass.  One workgroup
// holds a bundle of complete lines of one (velocity, component) in LDS; one
// wavefront (or half / quarter of one) owns a line, Q consecutive cells per
// lane.  On a line the outflow values obey the first-order recurrence
//     t_{j+1} = beta_j + g t_j,  beta_j = (C f_j^{n-1})[P-1] + e1[P-1] t_j^{n-1},
//     g = eth[P-1],
// reset at every subdomain start.  A segmented scan over the lanes
// (wavefront shuffles) gives, for every cell, q_j = the inflow it would get
// with zero inflow at its subdomain start, and per subdomain s the outflow
// P_s with zero inflow.  With G = g^S, the outflow of subdomain s at iterate p
// is T_s^p = P_s + G T_{s-1}^{p-1}, T^0 = outflow of f^{n-1}, and the final
// iterate K has inflow t_in(s) = T_{s-1}^{K-1}, so t_j^n = q_j + g^{j-j_s} t_in(s).
// This is the same linear algebra as K literal sweeps (exact reformulation,
// different rounding order); the state is read and written once.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_sweep_line(T* __restrict__ f, Geom g, SweepTab<T> tab,
                                                    LinePlan pl) {
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);

  const int64_t bid = blockIdx.x;
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
  const int nn = g.nn;
  const int per = nn / P;

  const int64_t kc_base = (int64_t)kc * g.ncell * nn;
  int64_t rowbase, rowstride;
  int R, n_lines;
  if (a == 0) {
    rowbase = kc_base + bundle * (int64_t)Na * nn;
    rowstride = nn;
    R = nn;
    n_lines = per;
  } else {
    const int B = pl.bw[k];
    const int nbx = (g.N[0] + B - 1) / B;
    const int bx = (int)(bundle % nbx);
    const int64_t other = bundle / nbx;
    const int x0 = bx * B;
    const int Bw = min(B, g.N[0] - x0);
    if (a == 1) {
      rowbase = kc_base + (other * g.N[1] * g.N[0] + x0) * (int64_t)nn;
      rowstride = (int64_t)g.N[0] * nn;
    } else {
      rowbase = kc_base + (other * g.N[0] + x0) * (int64_t)nn;
      rowstride = (int64_t)g.N[0] * g.N[1] * nn;
    }
    R = Bw * nn;
    n_lines = Bw * per;
  }

  copy_tile<T, true>(f, tile, rowbase, rowstride, R, Na);
  __syncthreads();

  int ns = 1;
  for (int ax = 0; ax < a; ++ax) ns *= P;

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
  const int j0 = lil * Q;
  const int Ls = S / Q;          // lanes per subdomain (Q divides S)
  const int sl = lil % Ls;       // lane index inside its subdomain
  const int s_me = lil / Ls;
  const int s_up = s_me == 0 ? nseg - 1 : s_me - 1;
  const int end_up = lbase + (s_up + 1) * Ls - 1;  // lane holding the upwind subdomain's end
  const int src_prev = lbase + (lil == 0 ? NL - 1 : lil - 1);
  const bool dpp_ok = Ls <= 16 && (16 % Ls) == 0;  // subdomains never straddle a 16-lane row
  const T gQ = powi(gg, Q);

  for (int lb = wave * LW; lb < n_lines; lb += nwaves * LW) {
    const int l = lb + slot;
    const bool act = (l < n_lines) && (lil < NL);
    const int xl = act ? l / per : 0;
    const int on = act ? l % per : 0;
    const int loff = xl * nn + other_node_offset(on, a, P, g.dim);

    T fo[kMaxQ][P];
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) {
      const int j = j0 + q;
      const int r = sg > 0 ? j : Na - 1 - j;
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const int pb = sg > 0 ? b : P - 1 - b;
        fo[q][b] = (act && q < Q) ? tile[r * R + loff + pb * ns] : T(0);
      }
    }
    T last_old = T(0);
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q)
      if (q == Q - 1) last_old = fo[q][P - 1];
    // old-time inflow of my first cell: outflow node of the upwind cell
    const T t_old0 = __shfl(last_old, src_prev, 64);

    // zero-inflow recurrence over my cells: x <- beta + g x, x = 0 entering
    // my chunk; mB = value leaving my chunk.
    T beta[kMaxQ];
    T mB = T(0);
    {
      T to = t_old0;
#pragma unroll
      for (int q = 0; q < kMaxQ; ++q) {
        if (q < Q) {
          T bq = e1[P - 1] * to;
#pragma unroll
          for (int c = 0; c < P; ++c) bq += C[P - 1][c] * fo[q][c];
          beta[q] = bq;
          mB = gg * mB + bq;
          to = fo[q][P - 1];
        } else {
          beta[q] = T(0);
        }
      }
    }
    // segmented inclusive scan over the lanes of each subdomain: a window of
    // `off` lanes that does not reach the subdomain start multiplies the
    // incoming value by g^(Q off)
    {
      T gw = gQ;
      if (dpp_ok) {
#define KDS_SCAN_STEP(OFF)                                  \
  if ((OFF) < Ls) {                                         \
    const T pB = dpp_row_shr<T, (OFF)>(mB);                 \
    if (sl >= (OFF)) mB = gw * pB + mB;                     \
    gw = gw * gw;                                           \
  }
        KDS_SCAN_STEP(1)
        KDS_SCAN_STEP(2)
        KDS_SCAN_STEP(4)
        KDS_SCAN_STEP(8)
#undef KDS_SCAN_STEP
      } else {
        for (int off = 1; off < Ls; off <<= 1) {
          const T pB = __shfl_up(mB, off, LPL2);
          if (sl >= off) mB = gw * pB + mB;
          gw = gw * gw;
        }
      }
    }
    T x_in = dpp_ok ? dpp_row_shr<T, 1>(mB) : __shfl_up(mB, 1, LPL2);
    if (sl == 0) x_in = T(0);

    T qv[kMaxQ];
    {
      T x = x_in;
#pragma unroll
      for (int q = 0; q < kMaxQ; ++q) {
        qv[q] = x;
        if (q < Q) x = beta[q] + gg * x;
      }
    }
    // subdomain iteration on the outflow values (meaningful on end lanes,
    // where mB is the zero-inflow outflow P_s of the subdomain)
    const T Pseg = mB;
    T Tv = last_old;
    for (int it = 1; it < g.K; ++it) {
      const T up = __shfl(Tv, end_up, 64);
      Tv = Pseg + G * up;
    }
    const T t_in = __shfl(Tv, end_up, 64);

    if (act) {
      T gp = powi(gg, j0 % S);
      T to = t_old0;
#pragma unroll
      for (int q = 0; q < kMaxQ; ++q) {
        if (q < Q) {
          const T tn = qv[q] + gp * t_in;
          const int j = j0 + q;
          const int r = sg > 0 ? j : Na - 1 - j;
#pragma unroll
          for (int b = 0; b < P; ++b) {
            T s = e1[b] * to + eth[b] * tn;
#pragma unroll
            for (int c = 0; c < P; ++c) s += C[b][c] * fo[q][c];
            const int pb = sg > 0 ? b : P - 1 - b;
            tile[r * R + loff + pb * ns] = s;
          }
          to = fo[q][P - 1];
          gp *= gg;
        }
      }
    }
  }
  __syncthreads();
  copy_tile<T, false>(f, tile, rowbase, rowstride, R, Na);
}

// ============================================================ launchers

namespace {

inline unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

template <int LAW, int D, int M, int NV>
struct EqCombo {
  using Tab = EqTab<D, M, NV>;
  static bool build(const std::vector<double>& lp, const std::vector<double>& a,
                    const std::vector<double>& b, double omega, std::vector<unsigned char>& blob) {
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
                double, std::vector<unsigned char>&);
  hipError_t (*init64)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*init32)(const Geom&, const void*, const double*, void*, hipStream_t);
  hipError_t (*relax64)(const Geom&, const void*, const void*, void*, hipStream_t);
  hipError_t (*relax32)(const Geom&, const void*, const void*, void*, hipStream_t);
};

#define KDS_COMBO(LAW, D, M, NV)                                                          \
  ComboEntry {                                                                            \
    LAW, D, M, NV, &EqCombo<LAW, D, M, NV>::build, &EqCombo<LAW, D, M, NV>::init<double>, \
        &EqCombo<LAW, D, M, NV>::init<float>, &EqCombo<LAW, D, M, NV>::relax<double>,     \
        &EqCombo<LAW, D, M, NV>::relax<float>                                             \
  }

// (law, dim, m, n_vel) combinations with compiled pointwise kernels
const ComboEntry kCombos[] = {
    KDS_COMBO(KDS_LAW_LINEAR, 1, 1, 2), KDS_COMBO(KDS_LAW_LINEAR, 1, 2, 2),
    KDS_COMBO(KDS_LAW_LINEAR, 2, 1, 4), KDS_COMBO(KDS_LAW_LINEAR, 2, 3, 4),
    KDS_COMBO(KDS_LAW_LINEAR, 3, 1, 6), KDS_COMBO(KDS_LAW_LINEAR, 3, 4, 6),
    KDS_COMBO(KDS_LAW_LINEAR, 3, 6, 6), KDS_COMBO(KDS_LAW_EULER, 1, 3, 2),
    KDS_COMBO(KDS_LAW_EULER, 2, 4, 4),  KDS_COMBO(KDS_LAW_EULER, 3, 5, 6),
};

const ComboEntry* find_combo(int law, int dim, int m, int nv) {
  for (const auto& c : kCombos)
    if (c.law == law && c.dim == dim && c.m == m && c.nv == nv) return &c;
  return nullptr;
}

template <typename T>
hipError_t sweep_plain_t(const Geom& g, const void* tab, const void* f_old, void* f_new,
                         const void* tr_prev, void* tr_out, hipStream_t s) {
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
                       (const T*)tr_prev, (T*)tr_out, g, t);                                   \
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
                        hipStream_t s) {
  const SweepTab<T>& t = *(const SweepTab<T>*)tab;
  const int64_t nblocks = plan.block_start[g.nv * g.m];
  const size_t lds = (size_t)plan.lds_elems * sizeof(T);
  switch (g.P) {
#define KDS_LINE(PP)                                                                            \
  case PP:                                                                                      \
    hipLaunchKernelGGL((k_sweep_line<T, PP>), dim3((unsigned)nblocks), dim3(plan.threads), lds, s, \
                       (T*)f, g, t, plan);                                                      \
    break;
    KDS_LINE(1)
    KDS_LINE(2)
    KDS_LINE(3)
    KDS_LINE(4)
#undef KDS_LINE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool build_eq_blob(int law, int dim, int m, int nv, const std::vector<double>& law_params,
                   const std::vector<double>& a, const std::vector<double>& b, double omega,
                   std::vector<unsigned char>& blob) {
  const ComboEntry* c = find_combo(law, dim, m, nv);
  if (!c) return false;
  return c->build(law_params, a, b, omega, blob);
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
                              void* f_new, const void* tr_prev, void* tr_out, hipStream_t s) {
  return prec == KDS_FP64 ? sweep_plain_t<double>(g, tab, f_old, f_new, tr_prev, tr_out, s)
                          : sweep_plain_t<float>(g, tab, f_old, f_new, tr_prev, tr_out, s);
}

hipError_t launch_sweep_line(int prec, const Geom& g, const void* tab, const LinePlan& plan,
                             void* f, hipStream_t s) {
  return prec == KDS_FP64 ? sweep_line_t<double>(g, tab, plan, f, s)
                          : sweep_line_t<float>(g, tab, plan, f, s);
}

}  // namespace kds
