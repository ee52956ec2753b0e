// kds_line.h -- the line schedule (axis-aligned velocities): all subdomain
// iterations of whole grid lines in one pass.  Included by kds_line_f32.hip
// and kds_line_f64.hip, one element type each.
#pragma once

#include "kds_device.h"

namespace kds {

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

// One contiguous block of n vectors: 32-bit offsets from a uniform base (the
// loads and stores take the scalar-base addressing form), U in flight.
template <typename T, int VW, bool LOAD>
__device__ __forceinline__ void copy_block(T* __restrict__ f, T* tile, int64_t base, int n) {
  using VT = typename VecT<T, VW>::type;
  constexpr int U = 16;
  VT* g = reinterpret_cast<VT*>(f + base);
  VT* t = reinterpret_cast<VT*>(tile);
  const int bs = blockDim.x;
  for (int e0 = threadIdx.x; e0 < n; e0 += U * bs) {
    if (LOAD) {
      VT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * bs;
        v[u] = g[e < n ? e : 0];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * bs;
        if (e < n) t[e] = v[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * bs;
        if (e < n) g[e] = t[e];
      }
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
  if (rows == 1) {
    if (VMAX >= 4 && R % 4 == 0 && rowbase % 4 == 0)
      copy_block<T, (VMAX >= 4 ? 4 : 1), LOAD>(f, tile, rowbase, R / 4);
    else if (R % 2 == 0 && rowbase % 2 == 0)
      copy_block<T, 2, LOAD>(f, tile, rowbase, R / 2);
    else
      copy_block<T, 1, LOAD>(f, tile, rowbase, R);
    return;
  }
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

// Widest vector (16 B at most) whose width divides n elements.
template <typename T, int n>
struct LineVec {
  static constexpr int V16 = 16 / (int)sizeof(T);
  static constexpr int VW = n % V16 == 0 ? V16 : (n % 2 == 0 ? 2 : 1);
};

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
// d[q][.]: either all NN nodes of my cells (COMPACT = false, physical node
// offsets) or only the PER lines of this group, [line][physical index along
// the axis] (COMPACT = true, NN = PER * P).
template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, int O0, int PER,
          bool DIR, bool COMPACT = false>
__device__ __forceinline__ void line_group(T (&d)[QMAX][NN], const LineLane& ln,
                                           const T (&C)[P][P], const T (&e1)[P], const T (&eth)[P],
                                           T gg, T G, int K, const T* bo, const T* bn) {
  static_assert(COMPACT ? NN == PER * P : NN == ColShape<P, DIM>::NN, "cell size");
  const int Qn = ln.Q;  // cells per lane
  // Dirichlet axis: bo / bn point at this line's boundary values (inflow of
  // the first subdomain at the old / new time); nullptr on a periodic axis
  // (loaded where used: short live ranges; DIR = false compiles them out)
  const bool dir = DIR && bo != nullptr;
  // physical node of downwind node b along the axis, line O0 + o
#define KDS_ND(o, b)                                                         \
  (COMPACT ? (o) * P + (SIGN > 0 ? (b) : P - 1 - (b))                        \
           : node_of<P, DIM, AXIS>(O0 + (o), SIGN > 0 ? (b) : P - 1 - (b)))
  T last_old[PER], t_old0[PER], mB[PER];
  T beta[PER][QMAX];
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T lo = T(0);
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
      if (q == Qn - 1) lo = d[q][KDS_ND(o, P - 1)];
    last_old[o] = lo;
  }
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    t_old0[o] = __shfl(last_old[o], ln.src_prev, 64);
    if (dir && ln.first) t_old0[o] = bo[O0 + o];
  }
  // zero-inflow recurrence over my cells
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T to = t_old0[o], x = T(0);
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (q < Qn) {
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
    T gw = powi(gg, Qn);
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
  T bnew[PER];
#pragma unroll
  for (int o = 0; o < PER; ++o) bnew[o] = (dir && ln.s_me == 0) ? bn[O0 + o] : T(0);
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
      for (int o = 0; o < PER; ++o) t_in[o] += Gs * bn[O0 + o];
    } else {
      const T inv = T(1) / (T(1) - Gq);
#pragma unroll
      for (int o = 0; o < PER; ++o) t_in[o] *= inv;
    }
  }
  const T g0 = powi(gg, ln.sl * Qn);
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    T x = ln.dpp_ok ? dpp_row_shr<T, 1>(mB[o]) : __shfl_up(mB[o], 1, 64);
    if (ln.sl == 0) x = T(0);
    T gp = g0, to = t_old0[o];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (q < Qn) {
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

// Lines longer than a wavefront holds in registers (64 lanes x QMAX cells):
// the lane owns Q > QMAX consecutive cells and streams them from the LDS tile
// in rounds of QMAX.  The arithmetic is line_group's: pass 1 runs the
// zero-inflow recurrence over all the lane's cells, the lane scan and the
// subdomain iteration are the same, pass 2 recomputes each cell's beta and
// writes the new state into the tile in place (a lane's cells are its own;
// different line groups touch different nodes).  Cell q of the lane, in
// downwind order, is tile row `rowof(q)`; lanes without a line (act = false)
// read row 0 and store nothing.
template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, int O0, int PER,
          bool DIR>
__device__ __forceinline__ void line_group_rounds(T* tile, int cbase, int j0, int Na, bool act,
                                                  const LineLane& ln, const T (&C)[P][P],
                                                  const T (&e1)[P], const T (&eth)[P], T gg, T G,
                                                  int K, const T* bo, const T* bn) {
  const int Qn = ln.Q;
  const bool dir = DIR && bo != nullptr;
  auto rowof = [&](int q) { return act ? (SIGN > 0 ? j0 + q : Na - 1 - j0 - q) : 0; };
#define KDS_NDR(o, b) node_of<P, DIM, AXIS>(O0 + (o), SIGN > 0 ? (b) : P - 1 - (b))
  T last_old[PER], t_old0[PER], mB[PER];
  {
    const int rl = cbase + rowof(Qn - 1) * NN;
#pragma unroll
    for (int o = 0; o < PER; ++o) last_old[o] = tile[rl + KDS_NDR(o, P - 1)];
  }
#pragma unroll
  for (int o = 0; o < PER; ++o) {
    t_old0[o] = __shfl(last_old[o], ln.src_prev, 64);
    if (dir && ln.first) t_old0[o] = bo[O0 + o];
  }
  // pass 1: zero-inflow recurrence over all my cells, QMAX at a time
  {
    T to[PER], x[PER];
#pragma unroll
    for (int o = 0; o < PER; ++o) { to[o] = t_old0[o]; x[o] = T(0); }
    for (int q0 = 0; q0 < Qn; q0 += QMAX) {
      T dq[QMAX][PER][P];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int r = cbase + rowof(q0 + q < Qn ? q0 + q : 0) * NN;
#pragma unroll
        for (int o = 0; o < PER; ++o)
#pragma unroll
          for (int b = 0; b < P; ++b) dq[q][o][b] = tile[r + KDS_NDR(o, b)];
      }
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        if (q0 + q < Qn) {
#pragma unroll
          for (int o = 0; o < PER; ++o) {
            T bq = e1[P - 1] * to[o];
#pragma unroll
            for (int c = 0; c < P; ++c) bq += C[P - 1][c] * dq[q][o][c];
            x[o] = gg * x[o] + bq;
            to[o] = dq[q][o][P - 1];
          }
        }
      }
    }
#pragma unroll
    for (int o = 0; o < PER; ++o) mB[o] = x[o];
  }
  // segmented inclusive scan over the lanes of each subdomain (as line_group)
  {
    T gw = powi(gg, Qn);
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
  // subdomain iteration on the outflows (as line_group)
  T t_in[PER];
  T bnew[PER];
#pragma unroll
  for (int o = 0; o < PER; ++o) bnew[o] = (dir && ln.s_me == 0) ? bn[O0 + o] : T(0);
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
      for (int o = 0; o < PER; ++o) t_in[o] += Gs * bn[O0 + o];
    } else {
      const T inv = T(1) / (T(1) - Gq);
#pragma unroll
      for (int o = 0; o < PER; ++o) t_in[o] *= inv;
    }
  }
  // pass 2: the new state, QMAX cells at a time, into the tile
  {
    const T g0 = powi(gg, ln.sl * Qn);
    T x[PER], gp[PER], to[PER];
#pragma unroll
    for (int o = 0; o < PER; ++o) {
      T xv = ln.dpp_ok ? dpp_row_shr<T, 1>(mB[o]) : __shfl_up(mB[o], 1, 64);
      x[o] = ln.sl == 0 ? T(0) : xv;
      gp[o] = g0;
      to[o] = t_old0[o];
    }
    for (int q0 = 0; q0 < Qn; q0 += QMAX) {
      T dq[QMAX][PER][P];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int r = cbase + rowof(q0 + q < Qn ? q0 + q : 0) * NN;
#pragma unroll
        for (int o = 0; o < PER; ++o)
#pragma unroll
          for (int b = 0; b < P; ++b) dq[q][o][b] = tile[r + KDS_NDR(o, b)];
      }
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        if (q0 + q < Qn) {
          const int r = cbase + rowof(q0 + q) * NN;
#pragma unroll
          for (int o = 0; o < PER; ++o) {
            const T tn = x[o] + gp[o] * t_in[o];
            T fn[P];
#pragma unroll
            for (int b = 0; b < P; ++b) {
              T acc = e1[b] * to[o] + eth[b] * tn;
#pragma unroll
              for (int c = 0; c < P; ++c) acc += C[b][c] * dq[q][o][c];
              fn[b] = acc;
            }
            T bq = e1[P - 1] * to[o];
#pragma unroll
            for (int c = 0; c < P; ++c) bq += C[P - 1][c] * dq[q][o][c];
            if (act) {
#pragma unroll
              for (int b = 0; b < P; ++b) tile[r + KDS_NDR(o, b)] = fn[b];
            }
            x[o] = bq + gg * x[o];
            to[o] = dq[q][o][P - 1];
            gp[o] *= gg;
          }
        }
      }
    }
  }
#undef KDS_NDR
}

template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, bool DIR, int O0 = 0>
__device__ __forceinline__ void line_lanes_rounds(T* tile, int cbase, int j0, int Na, bool act,
                                                  const LineLane& ln, const T (&C)[P][P],
                                                  const T (&e1)[P], const T (&eth)[P], T gg, T G,
                                                  int K, const T* bo, const T* bn) {
  constexpr int ALL = ColShape<P, DIM>::PER;
  constexpr int GS = ALL <= 4 ? ALL : (ALL % 3 == 0 ? 3 : 4);
  if constexpr (O0 < ALL) {
    constexpr int n = ALL - O0 < GS ? ALL - O0 : GS;
    line_group_rounds<T, P, DIM, AXIS, SIGN, QMAX, NN, O0, n, DIR>(tile, cbase, j0, Na, act, ln, C,
                                                                   e1, eth, gg, G, K, bo, bn);
    line_lanes_rounds<T, P, DIM, AXIS, SIGN, QMAX, NN, DIR, O0 + n>(tile, cbase, j0, Na, act, ln, C,
                                                                    e1, eth, gg, G, K, bo, bn);
  }
}

template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, int NN, bool DIR, int O0 = 0>
__device__ __forceinline__ void line_lanes(T (&d)[QMAX][NN], const LineLane& ln,
                                           const T (&C)[P][P], const T (&e1)[P], const T (&eth)[P],
                                           T gg, T G, int K, const T* bo, const T* bn) {
  constexpr int ALL = ColShape<P, DIM>::PER;
  constexpr int GS = ALL <= 4 ? ALL : (ALL % 3 == 0 ? 3 : 4);
  if constexpr (O0 < ALL) {
    constexpr int n = ALL - O0 < GS ? ALL - O0 : GS;
    line_group<T, P, DIM, AXIS, SIGN, QMAX, NN, O0, n, DIR>(d, ln, C, e1, eth, gg, G, K, bo, bn);
    line_lanes<T, P, DIM, AXIS, SIGN, QMAX, NN, DIR, O0 + n>(d, ln, C, e1, eth, gg, G, K, bo, bn);
  }
}

// ------------------------------------------------- grouped mode (64 nodes)
//
// Cells of 64 nodes (p = 3 in 3-D): the 16 node lines through a cell along
// the velocity axis are solved in four groups of four lines, so a lane keeps
// 16 values per cell in registers.  The lines of different groups share no
// node, so the tile holds two groups at a time: pass h brings groups 2h and
// 2h + 1 (32 values) of every cell of the bundle into LDS, solves them, and
// writes them back while the next pass's values arrive.  A pass is eight runs
// of four nodes contiguous along x; for lines along x or y they form one
// contiguous half cell (128 B in FP32, a whole cache line).  In LDS a cell
// takes kGroupStride values and the cells of a column are interleaved by lane
// (cell j at slot (j mod Q) NL + j / Q, NL lanes per line), so the lanes of a
// wave reading their q-th cells hit distinct banks.

// node offset of run i (four nodes along x) of pass h of the lines along axis
// (z lines: groups 2h + (i mod 2), their runs at z index i / 2)
__device__ __forceinline__ constexpr int group_run(int axis, int h, int i) {
  return axis == 2 ? 8 * h + 4 * (i & 1) + 16 * (i >> 1) : 32 * h + 4 * i;
}

// position inside a cell's LDS slot of node (line O0 + o, index b on AXIS)
template <int P, int DIM, int AXIS>
__device__ constexpr int group_pos(int O0, int o, int b) {
  const int n = node_of<P, DIM, AXIS>(O0 + o, b);
  for (int i = 0; i < 8; ++i)
    if (group_run(AXIS, O0 / 8, i) == (n & ~3)) return 4 * i + (n & 3);
  return 0;
}

// Solve group gi (wave-uniform) of the lanes' cells; cell q of this lane sits
// at tile[cell[q]].
template <typename T, int P, int DIM, int AXIS, int SIGN, int QMAX, bool DIR, int O0 = 0>
__device__ __forceinline__ void group_solve(int gi, T* tile, const int (&cell)[QMAX], bool act,
                                            const LineLane& ln, const T (&C)[P][P],
                                            const T (&e1)[P], const T (&eth)[P], T gg, T G, int K,
                                            const T* bo, const T* bn) {
  constexpr int PER = ColShape<P, DIM>::PER;
  if constexpr (O0 < PER) {
    if (gi > 0) {
      group_solve<T, P, DIM, AXIS, SIGN, QMAX, DIR, O0 + 4>(gi - 1, tile, cell, act, ln, C, e1,
                                                            eth, gg, G, K, bo, bn);
      return;
    }
    T dg[QMAX][4 * P];
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
#pragma unroll
      for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int b = 0; b < P; ++b)
          dg[q][o * P + b] = tile[cell[q] + group_pos<P, DIM, AXIS>(O0, o, b)];
    line_group<T, P, DIM, AXIS, SIGN, QMAX, 4 * P, O0, 4, DIR, true>(dg, ln, C, e1, eth, gg, G, K,
                                                                     bo, bn);
    if (act) {
#pragma unroll
      for (int q = 0; q < QMAX; ++q)
        if (q < ln.Q)
#pragma unroll
          for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int b = 0; b < P; ++b)
              tile[cell[q] + group_pos<P, DIM, AXIS>(O0, o, b)] = dg[q][o * P + b];
    }
  }
}

// x / d for x, d < 2^16 (m = ceil(2^32 / d)): a multiply instead of a division
__device__ __forceinline__ int div_small(int x, uint64_t m) {
  return (int)(((uint64_t)(unsigned)x * m) >> 32);
}
__host__ __device__ __forceinline__ uint64_t div_magic(int d) {
  return ((1ull << 32) + (uint64_t)d - 1) / (uint64_t)d;
}

// The runs of one pass over a bundle: run e = (column c, cell j, run i), in
// the order that keeps neighbouring threads on neighbouring global addresses
// (x bundles: a column is contiguous; y / z bundles: a row of ncols cells is).
struct GroupRuns {
  int64_t gbase, cstride, jstride;  // cell j of column c at gbase + c cstride + j jstride
  int ncols, Na, Q, NL, CSg, axis;
  // a thread's runs: e = threadIdx.x + n blockDim.x; i = e mod 8 is the same
  // for all of them (blockDim.x is a multiple of 64)
  __device__ __forceinline__ int count() const { return ncols * Na * 8; }
  __device__ __forceinline__ void at(int e, int64_t& go, int& lo, uint64_t m_inner,
                                     uint64_t m_q) const {
    const int i = e & 7;
    const int cj = e >> 3;
    const int inner = axis == 0 ? Na : ncols;
    const int outer_i = div_small(cj, m_inner);
    const int inner_i = cj - outer_i * inner;
    const int c = axis == 0 ? outer_i : inner_i;
    const int j = axis == 0 ? inner_i : outer_i;
    const int jq = div_small(j, m_q);
    go = gbase + c * cstride + j * jstride + 4 * i;
    lo = c * CSg + ((j - jq * Q) * NL + jq) * kGroupStride + 4 * i;
  }
};

template <typename T>
struct Run4 {
  using V = typename VecT<T, 16 / sizeof(T)>::type;
  static constexpr int NV = 4 * sizeof(T) / 16;
  V v[NV];
  __device__ __forceinline__ void load(const T* p) {
#pragma unroll
    for (int u = 0; u < NV; ++u) v[u] = reinterpret_cast<const V*>(p)[u];
  }
  __device__ __forceinline__ void store(T* p) const {
#pragma unroll
    for (int u = 0; u < NV; ++u) reinterpret_cast<V*>(p)[u] = v[u];
  }
};

// Write pass h_store (>= 0) back from LDS, then bring pass h_load (>= 0)
// into the same LDS places.  Each thread reads its own places before it
// refills them, so no barrier is needed between the two; the stores are
// still in flight while the loads are issued (U per thread).
template <typename T>
__device__ __forceinline__ void group_exchange(T* __restrict__ f, T* tile, const GroupRuns& gr,
                                               int h_store, int h_load) {
  constexpr int U = 8;
  const int total = gr.count();
  const int bs = blockDim.x;
  const uint64_t m_inner = div_magic(gr.axis == 0 ? gr.Na : gr.ncols);
  const uint64_t m_q = div_magic(gr.Q);
  // run i of a pass sits at the cell's node group_run(axis, h, i); the
  // address from at() carries 4 i, so add the rest
  const int ti = threadIdx.x & 7;
  if (h_store >= 0) {
    const int64_t gadd = group_run(gr.axis, h_store, ti) - 4 * ti;
    for (int e = threadIdx.x; e < total; e += bs) {
      int64_t go;
      int lo;
      gr.at(e, go, lo, m_inner, m_q);
      Run4<T> ov;
      ov.load(tile + lo);
      ov.store(f + go + gadd);
    }
  }
  if (h_load >= 0) {
    const int64_t gadd = group_run(gr.axis, h_load, ti) - 4 * ti;
    for (int e0 = threadIdx.x; e0 < total; e0 += U * bs) {
      int64_t go[U];
      int lo[U];
      Run4<T> nv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // slots past the end re-read the first run (never stored)
        gr.at(e0 + u * bs < total ? e0 + u * bs : e0, go[u], lo[u], m_inner, m_q);
        nv[u].load(f + go[u] + gadd);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u * bs < total) nv[u].store(tile + lo[u]);
    }
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
// RND: some velocity's lanes own more cells than the registers hold (rounds
// through the tile; a separate instantiation keeps the other kernels'
// registers unchanged).
template <typename T, int P, int DIM, bool DIR, bool RND = false>
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

  // x lines with QMAX cells per lane: each lane's cells are one contiguous,
  // aligned block of QMAX * NN values, read and written straight from / to
  // registers (no LDS tile, no barriers)
  using LVT = typename VecT<T, LineVec<T, QMAX * NN>::VW>::type;
  constexpr int LV = LineVec<T, QMAX * NN>::VW;
  constexpr bool GROUPED = line_grouped(NN);
  const bool direct = !GROUPED && pl.xdirect && a == 0 && Q == QMAX && kc_base % LV == 0 &&
                      CS % LV == 0;
  const int64_t col0 = a == 0 ? bundle * bw : 0;

  // ------------------------------------------------------------ bundle
  // cell j of column c of the bundle sits at gbase + c cstride + j rowstride
  int ncols;
  int64_t gbase, rowstride;
  if (a == 0) {
    const int64_t nrows = g.ncell / Na;
    ncols = (int)min<int64_t>(bw, nrows - col0);
    gbase = kc_base + col0 * CS;
    rowstride = NN;
  } else {
    const int nbx = (g.N[0] + bw - 1) / bw;
    const int bx = (int)(bundle % nbx);
    const int64_t other = bundle / nbx;
    const int x0 = bx * bw;
    ncols = min(bw, g.N[0] - x0);
    gbase = a == 1 ? kc_base + (other * g.N[1] * g.N[0] + x0) * (int64_t)NN
                   : kc_base + (other * g.N[0] + x0) * (int64_t)NN;
    rowstride = a == 1 ? (int64_t)g.N[0] * NN : (int64_t)g.N[0] * g.N[1] * NN;
  }
  const GroupRuns gr{gbase, a == 0 ? (int64_t)CS : (int64_t)NN, rowstride, ncols, Na, Q, NL,
                     Na * kGroupStride, a};
  if constexpr (GROUPED) {
    group_exchange<T>(f, tile, gr, -1, 0);
  } else if (a == 0) {
    // consecutive rows of cells are one contiguous block
    if (!direct) copy_tile<T, true>(f, tile, gbase, CS, CS, ncols);
  } else {
    copy_cols<T, NN, true>(f, tile, gbase, rowstride, ncols, Na, CS);
  }
  if (!direct) __syncthreads();

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
  const int64_t boff = (DIR && bd.old != nullptr && bd.off[a][bside] >= 0)
                           ? (int64_t)kc * bd.nb + bd.off[a][bside] : -1;

  // grouped mode: passes of two groups of node lines each
  constexpr int NPASS = GROUPED ? ColShape<P, DIM>::PER / 8 : 1;
  for (int h = 0; h < NPASS; ++h) {
    if (GROUPED && h > 0) {
      // write pass h - 1 back while pass h arrives
      __syncthreads();
      group_exchange<T>(f, tile, gr, h - 1, h);
      __syncthreads();
    }
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
      if constexpr (GROUPED) {
        int cell[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int row = (act && q < Q) ? (sg > 0 ? j0 + q : Na - 1 - j0 - q) : 0;
          cell[q] = (act ? c : 0) * gr.CSg + ((row % Q) * NL + row / Q) * kGroupStride;
        }
        for (int gi = 2 * h; gi < 2 * h + 2; ++gi) {
          switch (a * 2 + (sg > 0 ? 1 : 0)) {
            case 0: group_solve<T, P, DIM, 0, -1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
            case 1: group_solve<T, P, DIM, 0, 1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
            case 2: if constexpr (DIM > 1) group_solve<T, P, DIM, 1, -1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
            case 3: if constexpr (DIM > 1) group_solve<T, P, DIM, 1, 1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
            case 4: if constexpr (DIM > 2) group_solve<T, P, DIM, 2, -1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
            default: if constexpr (DIM > 2) group_solve<T, P, DIM, 2, 1, QMAX, DIR>(gi, tile, cell, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          }
        }
        continue;
      } else if (RND && Q > QMAX) {
        // more cells per lane than the registers hold: rounds through the tile
        if constexpr (RND)
        switch (a * 2 + (sg > 0 ? 1 : 0)) {
          case 0: line_lanes_rounds<T, P, DIM, 0, -1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 1: line_lanes_rounds<T, P, DIM, 0, 1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 2: if constexpr (DIM > 1) line_lanes_rounds<T, P, DIM, 1, -1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 3: if constexpr (DIM > 1) line_lanes_rounds<T, P, DIM, 1, 1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 4: if constexpr (DIM > 2) line_lanes_rounds<T, P, DIM, 2, -1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          default: if constexpr (DIM > 2) line_lanes_rounds<T, P, DIM, 2, 1, QMAX, NN, DIR>(tile, cbase, j0, Na, act, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
        }
      } else {
        T d[QMAX][NN];
        // direct: my block starts at cell j0 (downwind = physical order) or at
        // Na - j0 - QMAX (reversed); lanes without a line read column 0
        const int64_t dbase = kc_base + (col0 + (act ? c : 0)) * CS +
                              (int64_t)(act ? (sg > 0 ? j0 : Na - j0 - QMAX) : 0) * NN;
        if (direct) {
          LVT v[QMAX * NN / LV];
          const LVT* src = reinterpret_cast<const LVT*>(f + dbase);
#pragma unroll
          for (int i = 0; i < QMAX * NN / LV; ++i) v[i] = src[i];
          const T* vs = reinterpret_cast<const T*>(v);
#pragma unroll
          for (int q = 0; q < QMAX; ++q)
#pragma unroll
            for (int n = 0; n < NN; ++n) d[q][n] = vs[(sg > 0 ? q : QMAX - 1 - q) * NN + n];
        } else {
#pragma unroll
          for (int q = 0; q < QMAX; ++q) {
            const int row = (act && q < Q) ? (sg > 0 ? j0 + q : Na - 1 - j0 - q) : 0;
#pragma unroll
            for (int n = 0; n < NN; ++n) d[q][n] = tile[cbase + row * NN + n];
          }
        }
        switch (a * 2 + (sg > 0 ? 1 : 0)) {
          case 0: line_lanes<T, P, DIM, 0, -1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 1: line_lanes<T, P, DIM, 0, 1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 2: if constexpr (DIM > 1) line_lanes<T, P, DIM, 1, -1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 3: if constexpr (DIM > 1) line_lanes<T, P, DIM, 1, 1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          case 4: if constexpr (DIM > 2) line_lanes<T, P, DIM, 2, -1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
          default: if constexpr (DIM > 2) line_lanes<T, P, DIM, 2, 1, QMAX, NN, DIR>(d, ln, C, e1, eth, gg, G, g.K, bo, bn); break;
        }
        if (act && direct) {
          LVT v[QMAX * NN / LV];
          T* vs = reinterpret_cast<T*>(v);
#pragma unroll
          for (int q = 0; q < QMAX; ++q)
#pragma unroll
            for (int n = 0; n < NN; ++n) vs[(sg > 0 ? q : QMAX - 1 - q) * NN + n] = d[q][n];
          LVT* dst = reinterpret_cast<LVT*>(f + dbase);
#pragma unroll
          for (int i = 0; i < QMAX * NN / LV; ++i) dst[i] = v[i];
        } else if (act) {
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
    }
  }  // passes
  if (direct) return;
  __syncthreads();

  // -------------------------------------------------------- write back
  if constexpr (GROUPED) {
    group_exchange<T>(f, tile, gr, NPASS - 1, -1);
  } else if (a == 0) {
    copy_tile<T, false>(f, tile, gbase, CS, CS, ncols);
  } else {
    copy_cols<T, NN, false>(f, tile, gbase, rowstride, ncols, Na, CS);
  }
}

// DIR: some axis has Dirichlet ends (a separate instantiation keeps the
// periodic kernel's registers unchanged); RND: lanes with cells in rounds
template <typename T, int P, int DIM, bool DIR, bool RND = false>
__global__ __launch_bounds__(256) void k_sweep_line(T* __restrict__ f, Geom g, SweepTab<T> tab,
                                                    LinePlan pl, BndRef<T> bd) {
  extern __shared__ unsigned char smem_raw[];
  line_bundle<T, P, DIM, DIR, RND>(f, g, tab, pl, bd, xcd_order(pl.block_start[g.nv * g.m]),
                                   reinterpret_cast<T*>(smem_raw));
}

// Many problems of one (precision, degree, dimension) in one launch: the
// bundles of all problems are numbered consecutively (start[] prefix).
template <typename T, int P, int DIM, bool RND = false, bool DIR = false>
__global__ __launch_bounds__(256) void k_sweep_line_batch(const LineTask<T>* __restrict__ tasks,
                                                          const int64_t* __restrict__ start,
                                                          int ntask) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t gbid = xcd_order(start[ntask]);
  int pid = 0;
  while (gbid >= start[pid + 1]) ++pid;
  const LineTask<T>& t = tasks[pid];
  // (DIR: members with Dirichlet axes, whose boundary data the records point to)
  line_bundle<T, P, DIM, DIR, RND>(t.f, t.g, t.tab, t.pl, t.bd, gbid - start[pid],
                                   reinterpret_cast<T*>(smem_raw));
}

template <typename T>
hipError_t sweep_line_t(const Geom& g, const void* tab, const LinePlan& plan, void* f,
                        const BndArgs& bnd, hipStream_t s) {
  const BndRef<T> bd = bnd_ref<T>(bnd);
  const SweepTab<T>& t = *(const SweepTab<T>*)tab;
  const int64_t nblocks = plan.block_start[g.nv * g.m];
  const size_t lds = (size_t)std::max(plan.lds_elems, plan.lds_alloc) * sizeof(T);
  const int key = g.P * 10 + g.dim;
  const bool rnd = line_plan_rounds(g, plan, (int)sizeof(T));
  switch (key) {
#define KDS_LINE(PP, DD)                                                                        \
  case PP * 10 + DD:                                                                            \
    if (rnd && !line_grouped(ColShape<PP, DD>::NN)) {                                           \
      if (bd.old != nullptr)                                                                    \
        hipLaunchKernelGGL((k_sweep_line<T, PP, DD, true, true>), dim3((unsigned)nblocks),      \
                           dim3(plan.threads), lds, s, (T*)f, g, t, plan, bd);                  \
      else                                                                                      \
        hipLaunchKernelGGL((k_sweep_line<T, PP, DD, false, true>), dim3((unsigned)nblocks),     \
                           dim3(plan.threads), lds, s, (T*)f, g, t, plan, bd);                  \
    } else if (bd.old != nullptr) {                                                             \
      hipLaunchKernelGGL((k_sweep_line<T, PP, DD, true>), dim3((unsigned)nblocks),              \
                         dim3(plan.threads), lds, s, (T*)f, g, t, plan, bd);                    \
    } else {                                                                                    \
      hipLaunchKernelGGL((k_sweep_line<T, PP, DD, false>), dim3((unsigned)nblocks),             \
                         dim3(plan.threads), lds, s, (T*)f, g, t, plan, bd);                    \
    }                                                                                           \
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


template <typename T>
hipError_t sweep_line_batch_t(int P, int dim, bool rounds, bool dir, const void* tasks,
                              const int64_t* start, int ntask, int64_t nblocks, int threads,
                              size_t lds_elems, hipStream_t s) {
  const size_t lds = lds_elems * sizeof(T);
  const LineTask<T>* tk = (const LineTask<T>*)tasks;
  switch (P * 10 + dim) {
#define KDS_LB(PP, DD)                                                                          \
  case PP * 10 + DD:                                                                            \
    if (rounds && !line_grouped(ColShape<PP, DD>::NN)) {                                        \
      if (dir)                                                                                  \
        hipLaunchKernelGGL((k_sweep_line_batch<T, PP, DD, true, true>), dim3((unsigned)nblocks),  \
                           dim3(threads), lds, s, tk, start, ntask);                            \
      else                                                                                      \
        hipLaunchKernelGGL((k_sweep_line_batch<T, PP, DD, true>), dim3((unsigned)nblocks),      \
                           dim3(threads), lds, s, tk, start, ntask);                            \
    } else if (dir) {                                                                           \
      hipLaunchKernelGGL((k_sweep_line_batch<T, PP, DD, false, true>), dim3((unsigned)nblocks), \
                         dim3(threads), lds, s, tk, start, ntask);                              \
    } else {                                                                                    \
      hipLaunchKernelGGL((k_sweep_line_batch<T, PP, DD>), dim3((unsigned)nblocks),              \
                         dim3(threads), lds, s, tk, start, ntask);                              \
    }                                                                                           \
    break;
    KDS_LB(1, 1) KDS_LB(2, 1) KDS_LB(3, 1) KDS_LB(4, 1)
    KDS_LB(1, 2) KDS_LB(2, 2) KDS_LB(3, 2) KDS_LB(4, 2)
    KDS_LB(1, 3) KDS_LB(2, 3) KDS_LB(3, 3) KDS_LB(4, 3)
#undef KDS_LB
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t line_allow_lds_t(size_t bytes) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* k) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  };
#define KDS_ALLOW(PP, DD)                                                      \
  set(reinterpret_cast<const void*>(&k_sweep_line<T, PP, DD, false>));         \
  set(reinterpret_cast<const void*>(&k_sweep_line<T, PP, DD, true>));          \
  if (!line_grouped(ColShape<PP, DD>::NN)) {                                   \
    set(reinterpret_cast<const void*>(&k_sweep_line<T, PP, DD, false, true>)); \
    set(reinterpret_cast<const void*>(&k_sweep_line<T, PP, DD, true, true>));  \
    set(reinterpret_cast<const void*>(&k_sweep_line_batch<T, PP, DD, true>));  \
    set(reinterpret_cast<const void*>(&k_sweep_line_batch<T, PP, DD, true, true>));   \
  }                                                                                  \
  set(reinterpret_cast<const void*>(&k_sweep_line_batch<T, PP, DD>));                \
  set(reinterpret_cast<const void*>(&k_sweep_line_batch<T, PP, DD, false, true>));
  KDS_ALLOW(1, 1) KDS_ALLOW(2, 1) KDS_ALLOW(3, 1) KDS_ALLOW(4, 1)
  KDS_ALLOW(1, 2) KDS_ALLOW(2, 2) KDS_ALLOW(3, 2) KDS_ALLOW(4, 2)
  KDS_ALLOW(1, 3) KDS_ALLOW(2, 3) KDS_ALLOW(3, 3) KDS_ALLOW(4, 3)
#undef KDS_ALLOW
  return e;
}

template <typename T>
void pack_line_task_t(void* f, const Geom& g, const void* tab, const LinePlan& pl,
                      const BndArgs& bnd, void* out) {
  LineTask<T> t;
  t.f = (T*)f;
  t.g = g;
  std::memcpy(&t.tab, tab, sizeof(t.tab));
  t.pl = pl;
  t.bd = bnd_ref<T>(bnd);
  std::memcpy(out, &t, sizeof(t));
}

// The host entry points of one element type (one translation unit each, so
// the two precisions compile in parallel).
#define KDS_LINE_TU(T, SFX)                                                                    \
  hipError_t sweep_line_##SFX(const Geom& g, const void* tab, const LinePlan& plan, void* f,   \
                              const BndArgs& bnd, hipStream_t s) {                             \
    return sweep_line_t<T>(g, tab, plan, f, bnd, s);                                           \
  }                                                                                            \
  hipError_t sweep_line_batch_##SFX(int P, int dim, bool rounds, bool dir, const void* tasks,  \
                                    const int64_t* start, int ntask, int64_t nblocks,          \
                                    int threads, size_t lds_elems, hipStream_t s) {            \
    return sweep_line_batch_t<T>(P, dim, rounds, dir, tasks, start, ntask, nblocks, threads,   \
                                 lds_elems, s);                                                \
  }                                                                                            \
  hipError_t line_allow_lds_##SFX(size_t bytes) { return line_allow_lds_t<T>(bytes); }         \
  size_t line_task_bytes_##SFX() { return sizeof(LineTask<T>); }                               \
  void pack_line_task_##SFX(void* f, const Geom& g, const void* tab, const LinePlan& pl,       \
                            const BndArgs& bnd, void* out) {                                   \
    pack_line_task_t<T>(f, g, tab, pl, bnd, out);                                              \
  }

}  // namespace kds
