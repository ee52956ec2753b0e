// kds_front_wave.hip -- the front schedule with one wave per
// (velocity, subdomain, component): the FP32 matrix-core forms for cells of
// up to 64 nodes (p <= 3), and FP64 on the FP64 matrix cores for cells of at
// most 32 nodes (p <= 2 in 3-D, p <= 3 in 2-D).
//
// The same computation as k_sweep_front (the solves of one anti-diagonal
// front of the V-oriented cell graph as one GEMM Y = W X per front, Sec. 3.2,
// one launch per subdomain iteration, eq:ibvp), arranged for latency:
//   * a wave owns a whole task and never waits at a barrier: the levels of a
//     subdomain follow each other in program order, and many independent
//     waves per SIMD hide each other's memory latency;
//   * the GEMM input never goes through LDS: lane (j, g) of the wave gathers
//     KS values of column j straight into the B operand registers of the
//     16x16 matrix-core products.  The K index of the products is permuted
//     so that register slot e holds the same kind of row in all four lane
//     groups g: slots 0 .. CS-1 a run of CS consecutive cell nodes, then FS
//     slots per inflow axis a with a run of face nodes.  Kind, axis and the
//     address pattern of a slot are compile-time constants, so the cell
//     values arrive with a few wide loads and a face slot costs one or two
//     loads with an immediate offset;
//   * the traces inside the subdomain stay in LDS: a cell writes
//     theta t^n + (1 - theta) t^{n-1} on its outflow faces into the wave's
//     frontier (one slot per grid line through the subdomain and axis),
//     where the next cell of that line reads its inflow;
//   * global memory is read through range-checked buffer loads with 32-bit
//     offsets: a row without a global source reads from an offset past the
//     buffer, which returns 0 (one load pattern for every lane, no 64-bit
//     address selects); stores of padding outputs are dropped the same way;
//   * the cell records (offset, downwind coordinates, frontier positions)
//     are built on the host, 16 bytes per cell in front order, and the next
//     tile's records load while the current tile computes.
#include "kds_device.h"

namespace kds {

namespace {

constexpr unsigned kOob = 0x80000000u;  // byte offset past every buffer of the kernel

typedef float wf32x4 __attribute__((ext_vector_type(4)));
typedef double wf64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 wf16x4 __attribute__((ext_vector_type(4)));
typedef short wi16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const void* p, int64_t bytes) {
  // raw buffer (stride 0), range `bytes`; word 3 = the gfx9 data format
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
// n consecutive values at byte offset o, with the widest loads
template <int N>
__device__ __forceinline__ void bload_run(__amdgpu_buffer_rsrc_t r, unsigned o, float* v) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u3 __attribute__((ext_vector_type(3)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if constexpr (N >= 4) {
    const u4 x = __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __uint_as_float(x[u]);
    bload_run<N - 4>(r, o + 16u, v + 4);
  } else if constexpr (N == 3) {
    const u3 x = __builtin_amdgcn_raw_buffer_load_b96(r, o, 0, 0);
#pragma unroll
    for (int u = 0; u < 3; ++u) v[u] = __uint_as_float(x[u]);
  } else if constexpr (N == 2) {
    const u2 x = __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0);
    v[0] = __uint_as_float(x[0]);
    v[1] = __uint_as_float(x[1]);
  } else if constexpr (N == 1) {
    v[0] = bload(r, o);
  }
}
// n consecutive values to byte offset o, with the widest stores
template <int N>
__device__ __forceinline__ void bstore_run(__amdgpu_buffer_rsrc_t r, unsigned o, const float* v) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u3 __attribute__((ext_vector_type(3)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if constexpr (N >= 4) {
    const u4 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                  __float_as_uint(v[3])};
    __builtin_amdgcn_raw_buffer_store_b128(x, r, o, 0, 0);
    bstore_run<N - 4>(r, o + 16u, v + 4);
  } else if constexpr (N == 3) {
    const u3 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
    __builtin_amdgcn_raw_buffer_store_b96(x, r, o, 0, 0);
  } else if constexpr (N == 2) {
    const u2 x = {__float_as_uint(v[0]), __float_as_uint(v[1])};
    __builtin_amdgcn_raw_buffer_store_b64(x, r, o, 0, 0);
  } else if constexpr (N == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), r, o, 0, 0);
  }
}

// the same for FP64 values (8-byte elements: pairs with 16-byte accesses)
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const u2 x = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  return __builtin_bit_cast(double, x);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float) {
  return bload(r, byte_off);
}
template <int N>
__device__ __forceinline__ void bload_run(__amdgpu_buffer_rsrc_t r, unsigned o, double* v) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if constexpr (N >= 2) {
    const u4 x = __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
    v[0] = __builtin_bit_cast(double, u2{x[0], x[1]});
    v[1] = __builtin_bit_cast(double, u2{x[2], x[3]});
    bload_run<N - 2>(r, o + 16u, v + 2);
  } else if constexpr (N == 1) {
    v[0] = bload(r, o, 0.0);
  }
}
template <int N>
__device__ __forceinline__ void bstore_run(__amdgpu_buffer_rsrc_t r, unsigned o, const double* v) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if constexpr (N >= 2) {
    const u2 a = __builtin_bit_cast(u2, v[0]), b = __builtin_bit_cast(u2, v[1]);
    const u4 x = {a[0], a[1], b[0], b[1]};
    __builtin_amdgcn_raw_buffer_store_b128(x, r, o, 0, 0);
    bstore_run<N - 2>(r, o + 16u, v + 2);
  } else if constexpr (N == 1) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v[0]), r, o, 0, 0);
  }
}

__device__ __forceinline__ unsigned short wbf16_rne(float x) {
  const unsigned int b = __float_as_uint(x);
  return (unsigned short)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float wbf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

// Compile-time shape of a cell: nodes, face nodes, register slots.
template <int DIM, int P>
struct WaveShape {
  static constexpr int NN = DIM == 3 ? P * P * P : P * P;
  static constexpr int NF = DIM == 3 ? P * P : P;
  static constexpr int CS = (NN + 3) / 4;       // cell slots
  static constexpr int FS = (NF + 3) / 4;       // slots per inflow axis
  static constexpr int FSTR = NF | 1;           // frontier values per line (odd: LDS banks)
  static constexpr int KS0 = CS + DIM * FS;
  static constexpr int MT = (NN + 15) / 16;     // 16-row output tiles
  static constexpr int XOS = 16 * MT + 1;       // cell values of a tile, per column
};

// One problem of a batched launch (one subdomain iteration).
template <typename T>
struct FrontWaveTask {
  const T* f_old;
  const T* f_prev;
  T* f_cur;
  Geom g;
  FrontParams fp;
  const T* Wop;
  const int* lvl_start;
  const int4* desc;
  int n_desc;
  BndRef<T> bd;
};

template <int MODE, int KS0>
struct WaveK {
  // slots per lane: the 16x16x16 products take four per step
  static constexpr int KS = MODE == kFrontMfma ? KS0 : (KS0 + 3) / 4 * 4;
};

// The tasks' work: levels of one subdomain, tiles of 16 cells of a level.
// BND: Dirichlet box faces on the subdomain's inflow side (boundary traces
// are a second pair of buffers).
template <typename T, int MODE, int DIM, int P, bool BND>
__device__ __forceinline__ void front_wave_task(
    const Geom& g, const FrontParams& fp, const T* __restrict__ Wk,
    const int* __restrict__ lvl_start, const int4* __restrict__ desc, int n_desc, int k,
    const int (&sg)[3], const int (&sdc)[3], const int (&nbrel)[3], const int (&isb)[3],
    const int (&boff)[3], unsigned sdb, __amdgpu_buffer_rsrc_t rfo, __amdgpu_buffer_rsrc_t rfp,
    __amdgpu_buffer_rsrc_t rfc, __amdgpu_buffer_rsrc_t rbo, __amdgpu_buffer_rsrc_t rbn, T* FR,
    T* XO) {
  using S = WaveShape<DIM, P>;
  constexpr int NN = S::NN, NF = S::NF, CS = S::CS, FS = S::FS, FSTR = S::FSTR, MT = S::MT,
                XOS = S::XOS;
  constexpr int KS = WaveK<MODE, S::KS0>::KS;
  constexpr int KB = KS / 4 > 0 ? KS / 4 : 1;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  const int Kd = fp.Kd;
  constexpr unsigned ES = sizeof(T);  // bytes per value (offsets below are in bytes)
  const T th = (T)fp.theta, th1 = T(1) - th;
  const int frn = 3 * fp.fr_pos * FSTR;  // frontier values; FR[frn] is a write sink
  // Slots of lane group lk: cell nodes cst .. cst + CS - 1 and face nodes
  // fst .. fst + FS - 1, runs inside the cell and the face (the last group's
  // run starts early; the slots it shares with the group before get zero
  // operator columns), so that every read stays inside its cell or face.
  const int cst = min(lk * CS, NN - CS), fst = min(lk * FS, NF - FS);

  // ---- the operator slice: lane (i, g) of row tile t holds operator row
  // 16 t + i at the K positions of slots e (e = st in the 16x16x4 products,
  // 4 st + u in the 16x16x16 ones)
  T afr[MODE == kFrontMfma ? MT : 1][MODE == kFrontMfma ? KS : 1];
  wf16x4 ah16[MODE == kFrontSplitF16 ? MT : 1][KB], al16[MODE == kFrontSplitF16 ? MT : 1][KB];
  wi16x4 ahb[MODE == kFrontSplitBf16 ? MT : 1][KB], alb[MODE == kFrontSplitBf16 ? MT : 1][KB];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int i = 16 * t + li;
#pragma unroll
    for (int e = 0; e < KS; ++e) {
      // the operator column of slot e in lane group lk (-1: a slot that
      // repeats a value of the group before)
      int col = -1;
      if (e < CS) {
        const int node = cst + e;
        col = node >= lk * CS ? node : -1;
      } else if (e < CS + DIM * FS) {
        const int a = (e - CS) / FS, q = fst + (e - CS) % FS;
        col = q >= lk * FS ? NN + a * NF + q : -1;
      }
      const T w = (i < NN && col >= 0) ? Wk[i * Kd + col] : T(0);
      if constexpr (MODE == kFrontMfma) {
        afr[t][e] = w;
      } else if constexpr (MODE == kFrontSplitF16) {
        const _Float16 h = (_Float16)w;
        ah16[t][e / 4][e % 4] = h;
        al16[t][e / 4][e % 4] = (_Float16)((w - (float)h) * 2048.0f);
      } else {
        const unsigned short h = wbf16_rne(w);
        ahb[t][e / 4][e % 4] = (short)h;
        alb[t][e / 4][e % 4] = (short)wbf16_rne(w - wbf16_to_f32(h));
      }
    }
  }

  // ---- per lane: the byte offset of face node q = 4 j + lk inside the
  // upwind neighbour's cell (its outflow index on axis a, the others from q,
  // x fastest) and inside a boundary face block
  unsigned nbn4[3][FS], bq4[FS];
#pragma unroll
  for (int j = 0; j < FS; ++j) {
    const int q = fst + j;
    bq4[j] = ES * q;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int side = sg[a] > 0 ? P - 1 : 0;
      const int node = a == 0 ? side + P * q
                              : (a == 1 ? (q % P) + P * side + P * P * (q / P) : q + P * P * side);
      nbn4[a][j] = a < DIM ? ES * node : kOob;
    }
  }
  // the frontier starts at zero (a read it serves before the upwind cell wrote
  // it is discarded, but stays a finite number)
  for (int x = lane; x <= frn; x += 64) FR[x] = T(0);

  // ---- the global loads of a tile (records d; columns with `ok`): the cell
  // values at t^{n-1}, and on inflow faces across an interface or a Dirichlet
  // box face the old and new traces.  None of them depends on the sweep, so
  // a tile's loads are issued while the tile before it computes.
  auto issue = [&](const int4 d, bool ok, T (&pc)[CS], T (&pvo)[DIM * FS],
                   T (&pvn)[DIM * FS]) {
    const unsigned off = sdb + (unsigned)d.x;  // node 0 of the cell in its plane
    const int pk = d.y;
    // nodes cst .. cst + CS - 1: consecutive, read with wide loads
    bload_run<CS>(rfo, ok ? (off + (unsigned)cst) * ES : kOob, pc);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      // the first cell of the subdomain along a reads across the interface
      // (iterate p-1, periodic wrap included) or the boundary data
      const int la = (pk >> (10 * a)) & 1023;
      const bool first = ok && sg[a] != 0 && la == 0;
      const unsigned nb4 = (first && !isb[a]) ? ((unsigned)((int)off + nbrel[a])) * ES : kOob;
      unsigned bb4 = kOob;
      if constexpr (BND) {
        // the boundary node block of the cell's face: cells over the other axes
        int fcell = 0, mul = 1;
#pragma unroll
        for (int o = 0; o < DIM; ++o)
          if (o != a) {
            const int lc = (pk >> (10 * o)) & 1023;
            const int pl = sg[o] < 0 ? g.S[o] - 1 - lc : lc;
            fcell += (sdc[o] * g.S[o] + pl) * mul;
            mul *= g.N[o];
          }
        if (first && isb[a]) bb4 = (unsigned)(boff[a] + fcell * NF) * ES;
      }
#pragma unroll
      for (int j = 0; j < FS; ++j) pvo[a * FS + j] = pvn[a * FS + j] = T(0);
      // (the host puts a front's first cells first: most tiles have none)
      if (__any(first)) {
#pragma unroll
        for (int j = 0; j < FS; ++j) {
          const int s = a * FS + j;
          pvo[s] = bload(rfo, nb4 + nbn4[a][j], T(0));
          pvn[s] = bload(rfp, nb4 + nbn4[a][j], T(0));
          if constexpr (BND) {
            // a row reads the state or the boundary data, never both: the
            // other load is out of range and adds an exact 0
            pvo[s] += bload(rbo, bb4 + bq4[j], T(0));
            pvn[s] += bload(rbn, bb4 + bq4[j], T(0));
          }
        }
      }
    }
  };
  // tiles: (first cell, end of its level, level); the successor of a tile is
  // the rest of its level, or the next level
  const int lo = fp.lvl_off[k], nlev = fp.nlev[k];
  auto advance = [&](int cb, int ce, int lev, int& ncb, int& nce, int& nlv) {
    ncb = cb + 16;
    nce = ce;
    nlv = lev;
    if (ncb >= ce) {
      ncb = ce;
      nlv = lev + 1;
      nce = nlv < nlev ? lvl_start[lo + nlv + 1] : ce;
    }
  };
  int cb = lvl_start[lo], ce = lvl_start[lo + 1], lev = 0;
  int ncb, nce, nlev2;
  advance(cb, ce, lev, ncb, nce, nlev2);
  int4 dc = desc[min(cb + li, n_desc - 1)];
  // Two sets of registers for the prefetched records and cell values, used
  // in turn: a tile reads the set the tile before it loaded and loads the
  // other one, so no load in flight is copied between registers (a copy at
  // the end of the loop would wait for the load there, a tile early).  The
  // face values are consumed before the next ones are loaded: one set.
  int4 dA = desc[min(ncb + li, n_desc - 1)], dB = dA;
  T pcA[CS], pcB[CS], pvo[DIM * FS], pvn[DIM * FS];
  issue(dc, cb + li < ce, pcA, pvo, pvn);
  // (the first tile needs these at once; waiting here also leaves nothing
  // in flight on the way into the loop, so the waits inside it count only
  // the loads a tile ahead, not the stores issued after them)
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
  // one tile: the current record dc, cell values pc and face values (pvo,
  // pvn); dn: the next tile's record (loaded a tile ago); dnn_out, pcN: where
  // the record after it and the next tile's cell values are loaded
  auto tile = [&](const int4& dn, int4& dnn_out, const T(&pc)[CS], T(&pcN)[CS])
                  __attribute__((always_inline)) {
    // ---- this tile's columns: lane j's cell (its loads were issued a tile ago)
    const bool valid = cb + li < ce;
    const unsigned off = sdb + (unsigned)dc.x;
    const int pk = dc.y;
    const int pos[3] = {dc.z & 0xffff, (int)((unsigned)dc.z >> 16), dc.w};
    int frb[3];
    bool isfr[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      frb[a] = (a * fp.fr_pos + pos[a]) * FSTR;
      isfr[a] = valid && sg[a] != 0 && ((pk >> (10 * a)) & 1023) > 0;
    }
    // ---- the GEMM input: cell slots, then face slots (frontier, or the
    // theta-combined traces loaded with the cell values).  Every lane reads
    // its frontier slots (in range for any record) and both candidates are
    // formed before the selects: the reads go out together, and no lane
    // branches on its face kind.
    T bx[KS];
#pragma unroll
    for (int e = 0; e < CS; ++e) bx[e] = pc[e];
    T frv[DIM * FS], trv[DIM * FS];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int j = 0; j < FS; ++j) frv[a * FS + j] = FR[frb[a] + fst + j];
#pragma unroll
    for (int s = 0; s < DIM * FS; ++s) {
      trv[s] = th1 * pvo[s] + th * pvn[s];
      // (keeps each candidate a computed value, so the select below stays a
      // select rather than becoming a branch around a load)
      __asm__ volatile("" ::"v"(frv[s]), "v"(trv[s]));
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int j = 0; j < FS; ++j) {
        const int s = a * FS + j;
        bx[CS + s] = isfr[a] ? frv[s] : trv[s];
      }
#pragma unroll
    for (int e = CS + DIM * FS; e < KS; ++e) bx[e] = T(0);
    // the cell's own values, for the outflow traces of the epilogue
#pragma unroll
    for (int e = 0; e < CS; ++e) XO[li * XOS + cst + e] = bx[e];

    // ---- the next tile's loads, and the records of the one after
    int nncb, nnce, nlev3;
    advance(ncb, nce, nlev2, nncb, nnce, nlev3);
    dnn_out = desc[min(nncb + li, n_desc - 1)];
    issue(dn, nlev2 < nlev && ncb + li < nce, pcN, pvo, pvn);

    // ---- Y = W X
    using AccV = typename std::conditional<sizeof(T) == 8, wf64x4, wf32x4>::type;
    AccV acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = AccV{T(0), T(0), T(0), T(0)};
    if constexpr (MODE == kFrontMfma) {
#pragma unroll
      for (int e = 0; e < KS; ++e)
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if constexpr (sizeof(T) == 8)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[t][e], bx[e], acc[t], 0, 0, 0);
          else
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[t][e], bx[e], acc[t], 0, 0, 0);
        }
    } else {
      wf32x4 cor[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) cor[t] = wf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < KS / 4; ++st) {
        if constexpr (MODE == kFrontSplitF16) {
          wf16x4 bh, bl;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float b = bx[4 * st + u];
            const _Float16 hb = (_Float16)b;
            bh[u] = hb;
            bl[u] = (_Float16)((b - (float)hb) * 2048.0f);
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah16[t][st], bh, acc[t], 0, 0, 0);
            cor[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah16[t][st], bl, cor[t], 0, 0, 0);
            cor[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(al16[t][st], bh, cor[t], 0, 0, 0);
          }
        } else {
          wi16x4 bh, bl;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float b = bx[4 * st + u];
            const unsigned short hb = wbf16_rne(b);
            bh[u] = (short)hb;
            bl[u] = (short)wbf16_rne(b - wbf16_to_f32(hb));
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahb[t][st], bh, acc[t], 0, 0, 0);
            cor[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahb[t][st], bl, cor[t], 0, 0, 0);
            cor[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alb[t][st], bh, cor[t], 0, 0, 0);
          }
        }
      }
      const float sc = MODE == kFrontSplitF16 ? 1.0f / 2048.0f : 1.0f;
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] += sc * cor[t][v];
    }

    // ---- the iterate and the outflow traces, through the tile buffer (a
    // product row is spread over four lanes; the buffer regroups the values
    // by cell): it holds the values at t^{n-1}, then the new ones, which each
    // lane stores as its run of nodes with wide stores, then the traces
    // theta y + (1 - theta) f^{n-1}, which each lane copies into the frontier
    // for its face-node runs (a cell's outflow node with face index q on axis
    // a is the node its downwind neighbour reads as the upwind one)
    T* TB = XO + li * XOS;
    // product row of item v of row tile t in this lane: FP32 products give
    // a lane four consecutive rows, FP64 products every fourth row
    auto orow = [&](int t, int v) {
      return sizeof(T) == 8 ? 16 * t + 4 * v + lk : 16 * t + 4 * lk + v;
    };
    T xo[MT][4];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) xo[t][v] = TB[orow(t, v)];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) TB[orow(t, v)] = acc[t][v];
    T yr[CS];
#pragma unroll
    for (int e = 0; e < CS; ++e) yr[e] = TB[cst + e];
    bstore_run<CS>(rfc, valid ? (off + (unsigned)cst) * ES : kOob, yr);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) TB[orow(t, v)] = th * acc[t][v] + th1 * xo[t][v];
    // (all trace reads before the frontier writes: one LDS round trip)
    T zv[DIM * FS];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int j = 0; j < FS; ++j) zv[a * FS + j] = TB[nbn4[a][j] / ES];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int j = 0; j < FS; ++j)
        FR[(valid && sg[a] != 0) ? frb[a] + fst + j : frn] = zv[a * FS + j];

    cb = ncb;
    ce = nce;
    lev = nlev2;
    ncb = nncb;
    nce = nnce;
    nlev2 = nlev3;
    dc = dn;
  };
  while (lev < nlev) {
    tile(dA, dB, pcA, pcB);
    if (lev >= nlev) break;
    tile(dB, dA, pcB, pcA);
  }
}

// waves per SIMD the register budget aims at: with the 27-node cell every
// form needs more than a quarter of the register file (the operator slice,
// two sets of prefetched cell values; the split forms hold hi / lo halves):
// three waves without spills measured as fast as four with them.  FP64
// takes two registers per value: two waves
template <typename T, int MODE, int DIM, int P>
constexpr int wave_occupancy() {
  return WaveShape<DIM, P>::NN > 32 ? 1 : (sizeof(T) == 8 ? 2 : (WaveShape<DIM, P>::NN > 16 ? 3 : 4));
}

// One task (velocity, subdomain, component) of one problem: the body of the
// single-problem and the batched kernels.
template <typename T, int MODE, int DIM, int P>
__device__ __forceinline__ void front_wave_block(
    const T* __restrict__ f_old, const T* __restrict__ f_prev, T* __restrict__ f_cur,
    const Geom& g, const FrontParams& fp, const T* __restrict__ Wop,
    const int* __restrict__ lvl_start, const int4* __restrict__ desc, int n_desc,
    const BndRef<T>& bd, int task, T* wave_lds) {
  using S = WaveShape<DIM, P>;
  const int m = g.m, nn = S::NN;
  const int nsd = fp.nsub[0] * fp.nsub[1] * fp.nsub[2];
  const int c = task % m;
  const int sd = (task / m) % nsd;
  const int k = task / (m * nsd);
  T* FR = wave_lds;                                    // [3][fr_pos][FSTR], then the sink
  T* XO = FR + 3 * fp.fr_pos * S::FSTR + 4;            // [16][XOS]

  int sg[3], sdc[3], nbrel[3], isb[3], boff[3];
  sdc[0] = sd % fp.nsub[0];
  sdc[1] = (sd / fp.nsub[0]) % fp.nsub[1];
  sdc[2] = sd / (fp.nsub[0] * fp.nsub[1]);
  bool any_bnd = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sg[a] = a < DIM ? fp.sg[k][a] : 0;
    nbrel[a] = 0;
    isb[a] = 0;
    boff[a] = 0;
    if (sg[a] == 0) continue;
    // the upwind neighbour of the subdomain's first cells along a: across an
    // interface (iterate p-1), across the periodic wrap, or a Dirichlet box face
    const int Sa = g.S[a], Na = g.N[a];
    const int ga = sdc[a] * Sa + (sg[a] > 0 ? 0 : Sa - 1);
    int nb = ga - sg[a];
    const int64_t bo = bd.old != nullptr ? bd.off[a][sg[a] > 0 ? 0 : 1] : -1;
    if ((nb < 0 || nb >= Na) && bo >= 0) {
      isb[a] = 1;
      boff[a] = (int)bo;
      any_bnd = true;
      continue;
    }
    if (nb < 0) nb += Na;
    if (nb >= Na) nb -= Na;
    const int stride = a == 0 ? 1 : (a == 1 ? g.N[0] : g.N[0] * g.N[1]);
    nbrel[a] = (nb - ga) * stride * nn;
  }
  const int64_t plane = g.ncell * nn;
  const int64_t pc = (int64_t)k * m + c;
  const unsigned sdb = (unsigned)((sdc[0] * g.S[0] +
                                   (int64_t)g.N[0] * (sdc[1] * g.S[1] + (int64_t)g.N[1] * sdc[2] * g.S[2])) *
                                  nn);
  const __amdgpu_buffer_rsrc_t rfo = wave_rsrc(f_old + pc * plane, plane * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rfp = wave_rsrc(f_prev + pc * plane, plane * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rfc = wave_rsrc(f_cur + pc * plane, plane * (int64_t)sizeof(T));
  const T* Wk = Wop + (int64_t)k * nn * fp.Kd;
  if (any_bnd) {
    const __amdgpu_buffer_rsrc_t rbo = wave_rsrc(bd.old + pc * bd.nb, bd.nb * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rbn = wave_rsrc(bd.neu + pc * bd.nb, bd.nb * (int64_t)sizeof(T));
    front_wave_task<T, MODE, DIM, P, true>(g, fp, Wk, lvl_start, desc, n_desc, k, sg, sdc, nbrel, isb,
                                        boff, sdb, rfo, rfp, rfc, rbo, rbn, FR, XO);
  } else {
    front_wave_task<T, MODE, DIM, P, false>(g, fp, Wk, lvl_start, desc, n_desc, k, sg, sdc, nbrel,
                                         isb, boff, sdb, rfo, rfp, rfc, rfo, rfp, FR, XO);
  }
}

template <typename T, int MODE, int DIM, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(wave_occupancy<T, MODE, DIM, P>())))
void k_sweep_front_wave(
    const T* __restrict__ f_old, const T* __restrict__ f_prev, T* __restrict__ f_cur,
    Geom g, FrontParams fp, const T* __restrict__ Wop, const int* __restrict__ lvl_start,
    const int4* __restrict__ desc, int n_desc, BndRef<T> bd) {
  extern __shared__ double wave_lds_d[];  // (8-byte aligned; FP32 values use it as floats)
  front_wave_block<T, MODE, DIM, P>(f_old, f_prev, f_cur, g, fp, Wop, lvl_start, desc, n_desc, bd,
                                    (int)blockIdx.x, reinterpret_cast<T*>(wave_lds_d));
}

// Many problems of one (form, dimension, degree) in one launch, one
// subdomain iteration each: the tasks of all problems are numbered
// consecutively (start[] prefix over the problems).
template <typename T, int MODE, int DIM, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(wave_occupancy<T, MODE, DIM, P>())))
void k_sweep_front_wave_batch(const FrontWaveTask<T>* __restrict__ tasks,
                              const int64_t* __restrict__ start, int ntask) {
  extern __shared__ double wave_lds_b[];  // (8-byte aligned; FP32 values use it as floats)
  const int64_t gb = blockIdx.x;
  int pid = 0;
  while (pid + 1 < ntask && gb >= start[pid + 1]) ++pid;
  const FrontWaveTask<T>& t = tasks[pid];
  front_wave_block<T, MODE, DIM, P>(t.f_old, t.f_prev, t.f_cur, t.g, t.fp, t.Wop, t.lvl_start,
                                    t.desc, t.n_desc, t.bd, (int)(gb - start[pid]),
                                    reinterpret_cast<T*>(wave_lds_b));
}

// the (dim, nodes per axis) shapes the kernel is built for: 0..5, or -1
// (5: 64-node cells, the FP32 forms only)
int front_wave_shape(const Geom& g) {
  if (g.dim == 3 && g.P == 2) return 0;
  if (g.dim == 3 && g.P == 3) return 1;
  if (g.dim == 2 && g.P == 2) return 2;
  if (g.dim == 2 && g.P == 3) return 3;
  if (g.dim == 2 && g.P == 4) return 4;
  if (g.dim == 3 && g.P == 4) return 5;
  return -1;
}

template <int DIM, int P>
size_t wave_lds_size(const FrontParams& fp) {
  using S = WaveShape<DIM, P>;
  return (3 * (size_t)fp.fr_pos * S::FSTR + 4 + 16 * (size_t)S::XOS) * sizeof(float);
}

}  // namespace

size_t front_wave_lds_bytes(const Geom& g, const FrontParams& fp, int prec) {
  const size_t es = prec == KDS_FP64 ? 2 : 1;  // the sizes below count FP32 values
  switch (front_wave_shape(g)) {
    case 0: return es * wave_lds_size<3, 2>(fp);
    case 1: return es * wave_lds_size<3, 3>(fp);
    case 2: return es * wave_lds_size<2, 2>(fp);
    case 3: return es * wave_lds_size<2, 3>(fp);
    case 4: return es * wave_lds_size<2, 4>(fp);
    case 5: return es * wave_lds_size<3, 4>(fp);
    default: return 0;
  }
}

bool front_wave_fits(int prec, int mode, const Geom& g, const FrontParams& fp, int64_t nb) {
  // FP32: the matrix-core forms; FP64: the FP64 matrix cores, for the FMA mode
  const bool f32 = prec == KDS_FP32 && mode != kFrontFma;
  const bool f64 = prec == KDS_FP64 && mode == kFrontFma && front_wave_shape(g) != 5;
  const int64_t plane = g.ncell * g.nn, es = f64 ? 8 : 4;
  return (f32 || f64) && front_wave_shape(g) >= 0 && fp.Kd == g.nn + 3 * fp.nf &&
         plane * es < ((int64_t)1 << 31) && nb * es < ((int64_t)1 << 31) && fp.fr_pos > 0 &&
         front_wave_lds_bytes(g, fp, prec) <= 64 * 1024;
}

hipError_t launch_sweep_front_wave(int prec, int mode, const Geom& g, const FrontParams& fp,
                                   const void* Wop, const int* lvl_start, const int4* desc,
                                   int n_desc, const void* f_old, const void* f_prev, void* f_cur,
                                   const BndArgs& bnd, hipStream_t s) {
  if (!front_wave_fits(prec, mode, g, fp, bnd.nb) || n_desc <= 0) return hipErrorInvalidValue;
  const int nsd = fp.nsub[0] * fp.nsub[1] * fp.nsub[2];
  const dim3 grid((unsigned)(nsd * g.nv * g.m)), block(64);
  const size_t lds = front_wave_lds_bytes(g, fp, prec);
  const int shape = front_wave_shape(g);
  if (prec == KDS_FP64) {
    const double* dfo = (const double*)f_old;
    const double* dfp = (const double*)f_prev;
    double* dfc = (double*)f_cur;
    const double* dW = (const double*)Wop;
    const BndRef<double> dbd = bnd_ref<double>(bnd);
#define KDS_WAVE64(DIM, P)                                                                    \
  hipLaunchKernelGGL((k_sweep_front_wave<double, kFrontMfma, DIM, P>), grid, block, lds, s, dfo, \
                     dfp, dfc, g, fp, dW, lvl_start, desc, n_desc, dbd)
    switch (shape) {
      case 0: KDS_WAVE64(3, 2); break;
      case 1: KDS_WAVE64(3, 3); break;
      case 2: KDS_WAVE64(2, 2); break;
      case 3: KDS_WAVE64(2, 3); break;
      case 4: KDS_WAVE64(2, 4); break;
      default: return hipErrorInvalidValue;
    }
#undef KDS_WAVE64
    return hipGetLastError();
  }
  const float* fo = (const float*)f_old;
  const float* fpv = (const float*)f_prev;
  float* fc = (float*)f_cur;
  const float* W = (const float*)Wop;
  const BndRef<float> bd = bnd_ref<float>(bnd);
#define KDS_WAVE_LAUNCH(MODE, DIM, P)                                                            \
  hipLaunchKernelGGL((k_sweep_front_wave<float, MODE, DIM, P>), grid, block, lds, s, fo, fpv, fc, g, fp, \
                     W, lvl_start, desc, n_desc, bd)
#define KDS_WAVE(MODE)                              \
  switch (shape) {                                  \
    case 0: KDS_WAVE_LAUNCH(MODE, 3, 2); break;     \
    case 1: KDS_WAVE_LAUNCH(MODE, 3, 3); break;     \
    case 2: KDS_WAVE_LAUNCH(MODE, 2, 2); break;     \
    case 3: KDS_WAVE_LAUNCH(MODE, 2, 3); break;     \
    case 4: KDS_WAVE_LAUNCH(MODE, 2, 4); break;     \
    default: KDS_WAVE_LAUNCH(MODE, 3, 4); break;    \
  }
  switch (mode) {
    case kFrontMfma:
      KDS_WAVE(kFrontMfma)
      break;
    case kFrontSplitF16:
      KDS_WAVE(kFrontSplitF16)
      break;
    case kFrontSplitBf16:
      KDS_WAVE(kFrontSplitBf16)
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef KDS_WAVE
#undef KDS_WAVE_LAUNCH
  return hipGetLastError();
}

size_t front_wave_task_bytes(int prec) {
  return prec == KDS_FP64 ? sizeof(FrontWaveTask<double>) : sizeof(FrontWaveTask<float>);
}

namespace {
template <typename T>
void pack_front_wave_task_t(const Geom& g, const FrontParams& fp, const void* Wop,
                            const int* lvl_start, const int4* desc, int n_desc, const void* f_old,
                            const void* f_prev, void* f_cur, const BndArgs& bnd, void* out) {
  FrontWaveTask<T> t;
  t.f_old = (const T*)f_old;
  t.f_prev = (const T*)f_prev;
  t.f_cur = (T*)f_cur;
  t.g = g;
  t.fp = fp;
  t.Wop = (const T*)Wop;
  t.lvl_start = lvl_start;
  t.desc = desc;
  t.n_desc = n_desc;
  t.bd = bnd_ref<T>(bnd);
  std::memcpy(out, &t, sizeof(t));
}
}  // namespace

void pack_front_wave_task(int prec, const Geom& g, const FrontParams& fp, const void* Wop,
                          const int* lvl_start, const int4* desc, int n_desc, const void* f_old,
                          const void* f_prev, void* f_cur, const BndArgs& bnd, void* out) {
  if (prec == KDS_FP64)
    pack_front_wave_task_t<double>(g, fp, Wop, lvl_start, desc, n_desc, f_old, f_prev, f_cur, bnd,
                                   out);
  else
    pack_front_wave_task_t<float>(g, fp, Wop, lvl_start, desc, n_desc, f_old, f_prev, f_cur, bnd,
                                  out);
}

int64_t front_wave_blocks(const Geom& g, const FrontParams& fp) {
  return (int64_t)fp.nsub[0] * fp.nsub[1] * fp.nsub[2] * g.nv * g.m;
}

hipError_t launch_sweep_front_wave_batch(int prec, int mode, const Geom& g, const void* tasks,
                                         const int64_t* start, int ntask, int64_t nblocks,
                                         size_t lds_bytes, hipStream_t s) {
  const int shape = front_wave_shape(g);
  if (shape < 0 || ntask <= 0 || nblocks <= 0 || nblocks > 0x7fffffffLL || lds_bytes > 64 * 1024)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks), block(64);
  if (prec == KDS_FP64) {
    if (mode != kFrontFma) return hipErrorInvalidValue;
    const FrontWaveTask<double>* tk = (const FrontWaveTask<double>*)tasks;
#define KDS_WAVEB64(DIM, P)                                                                   \
  hipLaunchKernelGGL((k_sweep_front_wave_batch<double, kFrontMfma, DIM, P>), grid, block,       \
                     lds_bytes, s, tk, start, ntask)
    switch (shape) {
      case 0: KDS_WAVEB64(3, 2); break;
      case 1: KDS_WAVEB64(3, 3); break;
      case 2: KDS_WAVEB64(2, 2); break;
      case 3: KDS_WAVEB64(2, 3); break;
      case 4: KDS_WAVEB64(2, 4); break;
      default: return hipErrorInvalidValue;
    }
#undef KDS_WAVEB64
    return hipGetLastError();
  }
  const FrontWaveTask<float>* tk = (const FrontWaveTask<float>*)tasks;
#define KDS_WAVEB_LAUNCH(MODE, DIM, P)                                                            \
  hipLaunchKernelGGL((k_sweep_front_wave_batch<float, MODE, DIM, P>), grid, block, lds_bytes, s, tk, \
                     start, ntask)
#define KDS_WAVEB(MODE)                             \
  switch (shape) {                                  \
    case 0: KDS_WAVEB_LAUNCH(MODE, 3, 2); break;    \
    case 1: KDS_WAVEB_LAUNCH(MODE, 3, 3); break;    \
    case 2: KDS_WAVEB_LAUNCH(MODE, 2, 2); break;    \
    case 3: KDS_WAVEB_LAUNCH(MODE, 2, 3); break;    \
    case 4: KDS_WAVEB_LAUNCH(MODE, 2, 4); break;    \
    default: KDS_WAVEB_LAUNCH(MODE, 3, 4); break;   \
  }
  switch (mode) {
    case kFrontMfma:
      KDS_WAVEB(kFrontMfma)
      break;
    case kFrontSplitF16:
      KDS_WAVEB(kFrontSplitF16)
      break;
    case kFrontSplitBf16:
      KDS_WAVEB(kFrontSplitBf16)
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef KDS_WAVEB
#undef KDS_WAVEB_LAUNCH
  return hipGetLastError();
}

}  // namespace kds
