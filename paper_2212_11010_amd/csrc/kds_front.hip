// kds_front.hip -- the front schedule (velocities in any direction): the
// solves of one anti-diagonal front of a subdomain as one dense GEMM.
#include "kds_device.h"

namespace kds {

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
constexpr int kFrontMaxKpad = 112;  // operator columns nn + 3 nf (p = 3, d = 3), padded to 16

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

// KP: upper bound of the padded operator width Kpad (64 covers p <= 2 in 3-D,
// kFrontMaxKpad the rest), sizing the register-resident operator slice.
template <typename T, int MODE, int KP>
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
  T* X = reinterpret_cast<T*>(smem_raw);  // [Kpad][XS]
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
  // rows Kd..Kpad-1 of X stay zero (padding of the K dimension)
  for (int e = tid; e < Kpad * XS; e += bs) X[e] = T(0);

  // Matrix-core modes: a wave always computes the same 16-row tile of Y
  // (4 waves, Mpad / 16 in {1, 2, 4} row tiles), so its slice of the
  // operator W stays in registers for the whole kernel: per K step of the
  // 16x16x4 FP32 product one value, per step of the 16x16x16 split products
  // four values as hi / lo halves.
  const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt_n = Mpad / 16;
  const int i0 = (wave % mt_n) * 16;
  constexpr int KS4 = KP / 4, KS16 = KP / 16;
  float afr[MODE == kFrontMfma ? KS4 : 1];
  kds_f16x4 ah16[MODE == kFrontSplitF16 ? KS16 : 1], al16[MODE == kFrontSplitF16 ? KS16 : 1];
  kds_i16x4 ahb[MODE == kFrontSplitBf16 ? KS16 : 1], alb[MODE == kFrontSplitBf16 ? KS16 : 1];
  auto wval = [&](int i, int r) -> float {
    return (i < nn && r < Kd) ? (float)Wk[i * Kd + r] : 0.0f;
  };
  if constexpr (MODE == kFrontMfma) {
#pragma unroll
    for (int st = 0; st < KS4; ++st) afr[st] = 4 * st < Kpad ? wval(i0 + li, 4 * st + lk) : 0.0f;
  } else if constexpr (MODE == kFrontSplitF16) {
#pragma unroll
    for (int st = 0; st < KS16; ++st)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float w = 16 * st < Kpad ? wval(i0 + li, 16 * st + 4 * lk + u) : 0.0f;
        const _Float16 h = (_Float16)w;
        ah16[st][u] = h;
        al16[st][u] = (_Float16)((w - (float)h) * 2048.0f);
      }
  } else if constexpr (MODE == kFrontSplitBf16) {
#pragma unroll
    for (int st = 0; st < KS16; ++st)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float w = 16 * st < Kpad ? wval(i0 + li, 16 * st + 4 * lk + u) : 0.0f;
        const unsigned short h = bf16_rne(w);
        ahb[st][u] = (short)h;
        alb[st][u] = (short)bf16_rne(w - bf16_to_f32(h));
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

  // Gather: thread tid owns row r = tid % Kpad of X (a node of the cell, or
  // a node of one inflow face) for the whole kernel, and the columns
  // jr, jr + rstep, ...; everything about its row is decoded once.
  const int rstep = bs / Kpad;
  const int r = tid % Kpad, jr = tid / Kpad;
  const bool row_on = jr < rstep;
  const bool row_cell = r < nn;
  const int row_face = (row_cell || r >= Kd) ? -1 : (r - nn) / nf;
  const int row_q = row_face >= 0 ? r - nn - row_face * nf : 0;
  const int row_node = row_face >= 0 ? face_node[r - nn] : 0;

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
      // ---- gather X[r][jj]: U independent loads per thread in flight
      if (row_on) {
        constexpr int U = 4;
        for (int jb0 = jr; jb0 < CH; jb0 += U * rstep) {
          T vo[U], vn[U];
          int kind[U];  // -2: zero, -1: cell node, else the inflow face
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int jj = jb0 + u * rstep;
            int64_t at = 0;
            int kd = -2;
            const T* po = f_old;
            const T* pn = f_prev;
            if (jj < nc && r < Kd) {
              if (row_cell) {
                at = col_base[jj] + r;
                kd = -1;
              } else {
                const int64_t nbo = col_nb[row_face][jj];
                if (nbo >= 0) {
                  const int ci = col_int[row_face][jj];
                  // boundary values are numbered by face node (row q of the face)
                  at = nbo + (ci == 2 ? row_q : row_node);
                  kd = row_face;
                  if (ci == 2) {
                    po = bd.old;
                    pn = bd.neu;
                  } else if (ci == 1) {
                    pn = f_cur;
                  }
                }
              }
            }
            kind[u] = kd;
            // inactive slots re-read element 0 of the state (never used)
            vo[u] = po[at];
            vn[u] = pn[kd >= 0 ? at : 0];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int jj = jb0 + u * rstep;
            if (jj < CH) {
              T v = T(0);
              if (kind[u] == -1) v = vo[u];
              else if (kind[u] >= 0) v = th * vn[u] + (T(1) - th) * vo[u];
              X[r * XS + jj] = v;
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
        const int nt_n = (nc + 15) / 16;
        for (int t = wave; t < mt_n * nt_n; t += nw) {
          const int jb = (t / mt_n) * 16;  // (t % mt_n = wave % mt_n: this wave's row tile)
          kds_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          if constexpr (MODE == kFrontMfma) {
#pragma unroll
            for (int st = 0; st < KS4; ++st)
              if (4 * st < Kpad)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[st], (float)X[(4 * st + lk) * XS + jb + li],
                                                           acc, 0, 0, 0);
          } else {
            kds_f32x4 cor = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < KS16; ++st) {
              if (16 * st >= Kpad) continue;
              float bw[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) bw[u] = (float)X[(16 * st + 4 * lk + u) * XS + jb + li];
              if constexpr (MODE == kFrontSplitF16) {
                kds_f16x4 bh, bl;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const _Float16 hb = (_Float16)bw[u];
                  bh[u] = hb;
                  bl[u] = (_Float16)((bw[u] - (float)hb) * 2048.0f);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah16[st], bh, acc, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16f16(ah16[st], bl, cor, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16f16(al16[st], bh, cor, 0, 0, 0);
              } else {
                kds_i16x4 bh, bl;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const unsigned short hb = bf16_rne(bw[u]);
                  bh[u] = (short)hb;
                  bl[u] = (short)bf16_rne(bw[u] - bf16_to_f32(hb));
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahb[st], bh, acc, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahb[st], bl, cor, 0, 0, 0);
                cor = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alb[st], bh, cor, 0, 0, 0);
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

size_t front_lds_bytes(int prec, int mode, const Geom& g, const FrontParams& fp) {
  const int Mpad = (g.nn + 15) & ~15, Kpad = (fp.Kd + 15) & ~15;
  const size_t el = prec == KDS_FP64 ? 8 : 4;
  (void)mode;
  (void)Mpad;
  return (size_t)Kpad * (fp.col_chunk + 1) * el;
}

hipError_t launch_sweep_front(int prec, int mode, const Geom& g, const FrontParams& fp,
                              const void* Wop, const int* lvl_start, const int* lvl_cells,
                              const void* f_old, const void* f_prev, void* f_cur,
                              const BndArgs& bnd, hipStream_t s) {
  const int nsd = fp.nsub[0] * fp.nsub[1] * fp.nsub[2];
  const dim3 grid((unsigned)(nsd * g.nv)), block(256);
  const size_t lds = front_lds_bytes(prec, mode, g, fp);
  const int Kpad = (fp.Kd + 15) & ~15;
  if (Kpad > kFrontMaxKpad) return hipErrorInvalidValue;
  if (prec == KDS_FP64) {
    if (mode != kFrontFma) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep_front<double, kFrontFma, kFrontMaxKpad>), grid, block, lds, s, (const double*)f_old,
                       (const double*)f_prev, (double*)f_cur, g, fp, (const double*)Wop, lvl_start,
                       lvl_cells, bnd_ref<double>(bnd));
  } else {
    switch (mode) {
#define KDS_FRONT(MODE)                                                                         \
  case MODE:                                                                                    \
    if (Kpad <= 64)                                                                             \
      hipLaunchKernelGGL((k_sweep_front<float, MODE, 64>), grid, block, lds, s, (const float*)f_old, \
                         (const float*)f_prev, (float*)f_cur, g, fp, (const float*)Wop, lvl_start, \
                         lvl_cells, bnd_ref<float>(bnd));                                       \
    else                                                                                        \
      hipLaunchKernelGGL((k_sweep_front<float, MODE, kFrontMaxKpad>), grid, block, lds, s,       \
                         (const float*)f_old, (const float*)f_prev, (float*)f_cur, g, fp,       \
                         (const float*)Wop, lvl_start, lvl_cells, bnd_ref<float>(bnd));         \
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


}  // namespace kds
