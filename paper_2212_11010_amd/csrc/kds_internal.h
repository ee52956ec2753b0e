// kds_internal.h -- private declarations shared by the host setup, the
// kernels and the C ABI of libkds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kds.h"

namespace kds {

constexpr int kMaxVel = 8;   // kinetic velocities
constexpr int kMaxP = 4;     // nodes per axis (degree <= 3)
constexpr int kMaxM = 8;     // conserved components
constexpr int kMaxQ = 8;     // cells per lane in the line schedule, in registers
constexpr int kMaxRoundQ = 64;  // cells per lane streamed through the LDS tile in rounds
                                // (lines longer than 64 lanes x the register budget)
constexpr int kXcds = 8;     // accelerator complex dies of an MI355X (own L2 each)

// ---------------------------------------------------------------- host setup

// 1-D nodal DG data on the reference cell [0, 1] (Gauss-Lobatto points).
struct Basis1D {
  int P = 0;                 // nodes per axis
  std::vector<double> xi, w; // nodes, weights (sum 1)
  std::vector<double> D;     // D[b*P + a] = l_a'(xi_b)
};
Basis1D make_basis(int degree);

// Local (downwind-ordered) 1-D cell update for one velocity along an axis:
//   f^n = C f^{n-1} + e ((1 - theta) t^{n-1} + theta t^n)
// where t is the upwind neighbour's outflow node value (node P-1 of the
// neighbour in downwind order) and node 0 is the inflow node.
struct LineOp {
  int P = 0;
  double nu = 0;              // |V| dt / h
  std::vector<double> C;      // P x P, row-major
  std::vector<double> e;      // P
};
LineOp make_line_op(const Basis1D& b, double nu, double theta);

// Dense cell operator [C | E_0 | E_1 | E_2] (nn x (nn + 3 nf)) of the implicit
// upwind DG cell update for a velocity in any direction.
bool make_dense_op(const Basis1D& b, int dim, const double* V, const double* h, double dt,
                   double theta, std::vector<double>& Wop, int& nn, int& nf);

// Minimum-norm equilibrium weights (a_k, b_{k,i}) or the caller's.
bool eq_weights(int dim, int nv, const double* vel, const double* eq_a, const double* eq_b,
                std::vector<double>& a, std::vector<double>& b, std::string& err);

// Eigenvalues of a symmetric n x n matrix (row-major), Jacobi rotations.
void sym_eigenvalues(int n, std::vector<double> A, std::vector<double>& ev);

// Stability checks of a linear law's kinetic model: largest wave speed
// max_i rho(A^i) and smallest eigenvalue of the equilibrium derivatives
// a_k I + sum_i b_{k,i} A^i (checked only for symmetric A^i).
struct EqChecks {
  bool checked = false;
  double wave_speed = 0.0;
  double min_eig = 0.0;
};
EqChecks check_linear_law(int dim, int m, int nv, const std::vector<double>& A,
                          const std::vector<double>& a, const std::vector<double>& b);

// ------------------------------------------------------- device parameters

struct Geom {
  int dim;
  int N[3];
  int S[3];
  int P;
  int nn;      // P^dim
  int64_t ncell;
  int m;
  int nv;
  int K;       // subdomain iterations
  int64_t tr_stride;  // plain schedule: trace entries per (velocity, component)
};

template <typename T>
struct SweepTab {
  int axis[kMaxVel];
  int sign[kMaxVel];
  T C[kMaxVel][kMaxP * kMaxP];
  T e1[kMaxVel][kMaxP];   // (1 - theta) e
  T eth[kMaxVel][kMaxP];  // theta e
};

template <int D, int M, int NV>
struct EqTab {
  double A[D][M][M];  // linear law
  double a[NV];
  double b[NV][D];
  double omega;
  double gamma;       // Euler
  double mu[M];       // Crank-Nicolson source factors W+_c = mu_c W_c
  int has_source;
};

// Cells of 64 nodes (p = 3 in 3-D) are solved one group of node lines at a
// time from the LDS tile (16 values per cell in registers).
__host__ __device__ constexpr bool line_grouped(int nn) { return nn > 27; }

// Grouped mode streams two groups of four node lines (32 values per cell)
// through the LDS tile at a time; cells sit kGroupStride values apart there.
constexpr int kGroupStride = 36;

// LDS values per column of Na cells in the line kernel's tile.
__host__ __device__ constexpr int line_col_lds(int Na, int nn) {
  return line_grouped(nn) ? Na * kGroupStride : Na * nn;
}

// State values per cell a lane holds in registers at once.
__host__ __device__ constexpr int line_cell_values(int nn) { return line_grouped(nn) ? 16 : nn; }

// Most cells per lane the line kernel keeps in registers (a budget of 64
// state values per lane; 2 cells in grouped mode, whose copy passes need the
// registers more than the solve needs long lane blocks).
__host__ __device__ constexpr int line_qmax(int elem_bytes, int nn) {
  return (void)elem_bytes, line_grouped(nn) ? 2
         : 64 / line_cell_values(nn) >= 8 ? 8 : 64 / line_cell_values(nn) >= 4 ? 4 : 2;
}

// Line-schedule launch plan (per velocity).
struct LinePlan {
  int Q[kMaxVel];          // cells per lane (above line_qmax: rounds through the tile)
  int lpl2[kMaxVel];       // lanes per line, power of two
  int bw[kMaxVel];         // columns of cells per bundle
  int64_t block_start[kMaxVel * kMaxM + 1];  // prefix over (k, c) of bundles
  int lds_elems;           // max tile elements
  int lds_alloc;           // elements of LDS allocated per workgroup (>= lds_elems; more
                           // limits how many workgroups share a CU)
  int threads;             // block size
  int xdirect;             // x lines may bypass the LDS tile (cells per lane = QMAX)
};

// Some velocity's lanes own more cells than the registers hold (their cells
// go through the LDS tile in rounds; a kernel instantiation of its own).
inline bool line_plan_rounds(const Geom& g, const LinePlan& pl, int elem_bytes) {
  const int qmax = line_qmax(elem_bytes, g.nn);
  for (int k = 0; k < g.nv; ++k)
    if (pl.Q[k] > qmax) return true;
  return false;
}

// Dirichlet inflow data of the faces of non-periodic axes: kinetic values
// M_k(W_b) at the boundary nodes, [k][c][boundary node], at the start (old)
// and the end (neu) of the step.  Boundary nodes: faces of the non-periodic
// axes in x, y, z order, low end then high end; on a face, cells over the
// other axes, then face nodes over the other axes' node indices (lower axis
// fastest).
struct BndArgs {
  const void* old = nullptr;  // nullptr: periodic on every axis
  const void* neu = nullptr;
  int64_t nb = 0;             // boundary nodes
  int64_t off[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};  // first node of face (axis, side)
};

template <typename T>
struct BndRef {
  const T* old;
  const T* neu;
  int64_t nb;
  int64_t off[3][2];
};

template <typename T>
inline BndRef<T> bnd_ref(const BndArgs& b) {
  BndRef<T> r;
  r.old = (const T*)b.old;
  r.neu = (const T*)b.neu;
  r.nb = b.nb;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) r.off[a][s] = b.off[a][s];
  return r;
}

// One problem of a batched line-sweep launch.
template <typename T>
struct LineTask {
  T* f;
  Geom g;
  SweepTab<T> tab;
  LinePlan pl;
  BndRef<T> bd;
};

// One problem of a batched relaxation launch (pointwise kernel).
template <int D, int M, int NV>
struct RelaxTask {
  const void* fin;
  void* fout;
  int64_t plane;
  EqTab<D, M, NV> t;
};

// Front (level-ordered) sweep for velocities in any direction.
enum FrontMode { kFrontFma = 0, kFrontMfma = 1, kFrontSplitF16 = 2, kFrontSplitBf16 = 3 };

struct FrontParams {
  int nf;                  // nodes per face, (p+1)^(d-1)
  int Kd;                  // operator columns, nn + 3 nf
  int sg[kMaxVel][3];      // sign of V^a, 0 where V^a = 0
  int lvl_off[kMaxVel];    // offset of the velocity's level starts in lvl_start
  int nlev[kMaxVel];       // number of levels (fronts) per subdomain
  int col_chunk;           // GEMM columns per pass (multiple of 16)
  int nsub[3];             // subdomains per axis
  int fr_pos;              // wave kernel: frontier slots per axis, the largest
                           // product of two subdomain widths
  double theta;
};

// --------------------------------------------------------------- launchers


hipError_t launch_init(int prec, int law, const Geom& g, const void* eq, const double* W,
                       void* f, hipStream_t s);
// eq_dev: a device copy of the equilibrium table (the blob of build_eq_blob);
// vec: VW consecutive nodes per thread with 16-byte accesses where the node
// count allows (same arithmetic)
hipError_t launch_relax(int prec, int law, const Geom& g, const void* eq_dev, const void* fin,
                        void* fout, bool vec, hipStream_t s);
hipError_t launch_moments(int prec, const Geom& g, const void* f, double* W, hipStream_t s);
// W = sum_k f_k at nodes i0 .. i0 + n - 1 into W[(i - i0) m + r]
hipError_t launch_moments_range(int prec, const Geom& g, const void* f, int64_t i0, int64_t n,
                                double* W, hipStream_t s);

// Size of the static device scratch array (one per GPU) used by the entry
// points that allocate nothing, and its device address on the current device
// (looked up once per device).
constexpr size_t kScratchBytes = size_t(32) << 20;
hipError_t scratch_address(void** out);
hipError_t launch_get_kinetic(int prec, const Geom& g, const void* f, double* F, hipStream_t s);
hipError_t launch_set_kinetic(int prec, const Geom& g, const double* F, void* f, hipStream_t s);
hipError_t launch_check_finite(int prec, const Geom& g, const void* f, int* flag, hipStream_t s);
// Largest |u_i| + c of an Euler state W [node][d + 2] (FP64, device), as the
// bits of a double max-reduced into *out (which the caller zeroes).
hipError_t launch_euler_wave_speed(const double* W, int64_t nodes, int dim, double gamma,
                                   unsigned long long* out, hipStream_t s);
hipError_t launch_sweep_plain(int prec, const Geom& g, const void* tab, const void* f_old,
                              void* f_new, const void* tr_prev, void* tr_out, const BndArgs& bnd,
                              hipStream_t s);
hipError_t launch_sweep_line(int prec, const Geom& g, const void* tab, const LinePlan& plan,
                             void* f, const BndArgs& bnd, hipStream_t s);
hipError_t launch_copy(int prec, const void* src, void* dst, int64_t n, hipStream_t s);
// One subdomain iteration of the front sweep: reads f_old (state at t^{n-1})
// and f_prev (iterate p-1), writes f_cur (iterate p).  mode: FrontMode; for
// kFrontFma the element type follows prec (FP64 or FP32), the MFMA modes are FP32.
hipError_t launch_sweep_front(int prec, int mode, const Geom& g, const FrontParams& fp,
                              const void* Wop, const int* lvl_start, const int* lvl_cells,
                              const void* f_old, const void* f_prev, void* f_cur,
                              const BndArgs& bnd, hipStream_t s);
size_t front_lds_bytes(int prec, int mode, const Geom& g, const FrontParams& fp);
// The wave-per-task form of the same sweep (FP32 matrix-core modes for cells
// of up to 64 nodes, and the FMA mode in FP64 on the FP64 matrix cores for
// cells of up to 32 nodes).  desc: per cell in front order (the
// order of lvl_cells) {element offset of the cell inside its subdomain,
// downwind local coordinates lx | ly << 10 | lz << 20, frontier position on
// axis 0 | on axis 1 << 16, on axis 2}; n_desc entries.  nb: boundary nodes.
bool front_wave_fits(int prec, int mode, const Geom& g, const FrontParams& fp, int64_t nb);
size_t front_wave_lds_bytes(const Geom& g, const FrontParams& fp, int prec = KDS_FP32);
hipError_t launch_sweep_front_wave(int prec, int mode, const Geom& g, const FrontParams& fp,
                                   const void* Wop, const int* lvl_start, const int4* desc,
                                   int n_desc, const void* f_old, const void* f_prev, void* f_cur,
                                   const BndArgs& bnd, hipStream_t s);
// The same for many problems of one (precision, form, dimension, degree)
// and one subdomain iteration each: a task record per problem (the arguments
// above), start[] the prefix over the problems of front_wave_blocks,
// lds_bytes the largest front_wave_lds_bytes of the problems.
size_t front_wave_task_bytes(int prec);
void pack_front_wave_task(int prec, const Geom& g, const FrontParams& fp, const void* Wop,
                          const int* lvl_start, const int4* desc, int n_desc, const void* f_old,
                          const void* f_prev, void* f_cur, const BndArgs& bnd, void* out);
int64_t front_wave_blocks(const Geom& g, const FrontParams& fp);
hipError_t launch_sweep_front_wave_batch(int prec, int mode, const Geom& g, const void* tasks,
                                         const int64_t* start, int ntask, int64_t nblocks,
                                         size_t lds_bytes, hipStream_t s);

// Batched launches (many problems per kernel): task records are packed on the
// host, copied to device memory, and the kernels find their problem from the
// prefix start[] over the problems' work items.
size_t relax_task_bytes(int law, int dim, int m, int nv);
bool pack_relax_task(int law, int dim, int m, int nv, const void* eq, const void* fin, void* fout,
                     int64_t plane, void* out);
hipError_t launch_relax_batch(int prec, int law, int dim, int m, int nv, const void* tasks,
                              const int64_t* start, int ntask, int64_t nblocks, hipStream_t s);
hipError_t line_kernels_allow_lds(size_t bytes);
// per element type (kds_line_f32.hip, kds_line_f64.hip)
hipError_t sweep_line_f32(const Geom& g, const void* tab, const LinePlan& plan, void* f,
                          const BndArgs& bnd, hipStream_t s);
hipError_t sweep_line_f64(const Geom& g, const void* tab, const LinePlan& plan, void* f,
                          const BndArgs& bnd, hipStream_t s);
hipError_t sweep_line_batch_f32(int P, int dim, bool rounds, bool dir, const void* tasks,
                                const int64_t* start, int ntask, int64_t nblocks, int threads,
                                size_t lds_elems, hipStream_t s);
hipError_t sweep_line_batch_f64(int P, int dim, bool rounds, bool dir, const void* tasks,
                                const int64_t* start, int ntask, int64_t nblocks, int threads,
                                size_t lds_elems, hipStream_t s);
hipError_t line_allow_lds_f32(size_t bytes);
hipError_t line_allow_lds_f64(size_t bytes);
size_t line_task_bytes_f32();
size_t line_task_bytes_f64();
void pack_line_task_f32(void* f, const Geom& g, const void* tab, const LinePlan& pl,
                        const BndArgs& bnd, void* out);
void pack_line_task_f64(void* f, const Geom& g, const void* tab, const LinePlan& pl,
                        const BndArgs& bnd, void* out);
size_t line_task_bytes(int prec);
void pack_line_task(int prec, void* f, const Geom& g, const void* tab, const LinePlan& pl,
                    const BndArgs& bnd, void* out);
// rounds: some member's lanes stream their cells through the tile in rounds;
// dir: the members have Dirichlet axes
hipError_t launch_sweep_line_batch(int prec, int P, int dim, bool rounds, bool dir,
                                   const void* tasks, const int64_t* start, int ntask,
                                   int64_t nblocks, int threads, size_t lds_elems, hipStream_t s);

// Equilibrium tables are built into a byte blob matching EqTab<D, M, NV> for
// the (law, dim, m, nv) combination; returns false if the combination has no
// compiled kernel.
bool build_eq_blob(int law, int dim, int m, int nv, const std::vector<double>& law_params,
                   const std::vector<double>& a, const std::vector<double>& b, double omega,
                   const std::vector<double>& mu, std::vector<unsigned char>& blob);

}  // namespace kds
