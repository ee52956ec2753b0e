// kds_api.cpp -- the C ABI of libkds (declared in include/kds.h): problem
// creation and validation, device buffers, the captured per-step HIP graph.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kds_internal.h"
#include "kds_metrics.h"

using namespace kds;

namespace {

thread_local std::string g_create_error;

}  // namespace

struct kds_problem {
  // configuration
  int dim = 0, N[3] = {1, 1, 1}, S[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  int degree = 0, P = 1, nn = 1, m = 0, law = 0, nv = 0;
  std::vector<double> law_params, vel, eq_a, eq_b;
  double omega = 1, dt = 0, theta = 0.5;
  int K = 1, prec = KDS_FP32, sched = KDS_SCHED_PLAIN;
  int64_t ncell = 0;
  Geom geom{};
  // host tables
  std::vector<unsigned char> eq_blob;
  void* eq_dev = nullptr;             // device copy of eq_blob (read by the relaxation)
  std::vector<unsigned char> sweep_blob;  // SweepTab<T>
  LinePlan plan{};
  int line_Q[3] = {1, 1, 1}, line_bw[3] = {1, 1, 1};  // per-axis line-schedule choices
  FrontParams front{};   // front schedule
  int front_mode = 0;
  void* front_W = nullptr;      // [k][nn][Kd] dense cell operators
  int* front_lvl_start = nullptr;
  int* front_lvl_cells = nullptr;
  int4* front_desc = nullptr;   // wave kernel: per cell in front order (see front_wave_fits)
  int front_ndesc = 0;
  bool front_wave = false;      // the wave-per-task front kernel (else one workgroup per subdomain)
  void* fit[2] = {nullptr, nullptr};  // front schedule: iterates
  bool tuned = false;
  bool eager_steps = false;  // kds_step enqueues the kernels itself instead of
                             // replaying captured graphs (autotuner's choice)
  bool relax_vec = false;    // relaxation with 16-byte accesses (autotuner's choice)
  double max_nu = 0, min_sub_width = 0;
  bool proposition_ok = true;
  // stability warnings (kds_info): equilibrium monotonicity (linear law),
  // largest wave speed against the smallest kinetic speed
  int eq_monotone = -1;
  double eq_min_eig = 0.0, wave_speed = -1.0, min_speed = 0.0;
  unsigned long long* wmax = nullptr;  // device: reduction of the Euler wave speed
  // device
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t elem = 4;
  void* f = nullptr;
  void* f_tmp = nullptr;
  void* tr[2] = {nullptr, nullptr};
  double* stage = nullptr;  // FP64 staging for W / F transfers
  size_t stage_bytes = 0;
  int* flag = nullptr;
  void* scratch = nullptr;  // device address of the library's static scratch array
  hipGraph_t graph = nullptr;           // one captured step
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph_n = nullptr;         // kGraphSteps captured steps
  hipGraphExec_t graph_n_exec = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  int lds_cap = 64 * 1024;              // LDS bytes a workgroup may use on the device
  bool state_set = false;
  int steps_done = 0;
  // Dirichlet boundaries (axes with periodic = 0)
  int per[3] = {1, 1, 1};
  int64_t nbnd = 0;                  // boundary nodes
  int64_t boff[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};  // first node of face (axis, side)
  void* fb = nullptr;                // kinetic boundary values: old half, then new half
  double* Wb_dev = nullptr;          // staging of W_b
  bool bnd_set = false;
  int plan_version = 0;  // bumped when the launch plan changes (batches rebuild)
  std::string err;

  int64_t plane() const { return ncell * nn; }
  int64_t n_unknowns() const { return plane() * m * nv; }
  int64_t bnd_half() const { return (int64_t)nv * m * nbnd; }  // elements per time level
  BndArgs bnd() const {
    BndArgs b;
    if (nbnd == 0) return b;
    b.old = fb;
    b.neu = (const unsigned char*)fb + bnd_half() * elem;
    b.nb = nbnd;
    for (int a = 0; a < 3; ++a)
      for (int s = 0; s < 2; ++s) b.off[a][s] = boff[a][s];
    return b;
  }
};

namespace {

kds_status fail(kds_problem* p, kds_status st, const std::string& msg) {
  if (p) p->err = msg; else g_create_error = msg;
  return st;
}

kds_status hip_fail(kds_problem* p, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(p, KDS_E_DEVICE, msg);
}

#define KDS_HIP(p, call)                                    \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((p), e_, #call);  \
  } while (0)

bool finite(double x) { return std::isfinite(x); }

// Validation of the configuration (no device call).
kds_status validate(const kds_config* c, std::string& msg) {
  if (!c) { msg = "cfg is NULL"; return KDS_E_INVALID; }
  if (c->dim < 1 || c->dim > 3) { msg = "dim must be 1, 2 or 3"; return KDS_E_INVALID; }
  for (int a = 0; a < c->dim; ++a) {
    if (c->n_cells[a] < 1) { msg = "n_cells must be >= 1"; return KDS_E_INVALID; }
    if (c->sub_cells[a] < 1 || c->n_cells[a] % c->sub_cells[a] != 0) {
      msg = "sub_cells must be >= 1 and divide n_cells on every axis";
      return KDS_E_INVALID;
    }
    if (c->periodic[a] != 0 && c->periodic[a] != 1) {
      msg = "periodic[a] must be 1 (periodic) or 0 (Dirichlet ends)";
      return KDS_E_INVALID;
    }
    if (!finite(c->box_lo[a]) || !finite(c->box_hi[a]) || !(c->box_hi[a] > c->box_lo[a])) {
      msg = "box_hi must exceed box_lo";
      return KDS_E_INVALID;
    }
  }
  if (c->degree < 0 || c->degree > kMaxP - 1) { msg = "degree must be 0..3"; return KDS_E_INVALID; }
  if (c->m < 1 || c->m > kMaxM) { msg = "m must be 1..8"; return KDS_E_INVALID; }
  if (c->n_vel < 1 || c->n_vel > kMaxVel) { msg = "n_vel must be 1..8"; return KDS_E_INVALID; }
  if (!c->vel) { msg = "vel is NULL"; return KDS_E_INVALID; }
  for (int i = 0; i < c->n_vel * c->dim; ++i)
    if (!finite(c->vel[i])) { msg = "non-finite kinetic velocity"; return KDS_E_INVALID; }
  if (c->law == KDS_LAW_LINEAR) {
    if (!c->law_params || c->n_law_params < c->dim * c->m * c->m) {
      msg = "linear law needs dim*m*m parameters (A^1..A^d)";
      return KDS_E_INVALID;
    }
  } else if (c->law == KDS_LAW_EULER) {
    if (c->m != c->dim + 2) { msg = "Euler needs m = dim + 2"; return KDS_E_INVALID; }
    if (!c->law_params || c->n_law_params < 1 || !(c->law_params[0] > 1.0)) {
      msg = "Euler needs law_params = {gamma > 1}";
      return KDS_E_INVALID;
    }
  } else {
    msg = "unknown law";
    return KDS_E_INVALID;
  }
  if (!(c->omega >= 0.0 && c->omega <= 2.0)) { msg = "omega must be in [0, 2]"; return KDS_E_INVALID; }
  if (!(c->dt > 0.0) || !finite(c->dt)) { msg = "dt must be > 0"; return KDS_E_INVALID; }
  if (!(c->theta >= 0.5 && c->theta <= 1.0)) { msg = "theta must be in [1/2, 1]"; return KDS_E_INVALID; }
  if (c->n_iter < 0) { msg = "n_iter must be >= 0"; return KDS_E_INVALID; }
  if (c->precision < KDS_FP64 || c->precision > KDS_FP32_SPLIT_BF16) { msg = "unknown precision"; return KDS_E_INVALID; }
  if (c->schedule < KDS_SCHED_AUTO || c->schedule > KDS_SCHED_FRONT) { msg = "unknown schedule"; return KDS_E_INVALID; }
  const bool split = c->precision == KDS_FP32_SPLIT_F16 || c->precision == KDS_FP32_SPLIT_BF16;
  bool oblique = false;
  for (int k = 0; k < c->n_vel; ++k) {
    int nz = 0;
    for (int a = 0; a < c->dim; ++a) nz += c->vel[k * c->dim + a] != 0.0;
    if (nz == 0) { msg = "kinetic velocities must be nonzero"; return KDS_E_INVALID; }
    if (nz > 1) oblique = true;
  }
  if ((oblique || split) && c->schedule != KDS_SCHED_AUTO && c->schedule != KDS_SCHED_FRONT) {
    msg = oblique ? "velocities not parallel to a grid axis need the front schedule"
                  : "split precisions are a front-schedule feature";
    return KDS_E_UNSUPPORTED;
  }
  if (c->source_sigma)
    for (int r = 0; r < c->m; ++r)
      if (!(c->source_sigma[r] >= 0.0)) { msg = "source_sigma must be >= 0 (or +inf)"; return KDS_E_INVALID; }
  return KDS_OK;
}

int axis_of(const kds_problem* p, int k) {
  int ax = 0;
  for (int d = 0; d < p->dim; ++d)
    if (p->vel[k * p->dim + d] != 0.0) ax = d;
  return ax;
}

int pow2_at_least(int n) {
  int l2 = 1;
  while (l2 < n) l2 <<= 1;
  return l2;
}

// Is (Q cells per lane, bw columns per bundle) a valid line-schedule choice
// for velocities along axis ax?
bool line_choice_ok(const kds_problem* p, int ax, int Q, int bw) {
  const int Na = p->N[ax], S = p->S[ax];
  const int qmax = line_qmax((int)p->elem, p->nn);
  if (Q < 1 || S % Q || Na / Q > 64 || bw < 1) return false;
  // more cells per lane than the registers hold: rounds through the tile
  // (not in grouped mode, whose tile holds only part of each cell)
  if (Q > qmax && (line_grouped(p->nn) || Q > kMaxRoundQ)) return false;
  if ((int64_t)bw * line_col_lds(Na, p->nn) * (int)p->elem > p->lds_cap) return false;
  if (ax == 0 && bw > p->ncell / Na) return false;
  // (a row of a y / z bundle is copied by one pass of the workgroup, except
  // in grouped mode, which copies 16-value runs)
  if (ax != 0 && (bw > p->N[0] || (!line_grouped(p->nn) && bw * p->nn > 256))) return false;
  return true;
}

// Heuristic choice: many cells per lane as long as >= 3/4 of a line group's
// lanes work; as many columns per bundle as a 32 KB LDS tile holds.  Lines
// longer than 64 lanes of register-held cells: the fewest rounds through the
// tile that put the line in one wavefront.
bool heuristic_choice(const kds_problem* p, int ax, int* Qo, int* bwo) {
  const int Na = p->N[ax], S = p->S[ax];
  const int qmax = line_qmax((int)p->elem, p->nn);
  int bestQ = 0;
  double bestU = -1;
  for (int Q = qmax; Q >= 1; --Q) {
    if (S % Q || Na / Q > 64) continue;
    const double util = (double)(Na / Q) / pow2_at_least(Na / Q);
    if (util >= 0.74) { bestQ = Q; break; }
    if (util > bestU + 1e-12) { bestU = util; bestQ = Q; }
  }
  for (int Q = qmax + 1; !bestQ && Q <= std::min(S, kMaxRoundQ); ++Q)
    if (line_choice_ok(p, ax, Q, 1)) bestQ = Q;
  if (!bestQ) return false;
  const int col = line_col_lds(Na, p->nn) * (int)p->elem;
  int bw = std::max(1, 32 * 1024 / col);
  while (bw > 1 && !line_choice_ok(p, ax, bestQ, bw)) --bw;
  if (!line_choice_ok(p, ax, bestQ, bw)) return false;
  *Qo = bestQ;
  *bwo = bw;
  return true;
}

// Fill the per-velocity launch plan from per-axis choices.
bool finalize_plan(const kds_problem* p, const int* Qax, const int* bwax, LinePlan& pl) {
  std::memset(&pl, 0, sizeof(pl));
  int max_lds = 0, threads = 64;
  int64_t acc = 0;
  for (int k = 0; k < p->nv; ++k) {
    const int ax = axis_of(p, k);
    const int Na = p->N[ax], Q = Qax[ax], bw = bwax[ax];
    if (!line_choice_ok(p, ax, Q, bw)) return false;
    const int l2 = pow2_at_least(Na / Q);
    const int lw = 64 / l2;
    pl.Q[k] = Q;
    pl.lpl2[k] = l2;
    pl.bw[k] = bw;
    max_lds = std::max(max_lds, bw * line_col_lds(Na, p->nn));
    threads = std::max(threads, std::min(256, 64 * ((bw + lw - 1) / lw)));
    if (ax != 0 && !line_grouped(p->nn)) threads = std::max(threads, ((bw * p->nn + 63) / 64) * 64);
    int64_t nb;
    if (ax == 0) nb = (p->ncell / Na + bw - 1) / bw;
    else nb = (int64_t)((p->N[0] + bw - 1) / bw) * (p->ncell / p->N[0] / Na);
    for (int c = 0; c < p->m; ++c) {
      pl.block_start[k * p->m + c] = acc;
      acc += nb;
    }
  }
  pl.block_start[p->nv * p->m] = acc;
  pl.lds_elems = max_lds;
  pl.lds_alloc = max_lds;
  pl.threads = threads;
  pl.xdirect = 0;  // the autotuner switches it on where it is faster
  return threads <= 256 && acc <= 0x7fffffffLL;
}

// Line schedule plan from the heuristic choices.
bool plan_lines(kds_problem* p, std::string& why) {
  if (line_qmax((int)p->elem, p->nn) * line_cell_values(p->nn) * (int)p->elem > 512) {
    why = "line schedule: the cells of one lane do not fit the register budget";
    return false;
  }
  for (int ax = 0; ax < 3; ++ax) { p->line_Q[ax] = 1; p->line_bw[ax] = 1; }
  for (int k = 0; k < p->nv; ++k) {
    const int ax = axis_of(p, k);
    if (!heuristic_choice(p, ax, &p->line_Q[ax], &p->line_bw[ax])) {
      why = "line schedule: no cells-per-lane count divides the subdomain width with the line in one "
            "wavefront (at most " + std::to_string(kMaxRoundQ) + " cells per lane)";
      return false;
    }
  }
  if (!finalize_plan(p, p->line_Q, p->line_bw, p->plan)) {
    why = "line schedule: launch plan out of range";
    return false;
  }
  return true;
}

// Front schedule tables: dense operators per velocity and, per velocity, the
// cells of one subdomain sorted by level l = sum over axes with V^a != 0 of the
// downwind cell index (packed lx | ly << 10 | lz << 20).  desc: the same cells
// as the wave kernel's records (element offset of the cell inside its
// subdomain, downwind coordinates, frontier positions); empty where an offset
// or a position does not fit its field.
bool build_front(kds_problem* p, const Basis1D& basis, std::vector<double>& W,
                 std::vector<int>& lvl_start, std::vector<int>& lvl_cells,
                 std::vector<int4>& desc, std::string& why) {
  FrontParams& fp = p->front;
  std::memset(&fp, 0, sizeof(fp));
  int nn = 0, nf = 0;
  W.clear();
  for (int k = 0; k < p->nv; ++k) {
    std::vector<double> Wk;
    if (!make_dense_op(basis, p->dim, &p->vel[k * p->dim], p->h, p->dt, p->theta, Wk, nn, nf)) {
      why = "front schedule: singular cell operator";
      return false;
    }
    W.insert(W.end(), Wk.begin(), Wk.end());
    for (int a = 0; a < 3; ++a) {
      const double v = a < p->dim ? p->vel[k * p->dim + a] : 0.0;
      fp.sg[k][a] = v > 0 ? 1 : (v < 0 ? -1 : 0);
    }
  }
  fp.nf = nf;
  fp.Kd = nn + 3 * nf;
  for (int a = 0; a < 3; ++a) fp.nsub[a] = p->N[a] / p->S[a];
  fp.theta = p->theta;
  fp.col_chunk = 64;
  lvl_start.clear();
  lvl_cells.clear();
  desc.clear();
  const int S0 = p->S[0], S1 = p->S[1], S2 = p->S[2];
  if (S0 > 1024 || S1 > 1024 || S2 > 1024) { why = "front schedule: subdomain wider than 1024 cells"; return false; }
  // frontier slots per axis (a cell's position: its coordinates on the other two axes)
  fp.fr_pos = std::max(S1 * S2, std::max(S0 * S2, S0 * S1));
  bool desc_ok = fp.fr_pos <= 65536;
  for (int k = 0; k < p->nv; ++k) {
    int act[3];
    for (int a = 0; a < 3; ++a) act[a] = fp.sg[k][a] != 0;
    const int maxlev = act[0] * (S0 - 1) + act[1] * (S1 - 1) + act[2] * (S2 - 1);
    fp.lvl_off[k] = (int)lvl_start.size();
    fp.nlev[k] = maxlev + 1;
    std::vector<std::vector<int>> by(maxlev + 1);
    std::vector<std::vector<int4>> dby(maxlev + 1);
    for (int z = 0; z < S2; ++z)
      for (int y = 0; y < S1; ++y)
        for (int x = 0; x < S0; ++x) {
          const int l = act[0] * x + act[1] * y + act[2] * z;
          by[l].push_back(x | (y << 10) | (z << 20));
          // physical local coordinates run against the velocity where V^a < 0
          const int px = fp.sg[k][0] < 0 ? S0 - 1 - x : x;
          const int py = fp.sg[k][1] < 0 ? S1 - 1 - y : y;
          const int pz = fp.sg[k][2] < 0 ? S2 - 1 - z : z;
          const int64_t loc = ((int64_t)px + (int64_t)p->N[0] * (py + (int64_t)p->N[1] * pz)) * nn;
          if (loc > 0x7fffffffLL) desc_ok = false;
          dby[l].push_back(make_int4((int)loc, x | (y << 10) | (z << 20),
                                     (y + S1 * z) | ((x + S0 * z) << 16), x + S0 * y));
        }
    for (int l = 0; l <= maxlev; ++l) {
      // inside a front any order will do: the cells first along some active
      // axis (their inflow comes across an interface or a box face) go first,
      // so that the wave kernel's tiles of other cells skip those loads
      std::vector<int> ord(by[l].size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
      auto first = [&](int i) {
        const int pk = by[l][i];
        for (int a = 0; a < 3; ++a)
          if (act[a] && ((pk >> (10 * a)) & 1023) == 0) return true;
        return false;
      };
      std::stable_partition(ord.begin(), ord.end(), first);
      lvl_start.push_back((int)lvl_cells.size());
      for (int i : ord) {
        lvl_cells.push_back(by[l][i]);
        desc.push_back(dby[l][i]);
      }
    }
    lvl_start.push_back((int)lvl_cells.size());
  }
  if (!desc_ok) {
    desc.clear();
    fp.fr_pos = 0;
  }
  return true;
}

template <typename T>
void fill_sweep_tab(kds_problem* p, const Basis1D& basis) {
  SweepTab<T> t;
  std::memset(&t, 0, sizeof(t));
  for (int k = 0; k < p->nv; ++k) {
    int ax = 0;
    double v = 0;
    for (int d = 0; d < p->dim; ++d)
      if (p->vel[k * p->dim + d] != 0.0) { ax = d; v = p->vel[k * p->dim + d]; }
    const double nu = std::fabs(v) * p->dt / p->h[ax];  // (oblique velocities: front only)
    LineOp op = make_line_op(basis, nu, p->theta);
    t.axis[k] = ax;
    t.sign[k] = v > 0 ? 1 : -1;
    for (int i = 0; i < p->P * p->P; ++i) t.C[k][i] = (T)op.C[i];
    for (int i = 0; i < p->P; ++i) {
      t.e1[k][i] = (T)((1.0 - p->theta) * op.e[i]);
      t.eth[k][i] = (T)(p->theta * op.e[i]);
    }
  }
  p->sweep_blob.resize(sizeof(t));
  std::memcpy(p->sweep_blob.data(), &t, sizeof(t));
}

// Steps per captured multi-step graph: long kds_step calls launch it, so the
// per-launch cost of a graph is paid once per kGraphSteps steps.
constexpr int kGraphSteps = 8;

void drop_graphs(kds_problem* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->graph_n_exec) (void)hipGraphExecDestroy(p->graph_n_exec);
  if (p->graph_n) (void)hipGraphDestroy(p->graph_n);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  p->graph_n_exec = nullptr;
  p->graph_n = nullptr;
}

void free_device(kds_problem* p) {
  drop_graphs(p);
  for (auto& e : p->ev)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
  void* bufs[] = {p->f, p->f_tmp, p->tr[0], p->tr[1], p->stage, p->flag, p->wmax, p->front_W,
                  p->front_lvl_start, p->front_lvl_cells, p->front_desc, p->fit[0], p->fit[1],
                  p->fb, p->Wb_dev,
                  p->eq_dev};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  p->f = p->f_tmp = p->tr[0] = p->tr[1] = nullptr;
  p->front_W = p->fit[0] = p->fit[1] = nullptr;
  p->front_lvl_start = p->front_lvl_cells = nullptr;
  p->front_desc = nullptr;
  p->fb = nullptr;
  p->Wb_dev = nullptr;
  p->eq_dev = nullptr;
  p->stage = nullptr;
  p->flag = nullptr;
  p->wmax = nullptr;
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  p->stream = nullptr;
}

// One subdomain iteration of the front schedule, with the problem's kernel choice.
hipError_t launch_front_iter(kds_problem* p, const void* f_prev, void* f_cur, hipStream_t s) {
  if (p->front_wave)
    return launch_sweep_front_wave(p->prec, p->front_mode, p->geom, p->front, p->front_W,
                                   p->front_lvl_start, p->front_desc, p->front_ndesc, p->f, f_prev,
                                   f_cur, p->bnd(), s);
  return launch_sweep_front(p->prec, p->front_mode, p->geom, p->front, p->front_W,
                            p->front_lvl_start, p->front_lvl_cells, p->f, f_prev, f_cur, p->bnd(), s);
}

// Which front kernels can run this problem.
bool front_wave_ok(const kds_problem* p) {
  return p->front_ndesc > 0 && front_wave_fits(p->prec, p->front_mode, p->geom, p->front, p->nbnd);
}
bool front_wg_ok(const kds_problem* p) {
  return front_lds_bytes(p->prec, p->front_mode, p->geom, p->front) <= 64 * 1024;
}

// Enqueue one time step (transport then relaxation) on the problem's stream.
// With events, records ev[0] before the transport, ev[1] between transport and
// relaxation, ev[2] after.
kds_status enqueue_step(kds_problem* p, bool events, hipStream_t s) {
  const Geom& g = p->geom;
  if (events) KDS_HIP(p, hipEventRecord(p->ev[0], s));
  if (p->sched == KDS_SCHED_FRONT) {
    for (int it = 1; it <= p->K; ++it) {
      const void* f_prev = it == 1 ? p->f : p->fit[(it - 1) & 1];
      KDS_HIP(p, launch_front_iter(p, f_prev, p->fit[it & 1], s));
    }
    if (events) KDS_HIP(p, hipEventRecord(p->ev[1], s));
    KDS_HIP(p, launch_relax(p->prec, p->law, g, p->eq_dev, p->fit[p->K & 1], p->f, p->relax_vec, s));
  } else if (p->sched == KDS_SCHED_LINE) {
    KDS_HIP(p, launch_sweep_line(p->prec, g, p->sweep_blob.data(), p->plan, p->f, p->bnd(), s));
    if (events) KDS_HIP(p, hipEventRecord(p->ev[1], s));
    KDS_HIP(p, launch_relax(p->prec, p->law, g, p->eq_dev, p->f, p->f, p->relax_vec, s));
  } else {
    for (int it = 1; it <= p->K; ++it) {
      const void* tr_prev = it == 1 ? nullptr : p->tr[(it - 1) & 1];
      void* f_new = it == p->K ? p->f_tmp : nullptr;
      KDS_HIP(p, launch_sweep_plain(p->prec, g, p->sweep_blob.data(), p->f, f_new, tr_prev,
                                    p->tr[it & 1], p->bnd(), s));
    }
    if (events) KDS_HIP(p, hipEventRecord(p->ev[1], s));
    KDS_HIP(p, launch_relax(p->prec, p->law, g, p->eq_dev, p->f_tmp, p->f, p->relax_vec, s));
  }
  // the boundary data at the end of this step are the start data of the next
  if (p->nbnd > 0) {
    const BndArgs b = p->bnd();
    KDS_HIP(p, launch_copy(p->prec, b.neu, p->fb, p->bnd_half(), s));
  }
  if (events) KDS_HIP(p, hipEventRecord(p->ev[2], s));
  return KDS_OK;
}

// Capture `steps` consecutive steps into (graph, exec) unless already there.
kds_status ensure_graph(kds_problem* p, int steps, hipGraph_t* graph_out, hipGraphExec_t* exec) {
  if (*exec) return KDS_OK;
  KDS_HIP(p, hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  kds_status st = KDS_OK;
  for (int i = 0; i < steps && st == KDS_OK; ++i) st = enqueue_step(p, false, p->stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &graph);
  if (st != KDS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(p, e, "hipStreamEndCapture");
  *graph_out = graph;
  KDS_HIP(p, hipGraphInstantiate(exec, graph, nullptr, nullptr, 0));
  return KDS_OK;
}

kds_status check_device_ptr(kds_problem* p, const void* ptr) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, KDS_E_INVALID, "on_device = 1 but the pointer is not HIP memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(p, KDS_E_INVALID, "on_device = 1 but the pointer is not device memory");
  if (attr.type == hipMemoryTypeDevice && attr.device != p->device)
    return fail(p, KDS_E_INVALID, "device pointer belongs to another GPU");
  return KDS_OK;
}

kds_status ensure_stage(kds_problem* p, size_t bytes) {
  if (p->stage_bytes >= bytes) return KDS_OK;
  if (p->stage) (void)hipFree(p->stage);
  p->stage = nullptr;
  p->stage_bytes = 0;
  hipError_t e = hipMalloc((void**)&p->stage, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, KDS_E_NOMEM, "staging buffer allocation failed");
  }
  p->stage_bytes = bytes;
  return KDS_OK;
}

}  // namespace

extern "C" {

kds_status kds_create(const kds_config* cfg, void* hip_stream, kds_problem** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, KDS_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string msg;
  kds_status st = validate(cfg, msg);
  if (st != KDS_OK) return fail(nullptr, st, msg);

  kds_problem* p = new kds_problem();
  p->dim = cfg->dim;
  p->ncell = 1;
  for (int a = 0; a < 3; ++a) {
    p->N[a] = a < cfg->dim ? cfg->n_cells[a] : 1;
    p->S[a] = a < cfg->dim ? cfg->sub_cells[a] : 1;
    p->lo[a] = a < cfg->dim ? cfg->box_lo[a] : 0.0;
    p->hi[a] = a < cfg->dim ? cfg->box_hi[a] : 1.0;
    p->h[a] = (p->hi[a] - p->lo[a]) / p->N[a];
    p->ncell *= p->N[a];
    p->per[a] = a < cfg->dim ? cfg->periodic[a] : 1;
  }
  p->degree = cfg->degree;
  p->P = cfg->degree + 1;
  p->nn = 1;
  for (int a = 0; a < p->dim; ++a) p->nn *= p->P;
  // boundary nodes: faces of the non-periodic axes, low end then high end
  for (int a = 0; a < p->dim; ++a) {
    if (p->per[a]) continue;
    const int64_t face = p->ncell / p->N[a] * (p->nn / p->P);
    p->boff[a][0] = p->nbnd;
    p->boff[a][1] = p->nbnd + face;
    p->nbnd += 2 * face;
  }
  p->m = cfg->m;
  p->law = cfg->law;
  p->nv = cfg->n_vel;
  p->law_params.assign(cfg->law_params, cfg->law_params + cfg->n_law_params);
  p->vel.assign(cfg->vel, cfg->vel + cfg->n_vel * cfg->dim);
  p->omega = cfg->omega;
  p->dt = cfg->dt;
  p->theta = cfg->theta;
  p->K = cfg->n_iter;
  p->prec = cfg->precision == KDS_FP64 ? KDS_FP64 : KDS_FP32;  // storage precision
  p->elem = p->prec == KDS_FP64 ? 8 : 4;
  p->front_mode = cfg->precision == KDS_FP32_SPLIT_F16    ? kFrontSplitF16
                  : cfg->precision == KDS_FP32_SPLIT_BF16 ? kFrontSplitBf16
                  : cfg->precision == KDS_FP32            ? kFrontMfma
                                                          : kFrontFma;

  std::vector<double> a, b;
  if (!eq_weights(p->dim, p->nv, p->vel.data(), cfg->eq_a, cfg->eq_b, a, b, msg)) {
    delete p;
    return fail(nullptr, KDS_E_INVALID, msg);
  }
  // warnings: sub-characteristic condition (Sec. 2.1) and equilibrium
  // monotonicity; for Euler the wave speed is taken from each kds_set_state
  p->min_speed = 1e300;
  for (int k = 0; k < p->nv; ++k) {
    double v2 = 0.0;
    for (int i = 0; i < p->dim; ++i) v2 += p->vel[k * p->dim + i] * p->vel[k * p->dim + i];
    p->min_speed = std::min(p->min_speed, std::sqrt(v2));
  }
  if (p->law == KDS_LAW_LINEAR) {
    const EqChecks ec = check_linear_law(p->dim, p->m, p->nv, p->law_params, a, b);
    if (ec.checked) {
      p->wave_speed = ec.wave_speed;
      p->eq_min_eig = ec.min_eig;
      double amax = 1.0;
      for (double x : a) amax = std::max(amax, std::fabs(x));
      p->eq_monotone = ec.min_eig >= -1e-12 * amax ? 1 : 0;
    }
  }
  std::vector<double> mu;
  if (cfg->source_sigma) {
    mu.resize(p->m);
    for (int r = 0; r < p->m; ++r) {
      const double sg = cfg->source_sigma[r];
      mu[r] = std::isinf(sg) ? -1.0 : (1.0 - 0.5 * sg * p->dt) / (1.0 + 0.5 * sg * p->dt);
    }
  }
  if (!build_eq_blob(p->law, p->dim, p->m, p->nv, p->law_params, a, b, p->omega, mu, p->eq_blob)) {
    delete p;
    return fail(nullptr, KDS_E_UNSUPPORTED,
                "no compiled relaxation kernel for this (law, dim, m, n_vel) combination");
  }
  Basis1D basis = make_basis(p->degree);
  bool oblique = false;
  for (int k = 0; k < p->nv; ++k) {
    int nz = 0;
    for (int a = 0; a < p->dim; ++a) nz += p->vel[k * p->dim + a] != 0.0;
    oblique |= nz > 1;
  }
  const bool want_front = oblique || cfg->schedule == KDS_SCHED_FRONT ||
                          cfg->precision == KDS_FP32_SPLIT_F16 || cfg->precision == KDS_FP32_SPLIT_BF16;
  if (!oblique) {
    if (p->prec == KDS_FP64) fill_sweep_tab<double>(p, basis);
    else fill_sweep_tab<float>(p, basis);
  }
  std::vector<double> frontW;
  std::vector<int> lvl_start, lvl_cells;
  std::vector<int4> front_desc;
  if (want_front && !build_front(p, basis, frontW, lvl_start, lvl_cells, front_desc, msg)) {
    delete p;
    return fail(nullptr, KDS_E_UNSUPPORTED, msg);
  }

  Geom& g = p->geom;
  g.dim = p->dim;
  for (int ax = 0; ax < 3; ++ax) { g.N[ax] = p->N[ax]; g.S[ax] = p->S[ax]; }
  g.P = p->P;
  g.nn = p->nn;
  g.ncell = p->ncell;
  g.m = p->m;
  g.nv = p->nv;
  g.K = p->K;
  g.tr_stride = 0;
  p->max_nu = 0;
  p->min_sub_width = 1e300;
  for (int k = 0; k < p->nv; ++k) {
    for (int ax = 0; ax < p->dim; ++ax) {
      double v = std::fabs(p->vel[k * p->dim + ax]);
      if (v == 0.0) continue;
      double nu = v * p->dt / p->h[ax];
      p->max_nu = std::max(p->max_nu, nu);
      // Sec. 5.1 Proposition: |V| dt <= subdomain diameter along the velocity
      if (v * p->dt > p->S[ax] * p->h[ax] * (1 + 1e-12)) p->proposition_ok = false;
      int64_t lines = (p->ncell / p->N[ax]) * (p->nn / p->P) * (p->N[ax] / p->S[ax]);
      g.tr_stride = std::max<int64_t>(g.tr_stride, lines);
    }
  }
  for (int ax = 0; ax < p->dim; ++ax) p->min_sub_width = std::min(p->min_sub_width, p->S[ax] * p->h[ax]);

  std::string why;
  {
    // LDS a workgroup may allocate (160 KiB on gfx950): bounds the line tiles
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      p->lds_cap = std::min(v, 160 * 1024);
    else
      (void)hipGetLastError();
  }
  const bool line_ok = !want_front && plan_lines(p, why);
  if (cfg->schedule == KDS_SCHED_LINE && !line_ok) {
    delete p;
    return fail(nullptr, KDS_E_UNSUPPORTED, why);
  }
  p->sched = (cfg->schedule == KDS_SCHED_PLAIN || !line_ok) ? KDS_SCHED_PLAIN : KDS_SCHED_LINE;
  if (want_front) {
    p->sched = KDS_SCHED_FRONT;
    p->front_ndesc = (int)front_desc.size();
    // the wave-per-task kernel where it applies (its records fit; FP32
    // matrix-core forms up to 64-node cells, FP64 up to 32), else one
    // workgroup per subdomain
    p->front_wave = front_wave_ok(p);
    if (!p->front_wave && !front_wg_ok(p)) {
      delete p;
      return fail(nullptr, KDS_E_UNSUPPORTED, "front schedule: cell operator too large for the LDS");
    }
  }
  if (p->K == 0 && p->sched != KDS_SCHED_LINE) {
    delete p;
    return fail(nullptr, KDS_E_UNSUPPORTED,
                "n_iter = 0 (converged subdomain iteration) needs the line schedule" +
                    (why.empty() ? std::string() : ": " + why));
  }

  // ---------------------------------------------------------------- device
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return fail(nullptr, KDS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  const size_t state_bytes = (size_t)p->n_unknowns() * p->elem;
  size_t need = state_bytes + 2 * (size_t)p->bnd_half() * p->elem + (size_t)p->nbnd * p->m * 8;
  if (p->sched == KDS_SCHED_PLAIN) need += state_bytes + 2 * (size_t)g.tr_stride * p->nv * p->m * p->elem;
  if (p->sched == KDS_SCHED_FRONT) need += 2 * state_bytes;
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) {
    delete p;
    return fail(nullptr, KDS_E_DEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
  }
  if (need + (64u << 20) > free_b) {
    delete p;
    return fail(nullptr, KDS_E_NOMEM, "the kinetic state does not fit the free device memory");
  }
  auto alloc = [&](void** ptr, size_t bytes) -> bool {
    hipError_t ee = hipMalloc(ptr, bytes);
    if (ee != hipSuccess) { (void)hipGetLastError(); *ptr = nullptr; return false; }
    return true;
  };
  bool ok = alloc(&p->f, state_bytes) && alloc((void**)&p->flag, sizeof(int)) &&
            alloc((void**)&p->wmax, sizeof(unsigned long long)) &&
            alloc(&p->eq_dev, p->eq_blob.size());
  if (ok)
    ok = hipMemcpy(p->eq_dev, p->eq_blob.data(), p->eq_blob.size(), hipMemcpyHostToDevice) ==
         hipSuccess;
  if (ok && p->nbnd > 0)
    ok = alloc(&p->fb, 2 * (size_t)p->bnd_half() * p->elem) &&
         alloc((void**)&p->Wb_dev, (size_t)p->nbnd * p->m * sizeof(double));
  if (ok && p->sched == KDS_SCHED_PLAIN) {
    const size_t trb = std::max<size_t>(1, (size_t)g.tr_stride * p->nv * p->m * p->elem);
    ok = alloc(&p->f_tmp, state_bytes) && alloc(&p->tr[0], trb) && alloc(&p->tr[1], trb);
  }
  if (ok && p->sched == KDS_SCHED_FRONT) {
    ok = alloc(&p->fit[0], state_bytes) && alloc(&p->fit[1], state_bytes) &&
         alloc(&p->front_W, frontW.size() * p->elem) &&
         alloc((void**)&p->front_lvl_start, lvl_start.size() * sizeof(int)) &&
         alloc((void**)&p->front_lvl_cells, lvl_cells.size() * sizeof(int)) &&
         (front_desc.empty() || alloc((void**)&p->front_desc, front_desc.size() * sizeof(int4)));
    if (ok) {
      std::vector<float> w32;
      const void* src = frontW.data();
      if (p->prec != KDS_FP64) {
        w32.assign(frontW.begin(), frontW.end());
        src = w32.data();
      }
      ok = hipMemcpy(p->front_W, src, frontW.size() * p->elem, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(p->front_lvl_start, lvl_start.data(), lvl_start.size() * sizeof(int),
                     hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(p->front_lvl_cells, lvl_cells.data(), lvl_cells.size() * sizeof(int),
                     hipMemcpyHostToDevice) == hipSuccess &&
           (front_desc.empty() ||
            hipMemcpy(p->front_desc, front_desc.data(), front_desc.size() * sizeof(int4),
                      hipMemcpyHostToDevice) == hipSuccess);
    }
  }
  if (!ok) {
    free_device(p);
    delete p;
    return fail(nullptr, KDS_E_NOMEM, "device allocation failed");
  }
  // the static scratch of the allocation-free entry points: its address on
  // this device (looked up once per device, the device current)
  e = scratch_address(&p->scratch);
  if (e != hipSuccess) {
    free_device(p);
    delete p;
    return fail(nullptr, KDS_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  }
  if (hip_stream) {
    p->stream = (hipStream_t)hip_stream;
    p->own_stream = false;
  } else {
    // a blocking stream: ordered after work on the legacy default stream
    e = hipStreamCreate(&p->stream);
    if (e != hipSuccess) {
      free_device(p);
      delete p;
      return fail(nullptr, KDS_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    p->own_stream = true;
  }
  for (auto& ev : p->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      free_device(p);
      delete p;
      return fail(nullptr, KDS_E_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  if (p->sched == KDS_SCHED_LINE) {
    if ((size_t)p->plan.lds_elems * p->elem > (size_t)p->lds_cap) {
      free_device(p);
      delete p;
      return fail(nullptr, KDS_E_UNSUPPORTED, "line schedule LDS tile too large");
    }
    // plans (also the autotuner's) may use up to lds_cap bytes of dynamic LDS
    e = line_kernels_allow_lds((size_t)p->lds_cap);
    if (e != hipSuccess) {
      free_device(p);
      delete p;
      return fail(nullptr, KDS_E_DEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
  }
  *out = p;
  return KDS_OK;
}

kds_status kds_set_state(kds_problem* p, const double* W, int32_t on_device) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!W) return fail(p, KDS_E_INVALID, "W is NULL");
  const size_t bytes = (size_t)p->plane() * p->m * sizeof(double);
  const double* src = W;
  if (on_device) {
    kds_status st = check_device_ptr(p, W);
    if (st != KDS_OK) return st;
  } else {
    kds_status st = ensure_stage(p, bytes);
    if (st != KDS_OK) return st;
    KDS_HIP(p, hipMemcpyAsync(p->stage, W, bytes, hipMemcpyHostToDevice, p->stream));
    src = p->stage;
  }
  KDS_HIP(p, launch_init(p->prec, p->law, p->geom, p->eq_blob.data(), src, p->f, p->stream));
  // a state with NaN / Inf (or equilibria that overflow the storage) is refused
  const int zero = 0;
  int flag = 0;
  KDS_HIP(p, hipMemcpyAsync(p->flag, &zero, sizeof(int), hipMemcpyHostToDevice, p->stream));
  KDS_HIP(p, launch_check_finite(p->prec, p->geom, p->f, p->flag, p->stream));
  KDS_HIP(p, hipMemcpyAsync(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  // Euler: the largest wave speed of this state (sub-characteristic check)
  unsigned long long wbits = 0;
  if (p->law == KDS_LAW_EULER) {
    const unsigned long long z = 0;
    KDS_HIP(p, hipMemcpyAsync(p->wmax, &z, sizeof(z), hipMemcpyHostToDevice, p->stream));
    KDS_HIP(p, launch_euler_wave_speed(src, p->plane(), p->dim, p->law_params[0], p->wmax, p->stream));
    KDS_HIP(p, hipMemcpyAsync(&wbits, p->wmax, sizeof(wbits), hipMemcpyDeviceToHost, p->stream));
  }
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  if (flag) {
    p->state_set = false;
    return fail(p, KDS_E_NONFINITE,
                "kds_set_state: W holds NaN or Inf (or values whose equilibria overflow the "
                "storage precision)");
  }
  if (p->law == KDS_LAW_EULER) {
    double ws;
    std::memcpy(&ws, &wbits, sizeof(ws));
    p->wave_speed = ws;
  }
  p->state_set = true;
  p->steps_done = 0;
  return KDS_OK;
}

kds_status kds_set_boundary(kds_problem* p, const double* Wb, int32_t on_device) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (p->nbnd == 0) return fail(p, KDS_E_INVALID, "the box is periodic on every axis");
  if (!Wb) return fail(p, KDS_E_INVALID, "W_b is NULL");
  const size_t bytes = (size_t)p->nbnd * p->m * sizeof(double);
  if (on_device) {
    kds_status st = check_device_ptr(p, Wb);
    if (st != KDS_OK) return st;
    KDS_HIP(p, hipMemcpyAsync(p->Wb_dev, Wb, bytes, hipMemcpyDeviceToDevice, p->stream));
  } else {
    KDS_HIP(p, hipMemcpyAsync(p->Wb_dev, Wb, bytes, hipMemcpyHostToDevice, p->stream));
  }
  // the boundary nodes as a one-node-per-cell grid: F_k = M_k(W_b) into the
  // new half, after the new half of the previous call moved to the old half
  Geom gb = p->geom;
  gb.ncell = p->nbnd;
  gb.nn = 1;
  const BndArgs b = p->bnd();
  void* neu = const_cast<void*>(b.neu);
  if (p->bnd_set) KDS_HIP(p, launch_copy(p->prec, b.neu, p->fb, p->bnd_half(), p->stream));
  KDS_HIP(p, launch_init(p->prec, p->law, gb, p->eq_blob.data(), p->Wb_dev, neu, p->stream));
  if (!p->bnd_set) KDS_HIP(p, launch_copy(p->prec, b.neu, p->fb, p->bnd_half(), p->stream));
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  p->bnd_set = true;
  return KDS_OK;
}

kds_status kds_step(kds_problem* p, int32_t n_steps) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (n_steps < 0) return fail(p, KDS_E_INVALID, "n_steps must be >= 0");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_step before kds_set_state / kds_set_kinetic");
  if (p->nbnd > 0 && !p->bnd_set)
    return fail(p, KDS_E_STATE, "Dirichlet axes: kds_set_boundary before kds_step");
  if (n_steps == 0) return KDS_OK;
  int left = n_steps;
  if (p->eager_steps) {
    for (; left > 0; --left) {
      kds_status st = enqueue_step(p, false, p->stream);
      if (st != KDS_OK) return st;
    }
  }
  if (left >= kGraphSteps) {
    kds_status st = ensure_graph(p, kGraphSteps, &p->graph_n, &p->graph_n_exec);
    if (st != KDS_OK) return st;
    for (; left >= kGraphSteps; left -= kGraphSteps)
      KDS_HIP(p, hipGraphLaunch(p->graph_n_exec, p->stream));
  }
  if (left > 0) {
    kds_status st = ensure_graph(p, 1, &p->graph, &p->graph_exec);
    if (st != KDS_OK) return st;
    for (; left > 0; --left) KDS_HIP(p, hipGraphLaunch(p->graph_exec, p->stream));
  }
  p->steps_done += n_steps;
  return KDS_OK;
}

kds_status kds_step_timed(kds_problem* p, int32_t n_steps, double* kernel_ms) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (n_steps < 0 || !kernel_ms) return fail(p, KDS_E_INVALID, "bad arguments");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_step_timed before kds_set_state");
  if (p->nbnd > 0 && !p->bnd_set) return fail(p, KDS_E_STATE, "Dirichlet axes: kds_set_boundary first");
  double acc[KDS_N_KERNEL_KINDS] = {0, 0};
  for (int i = 0; i < n_steps; ++i) {
    kds_status st = enqueue_step(p, true, p->stream);
    if (st != KDS_OK) return st;
    KDS_HIP(p, hipEventSynchronize(p->ev[2]));
    float t01 = 0, t12 = 0;
    KDS_HIP(p, hipEventElapsedTime(&t01, p->ev[0], p->ev[1]));
    KDS_HIP(p, hipEventElapsedTime(&t12, p->ev[1], p->ev[2]));
    acc[0] += t01;
    acc[1] += t12;
  }
  p->steps_done += n_steps;
  for (int i = 0; i < KDS_N_KERNEL_KINDS; ++i) kernel_ms[i] = acc[i];
  return KDS_OK;
}

kds_status kds_tune(kds_problem* p, int32_t reps, double* sweep_ms) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_tune needs a state (kds_set_state first)");
  if (p->nbnd > 0 && !p->bnd_set) return fail(p, KDS_E_STATE, "Dirichlet axes: kds_set_boundary first");
  // plain and front schedules: only the step launch mode is tuned
  const bool line = p->sched == KDS_SCHED_LINE;
  reps = std::max(1, std::min(reps, 100));
  const size_t bytes = (size_t)p->n_unknowns() * p->elem;
  void* save = nullptr;
  if (hipMalloc(&save, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, KDS_E_NOMEM, "kds_tune: no device memory to save the state");
  }
  KDS_HIP(p, hipMemcpyAsync(save, p->f, bytes, hipMemcpyDeviceToDevice, p->stream));
  // the choices before tuning, restored if the tuner fails part way
  const LinePlan plan0 = p->plan;
  int Q0[3], bw0[3];
  for (int a = 0; a < 3; ++a) { Q0[a] = p->line_Q[a]; bw0[a] = p->line_bw[a]; }
  const bool eager0 = p->eager_steps, vec0 = p->relax_vec, wave0 = p->front_wave;
  kds_status st = KDS_OK;
  auto time_plan = [&](const LinePlan& pl, float* ms) -> bool {
    hipError_t e = launch_sweep_line(p->prec, p->geom, p->sweep_blob.data(), pl, p->f, p->bnd(),
                                     p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->ev[0], p->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      e = launch_sweep_line(p->prec, p->geom, p->sweep_blob.data(), pl, p->f, p->bnd(), p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->ev[1], p->stream);
    if (e == hipSuccess) e = hipEventSynchronize(p->ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, p->ev[0], p->ev[1]);
    if (e != hipSuccess) {
      st = hip_fail(p, e, "kds_tune");
      return false;
    }
    *ms /= reps;
    return true;
  };
  float best = -1.0f;
  bool ok = !line || time_plan(p->plan, &best);
  bool used[3] = {false, false, false};
  for (int k = 0; k < p->nv; ++k) used[axis_of(p, k)] = true;
  const int bws[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16, 20, 24, 28, 32};
  // coordinate search: one axis at a time, over (cells per lane, bundle width)
  for (int ax = 0; ax < 3 && ok && line; ++ax) {
    if (!used[ax]) continue;
    for (int Q = 1; Q <= kMaxRoundQ && ok; ++Q)
      for (int bw : bws) {
        // (counts beyond the register budget, whose cells stream through the
        // tile in rounds, only where the line does not fit the registers:
        // elsewhere they cost 2-5x the register plans)
        const int qmax = std::max(1, line_qmax((int)p->elem, p->nn));
        if (Q > qmax && p->N[ax] / qmax <= 64) break;
        if (!line_choice_ok(p, ax, Q, bw)) continue;
        if (Q == p->line_Q[ax] && bw == p->line_bw[ax]) continue;
        int tq[3], tb[3];
        for (int i = 0; i < 3; ++i) { tq[i] = p->line_Q[i]; tb[i] = p->line_bw[i]; }
        tq[ax] = Q;
        tb[ax] = bw;
        LinePlan pl;
        if (!finalize_plan(p, tq, tb, pl)) continue;
        float ms = 0.0f;
        if (!(ok = time_plan(pl, &ms))) break;
        if (ms < 0.97f * best) {
          best = ms;
          p->line_Q[ax] = Q;
          p->line_bw[ax] = bw;
          p->plan = pl;
        }
      }
  }
  // x lines: the direct register path where it is clearly faster than the
  // LDS tile (both timed again, back to back); it applies to x lines with
  // line_qmax cells per lane, outside grouped mode
  if (ok && line && used[0] && !line_grouped(p->nn) &&
      p->line_Q[0] == line_qmax((int)p->elem, p->nn)) {
    LinePlan pl = p->plan;
    pl.xdirect = 1;
    float ms_tile = 0.0f, ms_direct = 0.0f;
    ok = time_plan(p->plan, &ms_tile) && time_plan(pl, &ms_direct);
    if (ok && ms_direct < 0.97f * ms_tile) {
      best = ms_direct;
      p->plan = pl;
    }
  }
  // workgroups per CU: more LDS per workgroup than the tile needs lets fewer
  // of them share a CU, so that later ones start while earlier ones compute
  if (ok && line) {
    const int cu_lds = 160 * 1024;
    for (int per_cu : {8, 6, 4, 3, 2}) {
      LinePlan pl = p->plan;
      const int want = std::min(p->lds_cap, cu_lds / per_cu) / (int)p->elem - 64;
      if (want <= pl.lds_elems) continue;
      pl.lds_alloc = want;
      float ms = 0.0f;
      if (!(ok = time_plan(pl, &ms))) break;
      if (ms < 0.97f * best) {
        best = ms;
        p->plan = pl;
      }
    }
  }
  // front schedule: the wave-per-task kernel against the workgroup kernel,
  // where both apply (one subdomain iteration from the saved state each;
  // the arithmetic is the same up to rounding order)
  if (ok && p->sched == KDS_SCHED_FRONT && front_wave_ok(p) && front_wg_ok(p)) {
    float ms_k[2] = {0.0f, 0.0f};
    for (int pass = 0; pass < 2 && ok; ++pass)
      for (int w = 0; w < 2 && ok; ++w) {
        p->front_wave = w == 1;
        hipError_t e = launch_front_iter(p, p->f, p->fit[1], p->stream);
        if (e == hipSuccess) e = hipEventRecord(p->ev[0], p->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
          e = launch_front_iter(p, p->f, p->fit[1], p->stream);
        if (e == hipSuccess) e = hipEventRecord(p->ev[1], p->stream);
        if (e == hipSuccess) e = hipEventSynchronize(p->ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->ev[0], p->ev[1]);
        if (e != hipSuccess) {
          st = hip_fail(p, e, "kds_tune");
          ok = false;
        }
        ms_k[w] += ms / reps;
      }
    if (ok) {
      p->front_wave = ms_k[1] < 0.97f * ms_k[0];
      best = 0.5f * (p->front_wave ? ms_k[1] : ms_k[0]);
    }
  }
  // step launch mode: captured graphs of kGraphSteps steps against the step's
  // kernels enqueued one by one (for short steps the graph replay can cost
  // more than it saves); then, in the chosen mode, the relaxation with 16-byte
  // accesses against one node per thread.  Whole steps, timed with events on
  // the stream, twice each.  Not for Dirichlet axes, whose steps also advance
  // the boundary data.
  if (ok && p->nbnd == 0) {
    // whole steps start from the saved state (the plan search above swept it
    // in place, without relaxing)
    hipError_t er = hipMemcpyAsync(p->f, save, bytes, hipMemcpyDeviceToDevice, p->stream);
    if (er != hipSuccess) {
      st = hip_fail(p, er, "kds_tune");
      ok = false;
    }
  }
  if (ok && p->nbnd == 0) {
    int nrep = 1;
    // ms per kGraphSteps * nrep steps in the current mode (graph or enqueued)
    auto time_steps = [&](float* ms) -> bool {
      hipError_t e = hipSuccess;
      if (!p->eager_steps) {
        st = ensure_graph(p, kGraphSteps, &p->graph_n, &p->graph_n_exec);
        if (st != KDS_OK) return false;
        e = hipGraphLaunch(p->graph_n_exec, p->stream);  // warm-up
      } else {
        st = enqueue_step(p, false, p->stream);
        if (st != KDS_OK) return false;
      }
      if (e == hipSuccess) e = hipEventRecord(p->ev[0], p->stream);
      for (int r = 0; r < nrep && e == hipSuccess; ++r) {
        if (!p->eager_steps) {
          e = hipGraphLaunch(p->graph_n_exec, p->stream);
        } else {
          for (int i = 0; i < kGraphSteps; ++i)
            if ((st = enqueue_step(p, false, p->stream)) != KDS_OK) return false;
        }
      }
      if (e == hipSuccess) e = hipEventRecord(p->ev[1], p->stream);
      if (e == hipSuccess) e = hipEventSynchronize(p->ev[1]);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, p->ev[0], p->ev[1]);
      if (e != hipSuccess) {
        st = hip_fail(p, e, "kds_tune");
        return false;
      }
      return true;
    };
    // samples of about 4 ms (at least kGraphSteps steps, at most 8 times that)
    float ms_one = 0.0f;
    drop_graphs(p);
    ok = time_steps(&ms_one);
    if (ok) nrep = std::max(1, std::min(8, (int)std::ceil(4.0f / std::max(ms_one, 1e-3f))));
    // each choice timed three times, alternating, and judged by its fastest
    // sample: a sporadic slow sample (another process, a clock change) then
    // cannot flip a choice whose margin is a few percent
    auto pick = [&](bool* flag) -> bool {
      float t0 = 1e30f, t1 = 1e30f;
      for (int pass = 0; pass < 3; ++pass)
        for (int v = 0; v < 2; ++v) {
          *flag = v == 1;
          drop_graphs(p);
          float ms = 0.0f;
          if (!time_steps(&ms)) return false;
          float& t = v ? t1 : t0;
          t = std::min(t, ms);
        }
      *flag = t1 < 0.98f * t0;
      drop_graphs(p);
      return true;
    };
    ok = ok && pick(&p->eager_steps) && pick(&p->relax_vec);
  }
  // restore the state and drop the graph captured with the old plan
  hipError_t e = hipMemcpyAsync(p->f, save, bytes, hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  (void)hipFree(save);
  if (!ok || e != hipSuccess) {
    p->plan = plan0;
    for (int a = 0; a < 3; ++a) { p->line_Q[a] = Q0[a]; p->line_bw[a] = bw0[a]; }
    p->eager_steps = eager0;
    p->relax_vec = vec0;
    p->front_wave = wave0;
    drop_graphs(p);
    return ok ? hip_fail(p, e, "kds_tune restore") : st;
  }
  drop_graphs(p);
  p->tuned = line;
  // (a batch regroups its members when a line plan or a front kernel changed)
  if (line || p->front_wave != wave0) ++p->plan_version;
  if (sweep_ms) *sweep_ms = (line || best > 0.0f) ? best : -1.0;
  return KDS_OK;
}

kds_status kds_set_launch(kds_problem* p, int32_t step_eager, int32_t relax_vec) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if ((step_eager != 0 && step_eager != 1) || (relax_vec != 0 && relax_vec != 1))
    return fail(p, KDS_E_INVALID, "kds_set_launch: flags must be 0 or 1");
  p->eager_steps = step_eager == 1;
  p->relax_vec = relax_vec == 1;
  drop_graphs(p);  // captured with the previous relaxation kernel
  return KDS_OK;
}

kds_status kds_get_plan(const kds_problem* p, kds_plan_t* pl) {
  if (!p || !pl) return fail(nullptr, KDS_E_INVALID, "NULL argument");
  std::memset(pl, 0, sizeof(*pl));
  if (p->sched == KDS_SCHED_LINE) {
    for (int k = 0; k < p->nv; ++k) {
      const int a = axis_of(p, k);
      pl->Q[a] = p->line_Q[a];
      pl->bw[a] = p->line_bw[a];
    }
    pl->xdirect = p->plan.xdirect;
    pl->lds_bytes = p->plan.lds_alloc > p->plan.lds_elems ? p->plan.lds_alloc * (int)p->elem : 0;
  }
  if (p->sched == KDS_SCHED_FRONT) pl->front_kernel = p->front_wave ? 2 : 1;
  pl->step_eager = p->eager_steps ? 1 : 0;
  pl->relax_vec = p->relax_vec ? 1 : 0;
  return KDS_OK;
}

kds_status kds_set_plan(kds_problem* p, const kds_plan_t* pl) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!pl) return fail(p, KDS_E_INVALID, "plan is NULL");
  auto flag = [](int32_t v) { return v == 0 || v == 1; };
  if (!flag(pl->xdirect) || !flag(pl->step_eager) || !flag(pl->relax_vec) || pl->lds_bytes < 0)
    return fail(p, KDS_E_INVALID, "kds_set_plan: flags must be 0 or 1 and lds_bytes >= 0");
  if (p->sched == KDS_SCHED_LINE) {
    bool used[3] = {false, false, false};
    for (int k = 0; k < p->nv; ++k) used[axis_of(p, k)] = true;
    int tq[3], tb[3];
    for (int a = 0; a < 3; ++a) {
      tq[a] = used[a] ? pl->Q[a] : p->line_Q[a];
      tb[a] = used[a] ? pl->bw[a] : p->line_bw[a];
      if (used[a] && !line_choice_ok(p, a, tq[a], tb[a]))
        return fail(p, KDS_E_INVALID,
                    "kds_set_plan: cells per lane / columns per workgroup outside the limits on axis " +
                        std::to_string(a));
    }
    LinePlan np;
    if (!finalize_plan(p, tq, tb, np)) return fail(p, KDS_E_INVALID, "kds_set_plan: launch plan out of range");
    if (pl->xdirect) {
      if (!used[0] || line_grouped(p->nn) || tq[0] != line_qmax((int)p->elem, p->nn))
        return fail(p, KDS_E_INVALID,
                    "kds_set_plan: xdirect needs a velocity along x and Q[0] = line_qmax "
                    "(and cells of at most 27 nodes)");
      np.xdirect = 1;
    }
    if (pl->lds_bytes > 0) {
      const int el = pl->lds_bytes / (int)p->elem;
      if (pl->lds_bytes > p->lds_cap || el < np.lds_elems)
        return fail(p, KDS_E_INVALID,
                    "kds_set_plan: lds_bytes must cover the tile (" +
                        std::to_string(np.lds_elems * (int)p->elem) + " bytes) and fit the device (" +
                        std::to_string(p->lds_cap) + " bytes)");
      np.lds_alloc = el;
    }
    for (int a = 0; a < 3; ++a) { p->line_Q[a] = tq[a]; p->line_bw[a] = tb[a]; }
    p->plan = np;
    ++p->plan_version;
  }
  if (p->sched == KDS_SCHED_FRONT && pl->front_kernel != 0) {
    const bool wave_before = p->front_wave;
    if (pl->front_kernel == 2 && front_wave_ok(p)) p->front_wave = true;
    else if (pl->front_kernel == 1 && front_wg_ok(p)) p->front_wave = false;
    else
      return fail(p, KDS_E_INVALID,
                  std::string("kds_set_plan: front_kernel ") + std::to_string(pl->front_kernel) +
                      " does not apply (1: workgroup kernel" + (front_wg_ok(p) ? "" : ", not here") +
                      "; 2: wave kernel" + (front_wave_ok(p) ? "" : ", not here") + ")");
    if (p->front_wave != wave_before) ++p->plan_version;
  }
  p->eager_steps = pl->step_eager == 1;
  p->relax_vec = pl->relax_vec == 1;
  drop_graphs(p);
  return KDS_OK;
}

namespace {

// The plan cache key of a problem (one line of text, no '|').
std::string plan_key(const kds_problem* p) {
  std::string k;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "sched=%d prec=%d P=%d dim=%d m=%d nv=%d N=%dx%dx%d S=%dx%dx%d",
                p->sched, p->prec, p->P, p->dim, p->m, p->nv, p->N[0], p->N[1], p->N[2], p->S[0],
                p->S[1], p->S[2]);
  k += buf;
  k += " vel=";
  for (int i = 0; i < p->nv; ++i) {
    for (int a = 0; a < p->dim; ++a) {
      const double v = p->vel[i * p->dim + a];
      k += v > 0 ? '+' : (v < 0 ? '-' : '0');
    }
    k += i + 1 < p->nv ? "," : "";
  }
  std::snprintf(buf, sizeof(buf), " dirichlet=%d%d%d", p->boff[0][0] >= 0, p->boff[1][0] >= 0,
                p->boff[2][0] >= 0);
  k += buf;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    k += " arch=";
    for (const char* c = prop.gcnArchName; *c && *c != ':'; ++c) k += *c;
  } else {
    (void)hipGetLastError();
    k += " arch=?";
  }
  return k;
}

constexpr int kPlanInts = 12;  // kds_plan_t as integers, in field order

void plan_to_ints(const kds_plan_t& pl, int32_t* v) {
  for (int a = 0; a < 3; ++a) { v[a] = pl.Q[a]; v[3 + a] = pl.bw[a]; }
  v[6] = pl.xdirect;
  v[7] = pl.lds_bytes;
  v[8] = pl.step_eager;
  v[9] = pl.relax_vec;
  v[10] = pl.front_kernel;
  v[11] = 0;
}
void plan_from_ints(const int32_t* v, kds_plan_t& pl) {
  for (int a = 0; a < 3; ++a) { pl.Q[a] = v[a]; pl.bw[a] = v[3 + a]; }
  pl.xdirect = v[6];
  pl.lds_bytes = v[7];
  pl.step_eager = v[8];
  pl.relax_vec = v[9];
  pl.front_kernel = v[10];
}

}  // namespace

kds_status kds_tune_subdomains(const kds_config* cfg, const double* W, int32_t reps,
                               int32_t* sub_cells, double* step_ms) {
  if (!cfg || !W || !sub_cells) return fail(nullptr, KDS_E_INVALID, "NULL argument");
  for (int a = 0; a < std::max(1, std::min(3, cfg->dim)); ++a)
    if (!cfg->periodic[a])
      return fail(nullptr, KDS_E_UNSUPPORTED,
                  "kds_tune_subdomains: periodic boxes only (the steps of a Dirichlet problem "
                  "need its boundary data)");
  reps = std::max(1, std::min(reps, 100));
  // one candidate: build, start from W, tune, time reps steps (ms per step,
  // or a negative value if the candidate cannot run)
  auto time_width = [&](const int32_t* S, double* ms) -> kds_status {
    kds_config c = *cfg;
    for (int a = 0; a < 3; ++a) c.sub_cells[a] = S[a];
    kds_problem* p = nullptr;
    kds_status st = kds_create(&c, nullptr, &p);
    *ms = -1.0;
    if (st != KDS_OK) return st;
    st = kds_set_state(p, W, 0);
    if (st == KDS_OK) {
      const kds_status tst = kds_tune(p, reps, nullptr);
      if (tst != KDS_OK && tst != KDS_E_NOMEM && tst != KDS_E_STATE) st = tst;
    }
    if (st == KDS_OK) st = kds_step(p, 1);  // warm-up (captures the step graphs)
    if (st == KDS_OK) st = kds_synchronize(p);
    if (st == KDS_OK) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      hipError_t he = hipEventCreate(&e0);
      if (he == hipSuccess) he = hipEventCreate(&e1);
      if (he == hipSuccess) he = hipEventRecord(e0, p->stream);
      if (he == hipSuccess && (st = kds_step(p, reps)) == KDS_OK) {
        he = hipEventRecord(e1, p->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float f = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&f, e0, e1);
        if (he == hipSuccess) *ms = f / reps;
      }
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (he != hipSuccess) {
        (void)hipGetLastError();
        st = KDS_E_DEVICE;
      }
    }
    kds_destroy(p);
    return st;
  };
  int32_t best[3] = {cfg->sub_cells[0], cfg->sub_cells[1], cfg->sub_cells[2]};
  double best_ms = 0.0;
  {
    const kds_status st = time_width(best, &best_ms);
    if (st != KDS_OK) return st;  // cfg itself must run
  }
  const int dim = std::max(1, std::min(3, cfg->dim));
  for (int a = 0; a < dim; ++a) {
    // the Proposition: max_k |V_k^a| dt <= S h_a
    double vmax = 0.0;
    for (int k = 0; k < cfg->n_vel; ++k) vmax = std::max(vmax, std::fabs(cfg->vel[k * cfg->dim + a]));
    if (vmax == 0.0) continue;
    const double h = (cfg->box_hi[a] - cfg->box_lo[a]) / cfg->n_cells[a];
    const double nu = vmax * cfg->dt / h;
    for (int S = 1; S <= cfg->n_cells[a]; ++S) {
      if (cfg->n_cells[a] % S || S == best[a] || S < nu * (1.0 - 1e-12)) continue;
      int32_t cand[3] = {best[0], best[1], best[2]};
      cand[a] = S;
      double ms = -1.0;
      if (time_width(cand, &ms) != KDS_OK || ms < 0.0) continue;
      if (ms < 0.97 * best_ms) {
        best_ms = ms;
        best[a] = S;
      }
    }
  }
  for (int a = 0; a < 3; ++a) sub_cells[a] = best[a];
  if (step_ms) *step_ms = best_ms;
  return KDS_OK;
}

kds_status kds_tune_cached(kds_problem* p, int32_t reps, const char* path, int32_t* hit) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!path) return fail(p, KDS_E_INVALID, "kds_tune_cached: path is NULL");
  if (hit) *hit = 0;
  const std::string key = plan_key(p);
  // the last line with this key wins (a re-tuned plan is appended)
  bool found = false;
  kds_plan_t cached;
  std::memset(&cached, 0, sizeof(cached));
  if (FILE* fp = std::fopen(path, "r")) {
    char line[1024];
    while (std::fgets(line, sizeof(line), fp)) {
      char* bar = std::strchr(line, '|');
      if (!bar) continue;
      std::string k(line, bar - line);
      while (!k.empty() && k.back() == ' ') k.pop_back();
      if (k != key) continue;
      int32_t v[kPlanInts];
      int n = 0;
      char* q = bar + 1;
      while (n < kPlanInts) {
        char* end = nullptr;
        const long x = std::strtol(q, &end, 10);
        if (end == q) break;
        v[n++] = (int32_t)x;
        q = end;
      }
      if (n == kPlanInts) {
        plan_from_ints(v, cached);
        found = true;
      }
    }
    std::fclose(fp);
  }
  if (found && kds_set_plan(p, &cached) == KDS_OK) {
    if (hit) *hit = 1;
    return KDS_OK;
  }
  kds_status st = kds_tune(p, reps, nullptr);
  if (st != KDS_OK) return st;
  kds_plan_t pl;
  kds_get_plan(p, &pl);
  int32_t v[kPlanInts];
  plan_to_ints(pl, v);
  FILE* fp = std::fopen(path, "a");
  if (!fp) return fail(p, KDS_E_INVALID, std::string("kds_tune_cached: cannot write ") + path);
  std::fprintf(fp, "%s |", key.c_str());
  for (int i = 0; i < kPlanInts; ++i) std::fprintf(fp, " %d", v[i]);
  std::fprintf(fp, "\n");
  const bool ok = std::fclose(fp) == 0;
  if (!ok) return fail(p, KDS_E_INVALID, std::string("kds_tune_cached: cannot write ") + path);
  return KDS_OK;
}

kds_status kds_time_kernels(kds_problem* p, int32_t reps, double* kernel_ms) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!kernel_ms || reps < 1) return fail(p, KDS_E_INVALID, "bad arguments");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_time_kernels needs a state");
  if (p->nbnd > 0 && !p->bnd_set) return fail(p, KDS_E_STATE, "Dirichlet axes: kds_set_boundary first");
  const size_t bytes = (size_t)p->n_unknowns() * p->elem;
  void* save = nullptr;
  if (hipMalloc(&save, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, KDS_E_NOMEM, "kds_time_kernels: no device memory to save the state");
  }
  const Geom& g = p->geom;
  hipError_t e = hipMemcpyAsync(save, p->f, bytes, hipMemcpyDeviceToDevice, p->stream);
  float ms[2] = {0, 0};
  for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
    auto launch = [&]() -> hipError_t {
      if (kind == 0) {
        if (p->sched == KDS_SCHED_FRONT)
          return launch_front_iter(p, p->f, p->fit[1], p->stream);
        if (p->sched == KDS_SCHED_LINE)
          return launch_sweep_line(p->prec, g, p->sweep_blob.data(), p->plan, p->f, p->bnd(),
                                   p->stream);
        // one plain subdomain iteration (the kernel a step launches n_iter times)
        return launch_sweep_plain(p->prec, g, p->sweep_blob.data(), p->f, p->f_tmp, nullptr,
                                  p->tr[0], p->bnd(), p->stream);
      }
      return launch_relax(p->prec, p->law, g, p->eq_dev, p->f, p->f, p->relax_vec, p->stream);
    };
    e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(p->ev[0], p->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(p->ev[1], p->stream);
    if (e == hipSuccess) e = hipEventSynchronize(p->ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[kind], p->ev[0], p->ev[1]);
  }
  hipError_t e2 = hipMemcpyAsync(p->f, save, bytes, hipMemcpyDeviceToDevice, p->stream);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(p->stream);
  (void)hipFree(save);
  if (e != hipSuccess) return hip_fail(p, e, "kds_time_kernels");
  if (e2 != hipSuccess) return hip_fail(p, e2, "kds_time_kernels restore");
  kernel_ms[0] = ms[0] / reps;
  kernel_ms[1] = ms[1] / reps;
  return KDS_OK;
}

kds_status kds_moments(kds_problem* p, double* W_out, int32_t on_device) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!W_out) return fail(p, KDS_E_INVALID, "W_out is NULL");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_moments before kds_set_state");
  const size_t bytes = (size_t)p->plane() * p->m * sizeof(double);
  if (on_device) {
    kds_status st = check_device_ptr(p, W_out);
    if (st != KDS_OK) return st;
    KDS_HIP(p, launch_moments(p->prec, p->geom, p->f, W_out, p->stream));
    KDS_HIP(p, hipStreamSynchronize(p->stream));
  } else {
    kds_status st = ensure_stage(p, bytes);
    if (st != KDS_OK) return st;
    KDS_HIP(p, launch_moments(p->prec, p->geom, p->f, p->stage, p->stream));
    KDS_HIP(p, hipMemcpyAsync(W_out, p->stage, bytes, hipMemcpyDeviceToHost, p->stream));
    KDS_HIP(p, hipStreamSynchronize(p->stream));
  }
  return KDS_OK;
}

kds_status kds_moments_static(kds_problem* p, int64_t node_begin, int64_t node_count,
                              double* W_out) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!W_out) return fail(p, KDS_E_INVALID, "W_out is NULL");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_moments_static before kds_set_state");
  if (node_begin < 0 || node_count < 0 || node_begin > p->plane() ||
      node_count > p->plane() - node_begin)
    return fail(p, KDS_E_INVALID, "kds_moments_static: node range outside the problem's nodes");
  const int64_t max_nodes = (int64_t)(kScratchBytes / (sizeof(double) * (size_t)p->m));
  if (node_count > max_nodes)
    return fail(p, KDS_E_INVALID,
                "kds_moments_static: at most " + std::to_string(max_nodes) +
                    " nodes per call (the static scratch holds " +
                    std::to_string(kScratchBytes >> 20) + " MiB)");
  if (node_count == 0) return KDS_OK;
  if (!p->scratch) return fail(p, KDS_E_DEVICE, "kds_moments_static: no scratch address");
  double* w = static_cast<double*>(p->scratch);
  KDS_HIP(p, launch_moments_range(p->prec, p->geom, p->f, node_begin, node_count, w, p->stream));
  KDS_HIP(p, hipMemcpyAsync(W_out, w, (size_t)node_count * p->m * sizeof(double),
                            hipMemcpyDeviceToHost, p->stream));
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  return KDS_OK;
}

kds_status kds_get_kinetic(kds_problem* p, double* F_out, int32_t on_device) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!F_out) return fail(p, KDS_E_INVALID, "F_out is NULL");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_get_kinetic before kds_set_state");
  const size_t bytes = (size_t)p->n_unknowns() * sizeof(double);
  if (on_device) {
    kds_status st = check_device_ptr(p, F_out);
    if (st != KDS_OK) return st;
    KDS_HIP(p, launch_get_kinetic(p->prec, p->geom, p->f, F_out, p->stream));
  } else {
    kds_status st = ensure_stage(p, bytes);
    if (st != KDS_OK) return st;
    KDS_HIP(p, launch_get_kinetic(p->prec, p->geom, p->f, p->stage, p->stream));
    KDS_HIP(p, hipMemcpyAsync(F_out, p->stage, bytes, hipMemcpyDeviceToHost, p->stream));
  }
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  return KDS_OK;
}

kds_status kds_set_kinetic(kds_problem* p, const double* F, int32_t on_device) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!F) return fail(p, KDS_E_INVALID, "F is NULL");
  const size_t bytes = (size_t)p->n_unknowns() * sizeof(double);
  const double* src = F;
  if (on_device) {
    kds_status st = check_device_ptr(p, F);
    if (st != KDS_OK) return st;
  } else {
    kds_status st = ensure_stage(p, bytes);
    if (st != KDS_OK) return st;
    KDS_HIP(p, hipMemcpyAsync(p->stage, F, bytes, hipMemcpyHostToDevice, p->stream));
    src = p->stage;
  }
  KDS_HIP(p, launch_set_kinetic(p->prec, p->geom, src, p->f, p->stream));
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  p->state_set = true;
  return KDS_OK;
}

kds_status kds_check_finite(kds_problem* p) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_check_finite before kds_set_state");
  int zero = 0, flag = 0;
  KDS_HIP(p, hipMemcpyAsync(p->flag, &zero, sizeof(int), hipMemcpyHostToDevice, p->stream));
  KDS_HIP(p, launch_check_finite(p->prec, p->geom, p->f, p->flag, p->stream));
  KDS_HIP(p, hipMemcpyAsync(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  if (flag) return fail(p, KDS_E_NONFINITE, "kinetic state holds NaN or Inf");
  return KDS_OK;
}

kds_status kds_trace_residual(kds_problem* p, double* out) {
  if (!p || !out) return fail(p, KDS_E_INVALID, "NULL argument");
  if (!p->state_set) return fail(p, KDS_E_STATE, "kds_trace_residual before kds_set_state");
  if (p->nbnd > 0 && !p->bnd_set)
    return fail(p, KDS_E_STATE, "Dirichlet axes: kds_set_boundary before kds_trace_residual");
  const Geom& g = p->geom;
  if (p->K == 0) {  // the converged iteration: no residual
    out[0] = 0.0;
    out[1] = -1.0;
    return KDS_OK;
  }
  if (p->sched == KDS_SCHED_FRONT) {
    // the front schedule's own iterates 1 .. K into its iterate buffers (the
    // state is not changed), then the change between the last two over the
    // subdomains' outflow faces
    unsigned long long* red = nullptr;
    if (hipMalloc((void**)&red, 16) != hipSuccess) {
      (void)hipGetLastError();
      return fail(p, KDS_E_NOMEM, "kds_trace_residual: no device memory");
    }
    hipError_t e = hipMemsetAsync(red, 0, 16, p->stream);
    for (int it = 1; it <= p->K && e == hipSuccess; ++it)
      e = launch_front_iter(p, it == 1 ? p->f : p->fit[(it - 1) & 1], p->fit[it & 1], p->stream);
    if (e == hipSuccess)
      e = launch_max_absdiff_outflow(p->prec, p->fit[p->K & 1],
                                     p->K == 1 ? p->f : p->fit[(p->K - 1) & 1], g, p->front, red,
                                     p->stream);
    unsigned long long bits[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(bits, red, 16, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(red);
    if (e != hipSuccess) return hip_fail(p, e, "kds_trace_residual");
    std::memcpy(&out[0], &bits[0], 8);
    std::memcpy(&out[1], &bits[1], 8);
    return KDS_OK;
  }
  if (p->sweep_blob.empty())
    return fail(p, KDS_E_UNSUPPORTED, "kds_trace_residual: no sweep table for this problem");
  // two trace sets, zeroed (entries no velocity uses stay 0 in both), and the
  // two reduction words
  const int64_t n = g.tr_stride * (int64_t)p->nv * p->m;
  const size_t bytes = (size_t)n * p->elem;
  unsigned char* buf = nullptr;
  if (hipMalloc((void**)&buf, 2 * bytes + 16) != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, KDS_E_NOMEM, "kds_trace_residual: no device memory for the traces");
  }
  void* tr[2] = {buf, buf + bytes};
  unsigned long long* red = (unsigned long long*)(buf + 2 * bytes);
  hipError_t e = hipMemsetAsync(buf, 0, 2 * bytes + 16, p->stream);
  // iterates 1 .. K of the sweep from the current state (the state itself
  // is not changed); with K = 1 the other set is iterate 0, the state's own
  // traces
  if (e == hipSuccess && p->K == 1)
    e = launch_trace_iterate0(p->prec, g, p->sweep_blob.data(), p->f, tr[0], p->stream);
  for (int it = 1; it <= p->K && e == hipSuccess; ++it)
    e = launch_sweep_plain(p->prec, g, p->sweep_blob.data(), p->f, nullptr,
                           it == 1 ? nullptr : tr[(it - 1) & 1], tr[it & 1], p->bnd(), p->stream);
  if (e == hipSuccess)
    e = launch_max_absdiff(p->prec, tr[p->K & 1], tr[(p->K - 1) & 1], n, red, p->stream);
  unsigned long long bits[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(bits, red, 16, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(p, e, "kds_trace_residual");
  std::memcpy(&out[0], &bits[0], 8);
  std::memcpy(&out[1], &bits[1], 8);
  return KDS_OK;
}

kds_status kds_synchronize(kds_problem* p) {
  if (!p) return fail(nullptr, KDS_E_INVALID, "problem is NULL");
  KDS_HIP(p, hipStreamSynchronize(p->stream));
  return KDS_OK;
}

kds_status kds_info(const kds_problem* p, kds_info_t* info) {
  if (!p || !info) return fail(nullptr, KDS_E_INVALID, "NULL argument");
  info->n_unknowns = p->n_unknowns();
  info->state_bytes = (int64_t)p->n_unknowns() * (int64_t)p->elem;
  info->schedule = p->sched;
  info->precision = p->prec;
  info->steps_done = p->steps_done;
  info->max_kinetic_courant = p->max_nu;
  info->min_subdomain_width = p->min_sub_width;
  info->proposition_ok = p->proposition_ok ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    info->line_Q[a] = p->sched == KDS_SCHED_LINE ? p->line_Q[a] : 0;
    info->line_bw[a] = p->sched == KDS_SCHED_LINE ? p->line_bw[a] : 0;
  }
  info->tuned = p->tuned ? 1 : 0;
  info->step_eager = p->eager_steps ? 1 : 0;
  info->relax_vec = p->relax_vec ? 1 : 0;
  info->line_xdirect = p->sched == KDS_SCHED_LINE ? p->plan.xdirect : 0;
  info->line_qmax = p->sched == KDS_SCHED_LINE ? line_qmax((int)p->elem, p->nn) : 0;
  info->line_lds_bytes =
      p->sched == KDS_SCHED_LINE
          ? (int32_t)(std::max(p->plan.lds_elems, p->plan.lds_alloc) * (int)p->elem)
          : 0;
  info->eq_monotone = p->eq_monotone;
  info->eq_min_eig = p->eq_min_eig;
  info->max_wave_speed = p->wave_speed;
  info->subchar_ok = p->wave_speed < 0.0 ? -1 : (p->min_speed > p->wave_speed ? 1 : 0);
  return KDS_OK;
}

void kds_destroy(kds_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  free_device(p);
  delete p;
}

const char* kds_last_error(const kds_problem* p) {
  return p ? p->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ================================================================ batches
// Many problems advanced together.  The line-schedule members that share
// (precision, degree, dimension, workgroup size, law, m, n_vel, periodic or
// Dirichlet) form a branch: ONE launch sweeps all of them (workgroups spread
// over the members), ONE launch relaxes them.  Branches touch disjoint memory
// and run as parallel branches of one captured HIP graph per step.  Front-
// schedule members on the wave kernel form branches of their own (one launch
// per subdomain iteration, one relaxation).  Plain-schedule members and front
// members on the workgroup kernel add their own kernel sequences on one more
// branch.  (A Dirichlet member's records point at its two boundary halves,
// which kds_set_boundary refills in place between steps; the batch step
// advances them as a member's own step does.)

struct kds_batch {
  struct Branch {
    int prec = 0, P = 0, dim = 0, threads = 0, law = 0, m = 0, nv = 0;
    bool rounds = false;  // members whose lanes stream their cells in rounds
    bool dir = false;     // members with Dirichlet axes
    std::vector<kds_problem*> members;
    size_t lds_elems = 0;
    std::vector<unsigned char> line_tasks, relax_tasks;  // packed records (host)
    std::vector<int64_t> line_start{0}, relax_start{0};  // block prefixes
    void* d_line = nullptr;
    void* d_relax = nullptr;
    int64_t* d_line_start = nullptr;
    int64_t* d_relax_start = nullptr;
    int ntask() const { return (int)line_start.size() - 1; }
  };
  // front-schedule members on the wave kernel that share (form, dimension,
  // degree, subdomain iterations, law, m, n_vel): one launch per iteration,
  // one relaxation launch
  struct FrontBranch {
    int prec = 0, mode = 0, dim = 0, P = 0, K = 0, law = 0, m = 0, nv = 0;
    Geom g{};             // the first member's (the kernel shape)
    size_t lds = 0;       // largest LDS of the members
    std::vector<kds_problem*> members;
    std::vector<std::vector<unsigned char>> it_tasks;  // per iteration 1..K (host)
    std::vector<unsigned char> relax_tasks;
    std::vector<int64_t> start{0}, relax_start{0};
    std::vector<void*> d_it;
    void* d_relax = nullptr;
    int64_t* d_start = nullptr;
    int64_t* d_relax_start = nullptr;
    int ntask() const { return (int)start.size() - 1; }
  };
  std::vector<kds_problem*> probs;
  std::vector<int> versions;
  std::vector<Branch> branches;
  std::vector<FrontBranch> fronts;
  int bw_mul = 1;  // line members' bundles widened this much in the batch (kds_batch_tune)
  std::vector<kds_problem*> others;  // members on the extra branch
  int device = 0;
  hipStream_t stream = nullptr;      // the batch's stream (branch 0 when captured)
  std::vector<hipStream_t> sides;    // capture streams of the other branches
  std::vector<hipEvent_t> joins;     // one per side stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::string err;
};

namespace {

kds_status bfail(kds_batch* b, kds_status st, const std::string& msg) {
  if (b) b->err = msg; else g_create_error = msg;
  return st;
}

#define KDS_BHIP(b, call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail((b), KDS_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

void batch_free_branches(kds_batch* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
  for (auto& br : b->branches) {
    void* bufs[] = {br.d_line, br.d_relax, br.d_line_start, br.d_relax_start};
    for (void* x : bufs)
      if (x) (void)hipFree(x);
  }
  for (auto& fb : b->fronts) {
    for (void* x : fb.d_it)
      if (x) (void)hipFree(x);
    void* bufs[] = {fb.d_relax, fb.d_start, fb.d_relax_start};
    for (void* x : bufs)
      if (x) (void)hipFree(x);
  }
  b->branches.clear();
  b->fronts.clear();
  b->others.clear();
}

hipError_t upload(void** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

// Group the members into branches and upload the task tables (blocking copies).
kds_status batch_build(kds_batch* b) {
  batch_free_branches(b);
  for (kds_problem* p : b->probs) {
    if (p->sched == KDS_SCHED_FRONT && p->front_wave && front_wave_ok(p)) {
      // front members on the wave kernel: grouped by their kernel and step
      const size_t rb = relax_task_bytes(p->law, p->dim, p->m, p->nv);
      if (rb == 0) return bfail(b, KDS_E_UNSUPPORTED, "no batched relaxation for a member's law");
      kds_batch::FrontBranch* fb = nullptr;
      for (auto& x : b->fronts)
        if (x.prec == p->prec && x.mode == p->front_mode && x.dim == p->dim && x.P == p->P &&
            x.K == p->K && x.law == p->law && x.m == p->m && x.nv == p->nv)
          fb = &x;
      if (!fb) {
        b->fronts.emplace_back();
        fb = &b->fronts.back();
        fb->prec = p->prec;
        fb->mode = p->front_mode;
        fb->dim = p->dim;
        fb->P = p->P;
        fb->K = p->K;
        fb->law = p->law;
        fb->m = p->m;
        fb->nv = p->nv;
        fb->g = p->geom;
        fb->it_tasks.resize(p->K);
      }
      fb->members.push_back(p);
      const size_t tb = front_wave_task_bytes(p->prec);
      for (int it = 1; it <= p->K; ++it) {
        const void* f_prev = it == 1 ? p->f : p->fit[(it - 1) & 1];
        auto& t = fb->it_tasks[it - 1];
        const size_t off = t.size();
        t.resize(off + tb);
        pack_front_wave_task(p->prec, p->geom, p->front, p->front_W, p->front_lvl_start,
                             p->front_desc, p->front_ndesc, p->f, f_prev, p->fit[it & 1], p->bnd(),
                             t.data() + off);
      }
      fb->start.push_back(fb->start.back() + front_wave_blocks(p->geom, p->front));
      fb->lds = std::max(fb->lds, front_wave_lds_bytes(p->geom, p->front, p->prec));
      const size_t off = fb->relax_tasks.size();
      fb->relax_tasks.resize(off + rb);
      pack_relax_task(p->law, p->dim, p->m, p->nv, p->eq_blob.data(), p->fit[p->K & 1], p->f,
                      p->plane(), fb->relax_tasks.data() + off);
      fb->relax_start.push_back(fb->relax_start.back() + (p->plane() + 255) / 256);
      continue;
    }
    // plain-schedule members, and front members on the workgroup kernel,
    // keep their own kernel sequences
    if (p->sched != KDS_SCHED_LINE) {
      b->others.push_back(p);
      continue;
    }
    const Geom& g = p->geom;
    // the member's plan, with its bundles widened by bw_mul where the cells
    // per lane allow it (the same lines and lane arithmetic, fewer and
    // larger workgroups)
    LinePlan pl = p->plan;
    if (b->bw_mul > 1) {
      int tq[3], tb[3];
      for (int a = 0; a < 3; ++a) {
        tq[a] = p->line_Q[a];
        tb[a] = p->line_bw[a];
        if (tq[a] <= 0) continue;
        for (int w = tb[a] * b->bw_mul; w > tb[a]; --w)
          if (line_choice_ok(p, a, tq[a], w)) {
            tb[a] = w;
            break;
          }
      }
      LinePlan np;
      if (finalize_plan(p, tq, tb, np)) {
        np.xdirect = p->plan.xdirect;
        pl = np;
      }
    }
    const bool rounds = line_plan_rounds(g, pl, (int)p->elem);
    const bool dir = p->nbnd > 0;
    kds_batch::Branch* br = nullptr;
    for (auto& x : b->branches)
      if (x.prec == p->prec && x.P == p->P && x.dim == p->dim && x.threads == pl.threads &&
          x.law == p->law && x.m == p->m && x.nv == p->nv && x.rounds == rounds && x.dir == dir)
        br = &x;
    if (!br) {
      b->branches.emplace_back();
      br = &b->branches.back();
      br->prec = p->prec;
      br->P = p->P;
      br->dim = p->dim;
      br->threads = pl.threads;
      br->law = p->law;
      br->m = p->m;
      br->nv = p->nv;
      br->rounds = rounds;
      br->dir = dir;
    }
    const size_t lb = line_task_bytes(p->prec);
    const size_t rb = relax_task_bytes(p->law, p->dim, p->m, p->nv);
    if (rb == 0) return bfail(b, KDS_E_UNSUPPORTED, "no batched relaxation for a member's law");
    br->members.push_back(p);
    size_t off = br->line_tasks.size();
    br->line_tasks.resize(off + lb);
    pack_line_task(p->prec, p->f, g, p->sweep_blob.data(), pl, p->bnd(),
                   br->line_tasks.data() + off);
    br->line_start.push_back(br->line_start.back() + pl.block_start[g.nv * g.m]);
    br->lds_elems = std::max(br->lds_elems, (size_t)std::max(pl.lds_elems, pl.lds_alloc));
    off = br->relax_tasks.size();
    br->relax_tasks.resize(off + rb);
    pack_relax_task(p->law, p->dim, p->m, p->nv, p->eq_blob.data(), p->f, p->f, p->plane(),
                    br->relax_tasks.data() + off);
    br->relax_start.push_back(br->relax_start.back() + (p->plane() + 255) / 256);
  }
  for (auto& br : b->branches) {
    if (br.line_start.back() > 0x7fffffffLL || br.relax_start.back() > 0x7fffffffLL)
      return bfail(b, KDS_E_UNSUPPORTED, "batched launch exceeds the grid limit");
    int cap = 64 * 1024;
    for (kds_problem* p : b->probs) cap = std::max(cap, p->lds_cap);
    if (br.lds_elems * (br.prec == KDS_FP64 ? 8 : 4) > (size_t)cap)
      return bfail(b, KDS_E_UNSUPPORTED, "batched line sweep needs more LDS than the device has");
    hipError_t e = upload(&br.d_line, br.line_tasks.data(), br.line_tasks.size());
    if (e == hipSuccess) e = upload(&br.d_relax, br.relax_tasks.data(), br.relax_tasks.size());
    if (e == hipSuccess)
      e = upload((void**)&br.d_line_start, br.line_start.data(), br.line_start.size() * 8);
    if (e == hipSuccess)
      e = upload((void**)&br.d_relax_start, br.relax_start.data(), br.relax_start.size() * 8);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, e == hipErrorOutOfMemory ? KDS_E_NOMEM : KDS_E_DEVICE,
                   std::string("batch task tables: ") + hipGetErrorString(e));
    }
  }
  for (auto& fb : b->fronts) {
    if (fb.start.back() > 0x7fffffffLL || fb.relax_start.back() > 0x7fffffffLL)
      return bfail(b, KDS_E_UNSUPPORTED, "batched launch exceeds the grid limit");
    hipError_t e = hipSuccess;
    fb.d_it.assign(fb.K, nullptr);
    for (int it = 0; it < fb.K && e == hipSuccess; ++it)
      e = upload(&fb.d_it[it], fb.it_tasks[it].data(), fb.it_tasks[it].size());
    if (e == hipSuccess) e = upload((void**)&fb.d_start, fb.start.data(), fb.start.size() * 8);
    if (e == hipSuccess) e = upload(&fb.d_relax, fb.relax_tasks.data(), fb.relax_tasks.size());
    if (e == hipSuccess)
      e = upload((void**)&fb.d_relax_start, fb.relax_start.data(), fb.relax_start.size() * 8);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, e == hipErrorOutOfMemory ? KDS_E_NOMEM : KDS_E_DEVICE,
                   std::string("batch task tables: ") + hipGetErrorString(e));
    }
  }
  // capture streams for the branches beyond the first
  const size_t ngrouped = b->branches.size() + b->fronts.size();
  const size_t nside = ngrouped - (ngrouped ? 1 : 0) + (b->others.empty() ? 0 : 1);
  while (b->sides.size() < nside) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    KDS_BHIP(b, hipStreamCreate(&st));
    b->sides.push_back(st);
    KDS_BHIP(b, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->joins.push_back(ev);
  }
  for (size_t i = 0; i < b->probs.size(); ++i) b->versions[i] = b->probs[i]->plan_version;
  return KDS_OK;
}

hipError_t launch_branch_line(const kds_batch::Branch& br, hipStream_t s) {
  return launch_sweep_line_batch(br.prec, br.P, br.dim, br.rounds, br.dir, br.d_line,
                                 br.d_line_start, br.ntask(), br.line_start.back(), br.threads,
                                 br.lds_elems, s);
}

hipError_t launch_front_branch_iter(const kds_batch::FrontBranch& fb, int it, hipStream_t s) {
  return launch_sweep_front_wave_batch(fb.prec, fb.mode, fb.g, fb.d_it[it], fb.d_start,
                                       fb.ntask(), fb.start.back(), fb.lds, s);
}

hipError_t launch_front_branch_relax(const kds_batch::FrontBranch& fb, hipStream_t s) {
  return launch_relax_batch(fb.prec, fb.law, fb.dim, fb.m, fb.nv, fb.d_relax, fb.d_relax_start,
                            fb.ntask(), fb.relax_start.back(), s);
}

hipError_t launch_branch_relax(const kds_batch::Branch& br, hipStream_t s) {
  return launch_relax_batch(br.prec, br.law, br.dim, br.m, br.nv, br.d_relax, br.d_relax_start,
                            br.ntask(), br.relax_start.back(), s);
}

// One batched step, under stream capture: fork every side stream from the
// batch stream, enqueue each branch on its stream, join them back.
kds_status batch_enqueue(kds_batch* b) {
  const size_t nb = b->branches.size(), nf = b->fronts.size();
  std::vector<hipStream_t> bs;
  bs.push_back(b->stream);
  for (hipStream_t s : b->sides) bs.push_back(s);
  const size_t nstreams = (nb + nf ? nb + nf : 1) + (b->others.empty() ? 0 : 1);
  if (nstreams > 1) {
    KDS_BHIP(b, hipEventRecord(b->ev_fork, b->stream));
    for (size_t i = 1; i < nstreams; ++i) KDS_BHIP(b, hipStreamWaitEvent(bs[i], b->ev_fork, 0));
  }
  for (size_t i = 0; i < nb; ++i) {
    const kds_batch::Branch& br = b->branches[i];
    KDS_BHIP(b, launch_branch_line(br, bs[i]));
    KDS_BHIP(b, launch_branch_relax(br, bs[i]));
    // the boundary data at the end of the step are the start data of the
    // next, as in a member's own step
    if (br.dir)
      for (kds_problem* p : br.members) {
        const BndArgs bd = p->bnd();
        KDS_BHIP(b, launch_copy(p->prec, bd.neu, p->fb, p->bnd_half(), bs[i]));
      }
  }
  for (size_t j = 0; j < nf; ++j) {
    const kds_batch::FrontBranch& fb = b->fronts[j];
    hipStream_t s = bs[nb + j];
    for (int it = 0; it < fb.K; ++it)
      KDS_BHIP(b, launch_front_branch_iter(fb, it, s));
    KDS_BHIP(b, launch_front_branch_relax(fb, s));
    for (kds_problem* p : fb.members)
      if (p->nbnd > 0) {
        const BndArgs bd = p->bnd();
        KDS_BHIP(b, launch_copy(p->prec, bd.neu, p->fb, p->bnd_half(), s));
      }
  }
  if (!b->others.empty()) {
    hipStream_t s = bs[nstreams - 1];
    for (kds_problem* p : b->others) {
      kds_status st = enqueue_step(p, false, s);
      if (st != KDS_OK) return bfail(b, st, "batch member: " + p->err);
    }
  }
  for (size_t i = 1; i < nstreams; ++i) {
    KDS_BHIP(b, hipEventRecord(b->joins[i - 1], bs[i]));
    KDS_BHIP(b, hipStreamWaitEvent(b->stream, b->joins[i - 1], 0));
  }
  return KDS_OK;
}

kds_status batch_prepare(kds_batch* b) {
  for (kds_problem* p : b->probs) {
    if (!p->state_set) return bfail(b, KDS_E_STATE, "a batch member has no state");
    if (p->nbnd > 0 && !p->bnd_set)
      return bfail(b, KDS_E_STATE, "a batch member has Dirichlet axes but no boundary data");
  }
  bool stale = b->branches.empty() && b->fronts.empty() && b->others.empty();
  for (size_t i = 0; i < b->probs.size(); ++i)
    if (b->versions[i] != b->probs[i]->plan_version) stale = true;
  if (stale) {
    kds_status st = batch_build(b);
    if (st != KDS_OK) return st;
  }
  if (!b->graph_exec) {
    KDS_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    kds_status st = batch_enqueue(b);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != KDS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    KDS_BHIP(b, e);
    b->graph = graph;
    KDS_BHIP(b, hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
  }
  return KDS_OK;
}

// Order the batch stream after every member stream (work queued there before
// the batch step), and every member stream after the batch stream.
kds_status batch_join_in(kds_batch* b) {
  for (kds_problem* p : b->probs) {
    if (p->stream == b->stream) continue;
    KDS_BHIP(b, hipEventRecord(b->ev_join, p->stream));
    KDS_BHIP(b, hipStreamWaitEvent(b->stream, b->ev_join, 0));
  }
  return KDS_OK;
}

kds_status batch_join_out(kds_batch* b, int32_t n_steps) {
  KDS_BHIP(b, hipEventRecord(b->ev_join, b->stream));
  for (kds_problem* p : b->probs) {
    if (p->stream != b->stream) KDS_BHIP(b, hipStreamWaitEvent(p->stream, b->ev_join, 0));
    p->steps_done += n_steps;
  }
  return KDS_OK;
}

}  // namespace

extern "C" {

kds_status kds_batch_create(kds_problem* const* problems, int32_t n, kds_batch** out) {
  if (!out) return bfail(nullptr, KDS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!problems || n < 1) return bfail(nullptr, KDS_E_INVALID, "need at least one problem");
  for (int i = 0; i < n; ++i) {
    if (!problems[i]) return bfail(nullptr, KDS_E_INVALID, "a problem is NULL");
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i])
        return bfail(nullptr, KDS_E_INVALID, "a problem appears twice in the batch");
    if (problems[i]->device != problems[0]->device)
      return bfail(nullptr, KDS_E_INVALID, "batch members must live on one device");
  }
  kds_batch* b = new kds_batch();
  b->probs.assign(problems, problems + n);
  b->versions.assign(n, -1);
  b->device = problems[0]->device;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess) e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipStreamCreate(&b->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&b->ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&b->ev[1]);
  kds_status st = KDS_OK;
  if (e != hipSuccess) st = bfail(nullptr, KDS_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
  if (st == KDS_OK) {
    st = batch_build(b);
    if (st != KDS_OK) g_create_error = b->err;
  }
  (void)hipSetDevice(cur);
  if (st != KDS_OK) {
    kds_batch_destroy(b);
    return st;
  }
  *out = b;
  return KDS_OK;
}

kds_status kds_batch_step(kds_batch* b, int32_t n_steps) {
  if (!b) return bfail(nullptr, KDS_E_INVALID, "batch is NULL");
  if (n_steps < 0) return bfail(b, KDS_E_INVALID, "n_steps must be >= 0");
  kds_status st = batch_prepare(b);
  if (st != KDS_OK || n_steps == 0) return st;
  if ((st = batch_join_in(b)) != KDS_OK) return st;
  for (int i = 0; i < n_steps; ++i) KDS_BHIP(b, hipGraphLaunch(b->graph_exec, b->stream));
  return batch_join_out(b, n_steps);
}

kds_status kds_batch_step_timed(kds_batch* b, int32_t n_steps, double* ms) {
  if (!b) return bfail(nullptr, KDS_E_INVALID, "batch is NULL");
  if (n_steps < 1 || !ms) return bfail(b, KDS_E_INVALID, "bad arguments");
  kds_status st = batch_prepare(b);
  if (st != KDS_OK) return st;
  if ((st = batch_join_in(b)) != KDS_OK) return st;
  KDS_BHIP(b, hipEventRecord(b->ev[0], b->stream));
  for (int i = 0; i < n_steps; ++i) KDS_BHIP(b, hipGraphLaunch(b->graph_exec, b->stream));
  KDS_BHIP(b, hipEventRecord(b->ev[1], b->stream));
  KDS_BHIP(b, hipEventSynchronize(b->ev[1]));
  float t = 0;
  KDS_BHIP(b, hipEventElapsedTime(&t, b->ev[0], b->ev[1]));
  *ms = t;
  return batch_join_out(b, n_steps);
}

kds_status kds_batch_time_kernels(kds_batch* b, int32_t reps, double* kernel_ms) {
  if (!b) return bfail(nullptr, KDS_E_INVALID, "batch is NULL");
  if (!kernel_ms || reps < 1) return bfail(b, KDS_E_INVALID, "bad arguments");
  kds_status st = batch_prepare(b);
  if (st != KDS_OK) return st;
  if ((st = batch_join_in(b)) != KDS_OK) return st;
  // the grouped kernels update their members' states in place: save them
  std::vector<kds_problem*> grouped;
  for (auto& br : b->branches) grouped.insert(grouped.end(), br.members.begin(), br.members.end());
  for (auto& fb : b->fronts) grouped.insert(grouped.end(), fb.members.begin(), fb.members.end());
  size_t total = 0;
  for (kds_problem* p : grouped) total += (size_t)p->n_unknowns() * p->elem;
  unsigned char* save = nullptr;
  if (total && hipMalloc((void**)&save, total) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, KDS_E_NOMEM, "kds_batch_time_kernels: no device memory to save the states");
  }
  hipError_t e = hipSuccess;
  size_t off = 0;
  for (kds_problem* p : grouped)
    if (e == hipSuccess) {
      const size_t n = (size_t)p->n_unknowns() * p->elem;
      e = hipMemcpyAsync(save + off, p->f, n, hipMemcpyDeviceToDevice, b->stream);
      off += n;
    }
  float ms[2] = {0, 0};
  const size_t nb = b->branches.size(), ng = nb + b->fronts.size();
  for (int kind = 0; kind < 2 && e == hipSuccess; ++kind)
    for (size_t i = 0; i < ng; ++i) {
      if (e != hipSuccess) break;
      // (a front group: all its subdomain iterations per repetition)
      auto launch = [&]() -> hipError_t {
        if (i < nb)
          return kind == 0 ? launch_branch_line(b->branches[i], b->stream)
                           : launch_branch_relax(b->branches[i], b->stream);
        const kds_batch::FrontBranch& fb = b->fronts[i - nb];
        if (kind == 1) return launch_front_branch_relax(fb, b->stream);
        hipError_t r = hipSuccess;
        for (int it = 0; it < fb.K && r == hipSuccess; ++it)
          r = launch_front_branch_iter(fb, it, b->stream);
        return r;
      };
      e = launch();  // warm-up
      if (e == hipSuccess) e = hipEventRecord(b->ev[0], b->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
      if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
      float t = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, b->ev[0], b->ev[1]);
      ms[kind] += t / reps;
    }
  off = 0;
  hipError_t e2 = hipSuccess;
  for (kds_problem* p : grouped)
    if (e2 == hipSuccess) {
      const size_t n = (size_t)p->n_unknowns() * p->elem;
      e2 = hipMemcpyAsync(p->f, save + off, n, hipMemcpyDeviceToDevice, b->stream);
      off += n;
    }
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(b->stream);
  if (save) (void)hipFree(save);
  if (e != hipSuccess) return bfail(b, KDS_E_DEVICE, std::string("kds_batch_time_kernels: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return bfail(b, KDS_E_DEVICE, std::string("kds_batch_time_kernels restore: ") + hipGetErrorString(e2));
  kernel_ms[0] = ms[0];
  kernel_ms[1] = ms[1];
  return batch_join_out(b, 0);
}

kds_status kds_batch_tune(kds_batch* b, int32_t reps, double* best_ms) {
  if (!b) return bfail(nullptr, KDS_E_INVALID, "batch is NULL");
  if (reps < 1) return bfail(b, KDS_E_INVALID, "reps must be >= 1");
  reps = std::min(reps, 100);
  kds_status st = batch_prepare(b);
  if (st != KDS_OK) return st;
  if ((st = batch_join_in(b)) != KDS_OK) return st;
  // every member's state (and boundary data, which a step advances) is
  // saved: the timed steps run the whole batch
  size_t total = 0;
  for (kds_problem* p : b->probs)
    total += ((size_t)p->n_unknowns() + (p->nbnd > 0 ? 2 * (size_t)p->bnd_half() : 0)) * p->elem;
  unsigned char* save = nullptr;
  if (hipMalloc((void**)&save, total) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, KDS_E_NOMEM, "kds_batch_tune: no device memory to save the states");
  }
  auto copy_states = [&](bool to_save) -> hipError_t {
    size_t off = 0;
    hipError_t e = hipSuccess;
    auto one = [&](void* buf, size_t n) {
      if (e == hipSuccess)
        e = to_save ? hipMemcpyAsync(save + off, buf, n, hipMemcpyDeviceToDevice, b->stream)
                    : hipMemcpyAsync(buf, save + off, n, hipMemcpyDeviceToDevice, b->stream);
      off += n;
    };
    for (kds_problem* p : b->probs) {
      one(p->f, (size_t)p->n_unknowns() * p->elem);
      if (p->nbnd > 0) one(p->fb, 2 * (size_t)p->bnd_half() * p->elem);
    }
    return e;
  };
  hipError_t e = copy_states(true);
  const int mul0 = b->bw_mul;
  int best_mul = mul0;
  double best = -1.0;
  for (int mul : {1, 2, 4}) {
    if (e != hipSuccess) break;
    b->bw_mul = mul;
    if ((st = batch_build(b)) != KDS_OK || (st = batch_prepare(b)) != KDS_OK) break;
    e = copy_states(false);
    // one untimed step, then reps (the members' step counts do not move)
    if (e == hipSuccess) e = hipGraphLaunch(b->graph_exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev[0], b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->graph_exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, b->ev[0], b->ev[1]);
    if (e == hipSuccess && (best < 0.0 || t / reps < 0.97 * best)) {
      best = t / reps;
      best_mul = mul;
    }
  }
  hipError_t e2 = copy_states(false);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(b->stream);
  (void)hipFree(save);
  // keep the fastest choice (the one before the search if the search failed)
  b->bw_mul = (st == KDS_OK && e == hipSuccess) ? best_mul : mul0;
  const kds_status st2 = batch_build(b);
  if (st != KDS_OK) return st;
  if (e != hipSuccess) return bfail(b, KDS_E_DEVICE, std::string("kds_batch_tune: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return bfail(b, KDS_E_DEVICE, std::string("kds_batch_tune restore: ") + hipGetErrorString(e2));
  if (st2 != KDS_OK) return st2;
  if (best_ms) *best_ms = best;
  return batch_join_out(b, 0);
}

kds_status kds_batch_synchronize(kds_batch* b) {
  if (!b) return bfail(nullptr, KDS_E_INVALID, "batch is NULL");
  KDS_BHIP(b, hipStreamSynchronize(b->stream));
  return KDS_OK;
}

void kds_batch_destroy(kds_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_free_branches(b);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto e : b->joins) (void)hipEventDestroy(e);
  for (auto st : b->sides) (void)hipStreamDestroy(st);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* kds_batch_last_error(const kds_batch* b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
