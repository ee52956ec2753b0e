/* kds.h -- C ABI of libkds, the MI355X (gfx950) kinetic DG time step.
 *
 * Method: Gerhard, Helluy, Michel-Dansac, Weber, "Parallel kinetic schemes
 * for conservation laws, with large time steps" (arXiv:2212.11010).
 *
 *   A system of m conservation laws in d dimensions (Sec. 2.1, eq:conslaw) is
 *   represented by n_vel vectorial kinetic functions F_k transported at
 *   constant velocities V_k, with W = sum_k F_k and equilibria M_k(W) that
 *   satisfy the moment conditions (eq:maxwell_def).  One time step (Sec. 2.2)
 *   transports every F_k for dt with the implicit upwind DG scheme (Sec. 3.1,
 *   eq:dg_imp; theta-scheme, Crank-Nicolson by default), solved by downwind
 *   sweeps inside subdomains (Sec. 3.2) coupled by the iterative subdomain
 *   algorithm of Sec. 5.1 (eq:ibvp, n_iter iterations), and then applies the
 *   over-relaxation F_k <- F_k + omega (M_k(W) - F_k) (eq:over_relaxation).
 *
 * Discretisation: Cartesian box, n_cells[a] uniform cells per axis, periodic
 * or with Dirichlet ends per axis, tensor Gauss-Lobatto nodal basis of degree p
 * ((p+1)^d nodes per cell), collocated Gauss-Lobatto quadrature.  Subdomains
 * are boxes of sub_cells[a] cells.  Periodic wrap faces are always subdomain
 * interfaces.
 *
 * Conventions for every call:
 *   - Status codes only; no exception or abort crosses the ABI.  After an
 *     error, kds_last_error() returns a message (for kds_create failures,
 *     call kds_last_error(NULL): a thread-local message).
 *   - Input arrays are read during the call; the caller keeps ownership.
 *     Output arrays are caller-allocated.
 *   - on_device = 1: the pointer is device memory on the problem's GPU, and
 *     the transfer is ordered on the problem's stream (the call returns after
 *     the stream has finished with the buffer).  on_device = 0: host memory.
 *   - Cells are numbered x-fastest; nodes inside a cell x-fastest; the
 *     component index is the fastest in W, F arrays.
 *   - A problem is not thread safe; distinct problems are independent.
 *   - The library allocates its own device memory (hipMalloc) in kds_create
 *     and frees it in kds_destroy.
 */
#ifndef KDS_H
#define KDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kds_problem kds_problem; /* opaque, library-owned */

typedef enum {
  KDS_OK = 0,
  KDS_E_INVALID = 1,     /* argument or configuration rejected */
  KDS_E_NOMEM = 2,       /* device allocation failed or would not fit */
  KDS_E_DEVICE = 3,      /* a HIP runtime call failed */
  KDS_E_STATE = 4,       /* call out of order (e.g. step before set_state) */
  KDS_E_NONFINITE = 5,   /* NaN/Inf found by kds_check_finite */
  KDS_E_UNSUPPORTED = 6  /* valid for the method, not implemented here */
} kds_status;

typedef enum {
  KDS_LAW_LINEAR = 0, /* Q^i(W) = A^i W; law_params = A^1..A^d, each m*m row-major */
  KDS_LAW_EULER = 1   /* compressible Euler, m = d + 2, W = (rho, rho u, E);
                         law_params = {gamma} */
} kds_law;

typedef enum {
  KDS_FP64 = 0,            /* transport and storage in FP64 */
  KDS_FP32 = 1,            /* transport and storage in FP32; W and M_k in FP64;
                              the front schedule multiplies on FP32 matrix cores */
  KDS_FP32_SPLIT_F16 = 2,  /* FP32 storage; front-schedule cell solves as three
                              FP16 matrix-core products (hi*hi + hi*lo + lo*hi) */
  KDS_FP32_SPLIT_BF16 = 3  /* same with BF16 halves */
} kds_prec;

typedef enum {
  KDS_SCHED_AUTO = 0,  /* the line schedule when the shape allows it (every grid
                          line along a velocity fits one wavefront: at most
                          64 x Q_max cells, Q_max = 8 for up to 8 nodes per
                          cell, 4 for up to 16, else 2), else plain */
  KDS_SCHED_PLAIN = 1, /* literal sweep: one launch per subdomain iteration,
                          one thread per (velocity, component, line, subdomain)
                          walking its cells in downwind order */
  KDS_SCHED_LINE = 2,  /* all n_iter subdomain iterations of a whole grid line
                          resolved in one pass by one wavefront (exact
                          reformulation, see kds_step) */
  KDS_SCHED_FRONT = 3  /* velocities in any direction: cells of a subdomain by
                          fronts of the oriented cell graph, the solves of a
                          front batched into one dense GEMM (matrix cores for
                          FP32 and the split precisions); one launch per
                          subdomain iteration.  Required (and chosen by AUTO)
                          when a velocity is not parallel to a grid axis. */
} kds_schedule;

typedef struct {
  int32_t dim;           /* d = 1, 2 or 3 */
  int32_t n_cells[3];    /* cells per axis (entries beyond dim ignored) */
  int32_t sub_cells[3];  /* subdomain size in cells; must divide n_cells */
  int32_t periodic[3];   /* 1: periodic axis; 0: Dirichlet ends (kds_set_boundary) */
  double box_lo[3];
  double box_hi[3];
  int32_t degree;        /* p = 0..3; p = 0 is the finite-volume limit */
  int32_t m;             /* conserved components, 1..8 */
  int32_t law;           /* kds_law */
  const double* law_params;
  int32_t n_law_params;
  int32_t n_vel;         /* kinetic velocities, 1..8 */
  const double* vel;     /* n_vel * dim, nonzero; oblique velocities need the front schedule */
  const double* eq_a;    /* n_vel weights, or NULL (see below) */
  const double* eq_b;    /* n_vel * dim weights, or NULL */
  double omega;          /* relaxation parameter, 0 <= omega <= 2 (Sec. 2.2) */
  double dt;             /* time step, > 0 */
  double theta;          /* 1/2 = Crank-Nicolson, 1 = implicit Euler; in [1/2, 1] */
  int32_t n_iter;        /* subdomain iterations K >= 1 (Sec. 5.1); 0 = the converged
                            limit K -> infinity (fully implicit periodic solve;
                            line schedule only) */
  int32_t precision;     /* kds_prec */
  int32_t schedule;      /* kds_schedule */
  const double* source_sigma; /* m damping rates sigma_c >= 0 (+inf allowed) of the
                                 source S(W)_c = -sigma_c W_c, or NULL (no source) */
} kds_config;
/* Source term (Sec. 2.3): the conservative data after the transport are
 * advanced by the Crank-Nicolson step of dW/dt = S(W) (eq:source_term_application_to_W),
 * W+_c = mu_c W_c with mu_c = (1 - sigma_c dt/2)/(1 + sigma_c dt/2) (mu_c = -1 for
 * sigma_c = +inf, the perfect-conductor limit); the kinetic data take the
 * equilibrium part of that change, F_k += M_k(W+) - M_k(W), then relax towards
 * M_k(W+).  This keeps sum_k F_k = W+ (a reading: the paper defers the
 * kinetic details to its reference on the method). */
/* Equilibria (eq:maxwell_def): M_k(W) = eq_a[k] W + sum_i eq_b[k*dim+i] Q^i(W).
 * With eq_a = eq_b = NULL the minimum-norm weights satisfying the moment
 * conditions for every W are used (for +-lambda e_i: M = W/(2d) +- Q^i/(2 lambda)). */

/* Validate cfg, build the FP64 operator tables on the host, allocate the
 * kinetic state on the current HIP device.  hip_stream: a hipStream_t of that
 * device used for all work of this problem, or NULL (the library then creates
 * its own stream).  Errors: KDS_E_INVALID (bad config), KDS_E_UNSUPPORTED
 * (e.g. a velocity not parallel to an axis), KDS_E_NOMEM, KDS_E_DEVICE.
 * Configuration is checked before any device call. */
kds_status kds_create(const kds_config* cfg, void* hip_stream, kds_problem** out);

/* Initial kinetic state F_k = M_k(W) at every node (Sec. 2.2).
 * W: FP64 [cell][node][c].  Resets the step counter.  A W with NaN or Inf
 * (or whose equilibria overflow the storage precision) is refused with
 * KDS_E_NONFINITE and leaves no state (kds_step then returns KDS_E_STATE).
 * Euler law: also records the state's largest wave speed (kds_info). */
kds_status kds_set_state(kds_problem* p, const double* W, int32_t on_device);

/* Dirichlet data on the faces of the axes with periodic[a] = 0 (the exact
 * solution imposed on the boundary, Sec. 6.2).  W_b: FP64 [boundary node][c],
 * the conservative state at the boundary nodes at the END of the next step.
 * Boundary nodes: for each non-periodic axis a (x, y, z order), the face at
 * the low end, then at the high end; on a face, the cells over the other axes
 * (lower axis fastest), then the cell's face nodes over the other axes' node
 * indices (lower axis fastest); count = sum over those axes of
 * 2 * (cells / n_cells[a]) * (p+1)^(d-1).  The upwind value at an inflow face
 * of the box is the kinetic equilibrium M_k(W_b) (a reading: the paper imposes
 * W and leaves the kinetic translation open), taken at the start and at the
 * end of the step by the theta-scheme.  A step goes from the previous call's
 * data (the same data at the first call) to this call's; after a step the
 * data hold their end value, so kds_step(n) with n > 1 keeps them constant.
 * Required before kds_step when some axis is not periodic (else KDS_E_STATE);
 * KDS_E_INVALID on a periodic box. */
kds_status kds_set_boundary(kds_problem* p, const double* W_b, int32_t on_device);

/* n_steps time steps (Sec. 2.2): transport of every F_k (K subdomain
 * iterations of the downwind sweep, eq:dg_imp / eq:ibvp) then relaxation
 * (eq:over_relaxation).  Launched asynchronously on the problem's stream: by
 * default as replays of a captured HIP graph of 8 steps (plus one of 1 step
 * for the rest), or the kernels enqueued step by step where kds_tune found
 * that faster; returns KDS_E_STATE before set_state. */
kds_status kds_step(kds_problem* p, int32_t n_steps);

/* Same steps launched one kernel at a time with HIP events around each kernel;
 * waits for completion and writes the summed milliseconds per kernel kind into
 * kernel_ms[KDS_N_KERNEL_KINDS] (sweep, relax).  For measurement. */
#define KDS_N_KERNEL_KINDS 2
kds_status kds_step_timed(kds_problem* p, int32_t n_steps, double* kernel_ms);

/* Autotuner of the line schedule: times the sweep kernel for candidate
 * launch plans on the current state (reps launches each) and keeps the
 * fastest: cells per lane and columns of cells per workgroup (one grid axis at
 * a time), then the direct register path for x lines against the LDS tile,
 * then fewer workgroups per CU (larger LDS allocation), then the step launch
 * mode of kds_step (graph replay or enqueued kernels) and the access width of
 * the relaxation (periodic problems only; whole steps timed); restores the
 * state.  Needs a state.  For the front schedule the front kernel (where both
 * apply) and the last two choices are tuned, for the plain schedule only the
 * last two (*sweep_ms = -1).  sweep_ms (nullable): best average
 * sweep time.  Needs one state's worth of free device memory (else
 * KDS_E_NOMEM). */
kds_status kds_tune(kds_problem* p, int32_t reps, double* sweep_ms);

/* Sets the two launch choices kds_tune otherwise makes for kds_step:
 * step_eager = 1 enqueues each step's kernels (0: replays captured graphs),
 * relax_vec = 1 runs the relaxation with 16-byte accesses, several nodes per
 * thread (0: one node per thread; also used where the node count is not a
 * multiple of the vector width).  Neither changes the arithmetic.  For callers
 * that capture kds_step into their own graphs, and for tests.  Errors:
 * KDS_E_INVALID for a NULL problem or a flag other than 0 / 1. */
kds_status kds_set_launch(kds_problem* p, int32_t step_eager, int32_t relax_vec);

/* The complete launch plan of a problem: every choice kds_tune makes.  For
 * the line schedule (Sec. 5.1 iterations of whole grid lines, one wavefront
 * per line): per grid axis a, Q[a] cells per lane (Q[a] divides sub_cells[a],
 * n_cells[a] / Q[a] <= 64; up to kds_info_t.line_qmax the lane holds its
 * cells in registers, above it -- at most 64, not for cells of 64 nodes --
 * it streams them through the LDS tile in rounds, which is how lines longer
 * than 64 x line_qmax cells run) and bw[a] columns of
 * cells per workgroup; xdirect = 1 lets x lines with Q[0] = line_qmax be read
 * and written straight between HBM and registers (no LDS tile); lds_bytes =
 * LDS allocated per workgroup (0: what the tile needs; more lets fewer
 * workgroups share a CU).  Axes that carry no velocity have Q = bw = 0.  For
 * the plain and front schedules these fields are 0 (kds_get_plan) and
 * ignored (kds_set_plan).  step_eager and relax_vec as in kds_set_launch.
 * front_kernel (front schedule; 0 elsewhere): 1 = one workgroup per
 * (velocity, subdomain), any cell size and precision; 2 = one wave per
 * (velocity, subdomain, component): the FP32 matrix-core forms with cells of
 * up to 64 nodes (p <= 3), FP64 (on the FP64 matrix cores) with cells of at
 * most 32 nodes (p <= 2 in 3-D, p <= 3 in 2-D), frontiers that fit the LDS;
 * kds_set_plan with front_kernel = 0 keeps the current kernel.
 * The FP64 results of every valid plan agree to rounding; FP32 results depend
 * on Q (the association of the line scan) and on the front kernel (the order
 * of the products' sums), so a plan saved with kds_get_plan and restored with
 * kds_set_plan reproduces results bitwise across runs. */
typedef struct {
  int32_t Q[3];
  int32_t bw[3];
  int32_t xdirect;
  int32_t lds_bytes;
  int32_t step_eager;
  int32_t relax_vec;
  int32_t front_kernel;
} kds_plan_t;

/* Current plan into *plan.  KDS_E_INVALID for NULL arguments. */
kds_status kds_get_plan(const kds_problem* p, kds_plan_t* plan);

/* Replace the plan.  Errors (the plan is left unchanged): KDS_E_INVALID for
 * NULL arguments, flags other than 0 / 1, a line-schedule choice outside the
 * limits above (xdirect = 1 needs a velocity along x with Q[0] = line_qmax),
 * lds_bytes above the device's per-workgroup LDS, or a front_kernel that does
 * not apply to the problem; Q and bw entries of an axis without velocities
 * are ignored. */
kds_status kds_set_plan(kds_problem* p, const kds_plan_t* plan);

/* Autotuner of the subdomain width (sub_cells), which -- unlike the launch
 * plan -- changes the answer (the Jacobi iteration of Sec. 5.1 couples the
 * subdomains through lagged interface traces), so it is a separate call whose
 * result the caller adopts: for each axis carrying a velocity component, the
 * widths S that divide n_cells and satisfy the Proposition of Sec. 5.1
 * (max_k |V_k^a| dt <= S h_a) are tried one axis at a time, the others kept
 * at their best so far, starting from cfg->sub_cells (which must be valid).
 * Each candidate is a temporary problem built from cfg with that width,
 * started from W (FP64 host [cell][node][c]), tuned (kds_tune, reps) and timed
 * over reps steps.  Out: sub_cells[3] the fastest widths, step_ms (nullable)
 * its time per step.  Candidates that cannot be built or run (e.g. a width no
 * schedule accepts, not enough memory) are skipped.  Periodic boxes only
 * (KDS_E_UNSUPPORTED otherwise: the steps of a Dirichlet problem need its
 * boundary data).  Errors: KDS_E_INVALID for NULL arguments, and those of
 * kds_create / kds_set_state / kds_step for cfg itself. */
kds_status kds_tune_subdomains(const kds_config* cfg, const double* W, int32_t reps,
                               int32_t* sub_cells, double* step_ms);

/* kds_tune through a plan cache: a text file of (key, plan) lines, so that
 * later runs and other processes on the same kind of device take the plan
 * that was tuned once instead of timing again -- their FP32 results then do
 * not depend on timing noise.  The key holds everything a plan depends on:
 * schedule, precision, degree, dimension, m, n_vel, n_cells, sub_cells, the
 * axis and sign of every velocity, the Dirichlet axes and the device's
 * architecture name.  If `path` holds the key its plan is applied
 * (kds_set_plan) and *hit = 1; otherwise kds_tune runs, its plan is appended
 * to the file and *hit = 0 (hit nullable).  A missing or unreadable file
 * counts as empty.  Errors: those of kds_tune and kds_set_plan (a cached plan
 * that no longer applies is re-tuned and appended), KDS_E_INVALID for a NULL
 * path or a file that cannot be written (the tuned plan stays in place). */
kds_status kds_tune_cached(kds_problem* p, int32_t reps, const char* path, int32_t* hit);

/* Average duration of one launch of each kernel kind (sweep: the line kernel,
 * or one plain subdomain iteration; relax), from HIP events around reps
 * back-to-back launches on the problem's stream; the state is saved before
 * and restored after (needs one state's worth of free device memory).
 * kernel_ms[KDS_N_KERNEL_KINDS].  For measurement. */
kds_status kds_time_kernels(kds_problem* p, int32_t reps, double* kernel_ms);

/* W = sum_k F_k (FP64, Sec. 2.2 step 3) into W_out [cell][node][c]. */
kds_status kds_moments(kds_problem* p, double* W_out, int32_t on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): kds_moments of
 * the nodes node_begin .. node_begin + node_count - 1 (node = cell * (p+1)^d +
 * node in cell) into HOST memory W_out [node_count][m], staged through a
 * fixed device scratch array of 32 MiB that the library holds on each GPU
 * until the process ends -- kds_moments with on_device = 0 instead allocates
 * a staging buffer of the whole W on its first call.  This call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the address
 * of the array is looked up in kds_create.  node_count * m * 8 bytes must fit
 * the array (at most 4194304 / m nodes per call; larger ranges are rejected
 * with KDS_E_INVALID, and the caller walks the nodes in several calls).
 * Returns after the copy has finished.  Values are bitwise those of
 * kds_moments.  Every call on one GPU shares its array: calls that overlap in
 * time on one GPU (other host threads, other problems) race.
 * Errors: KDS_E_INVALID (NULL, range outside the nodes or too large),
 * KDS_E_STATE (no state), KDS_E_DEVICE. */
kds_status kds_moments_static(kds_problem* p, int64_t node_begin, int64_t node_count,
                              double* W_out);

/* Checkpoint / resume of the kinetic state (F, not W: after the first step
 * F_k != M_k(W), Sec. 2.2 remark).  F: FP64 [k][cell][node][c]. */
kds_status kds_get_kinetic(kds_problem* p, double* F_out, int32_t on_device);
kds_status kds_set_kinetic(kds_problem* p, const double* F, int32_t on_device);

/* Scan the kinetic state for NaN/Inf: KDS_OK or KDS_E_NONFINITE. */
kds_status kds_check_finite(kds_problem* p);

/* Residual of the subdomain iteration (Sec. 5.1, eq:ibvp): for the step that
 * would start from the current state (and boundary data), the outflow traces
 * of every subdomain (every velocity and component, at every node on the
 * subdomain's downwind faces: for velocity k the faces across which V_k
 * leaves it) after the last iterate K and after iterate K-1 (iterate 0 = the
 * state itself), and
 *   out[0] = max |tr^(K) - tr^(K-1)|,  out[1] = max |tr^(K)|.
 * With lagged interface data, what leaves a subdomain through its downwind
 * face (iterate K) and what enters the next one (iterate K-1) differ by this
 * difference, weighted by theta |V_k| dt and the face quadrature, so out[0]
 * measures the conservation defect of a step; it goes to 0 as the iteration
 * converges (n_iter = 0: out = {0, -1}).  The state is not changed.  Runs,
 * on the problem's stream, and waits: on the front schedule (any velocity
 * set) its own K iterates into its iterate buffers; otherwise the literal
 * sweep's kernels (one launch per iterate, two trace sets allocated).  Errors
 * KDS_E_INVALID, KDS_E_STATE (no state, or Dirichlet data missing),
 * KDS_E_NOMEM, KDS_E_DEVICE. */
kds_status kds_trace_residual(kds_problem* p, double* out);

/* Wait for all work of the problem's stream. */
kds_status kds_synchronize(kds_problem* p);

typedef struct {
  int64_t n_unknowns;     /* cells * (p+1)^d * m * n_vel */
  int64_t state_bytes;    /* device bytes of one kinetic state */
  int32_t schedule;       /* schedule actually used (KDS_SCHED_PLAIN / LINE / FRONT) */
  int32_t precision;
  int32_t steps_done;
  double max_kinetic_courant; /* max_k |V_k| dt / h_axis */
  double min_subdomain_width; /* min over used axes of sub_cells * h */
  int32_t proposition_ok; /* 1 if |V| dt <= subdomain width (Sec. 5.1 Proposition) */
  int32_t line_Q[3];      /* line schedule, per axis: cells per lane (0 for plain) */
  int32_t line_bw[3];     /* line schedule, per axis: columns of cells per workgroup */
  int32_t tuned;          /* 1 after kds_tune */
  int32_t line_xdirect;   /* line schedule: x lines read / written straight to registers */
  int32_t line_lds_bytes; /* line schedule: LDS allocated per workgroup */
  int32_t step_eager;     /* kds_step enqueues each step's kernels instead of
                             replaying a captured graph (kds_tune's choice) */
  int32_t relax_vec;      /* relaxation with 16-byte accesses, several nodes
                             per thread (kds_tune's choice) */
  int32_t line_qmax;      /* line schedule: most cells per lane held in
                             registers (budget of 64 state values per lane;
                             more are streamed in rounds), 0 otherwise */
  /* Stability warnings (the problem runs regardless):
   * eq_monotone: 1 if every equilibrium derivative dM_k/dW =
   *   a_k I + sum_i b_{k,i} A^i is positive semidefinite (linear law with
   *   symmetric A^i, checked at create; the bound on lambda that keeps the
   *   relaxation monotone, under which the entropy argument of Sec. 2.2
   *   holds), 0 if one has a negative eigenvalue (eq_min_eig, the smallest),
   *   -1 if not checked (Euler law, non-symmetric A^i);
   * max_wave_speed: linear law, max_i of the spectral radius of A^i (at
   *   create); Euler, max over the nodes of the last kds_set_state and the
   *   axes of |u_i| + c (+inf where rho <= 0 or p <= 0); -1 if unknown;
   * subchar_ok: 1 if min_k |V_k| > max_wave_speed (the sub-characteristic
   *   condition of Sec. 2.1, along the coordinate directions), 0 if not, -1
   *   if max_wave_speed is unknown. */
  int32_t eq_monotone;
  double eq_min_eig;
  double max_wave_speed;
  int32_t subchar_ok;
} kds_info_t;
kds_status kds_info(const kds_problem* p, kds_info_t* info);

/* Release device memory, graph and (own) stream.  NULL is allowed.  A batch
 * holding p must be destroyed first. */
void kds_destroy(kds_problem* p);

/* Last error message of p, or the thread-local kds_create message if p is NULL. */
const char* kds_last_error(const kds_problem* p);

/* ------------------------------------------------------------------ batches
 * Many independent problems (any sizes, laws, degrees, schedules) advanced
 * together by one time step each per kds_batch_step.  The members keep their
 * own states; a batch step gives exactly the results of kds_step on every
 * member (the same kernels' arithmetic), but the line-schedule members that
 * share (precision, degree, dimension, workgroup size, law, m, n_vel,
 * periodic or Dirichlet) are swept by ONE launch whose workgroups are spread
 * over the members and relaxed by ONE more launch; front-schedule members on
 * the wave kernel that share (precision, form, dimension, degree, subdomain
 * iterations, law, m, n_vel) take ONE launch per subdomain iteration and ONE
 * relaxation; plain-schedule members and front members on the workgroup
 * kernel add their own kernel sequences.  Dirichlet members advance their boundary data at
 * the end of each step as in kds_step.  A whole batched step is one captured HIP graph whose
 * groups are parallel branches (they touch disjoint memory), launched on the
 * batch's own stream, ordered after the work already queued on every member's
 * stream; the members' streams are ordered after it.
 * Members must be on one device and distinct; the batch keeps pointers to
 * them (destroy the batch before its members).  A member re-tuned by kds_tune
 * is picked up at the next batch step.  Not thread safe. */
typedef struct kds_batch kds_batch; /* opaque, library-owned */

/* Group the members and upload the task tables (device memory owned by the
 * batch).  Errors: KDS_E_INVALID (NULL, duplicate, devices differ),
 * KDS_E_UNSUPPORTED (a grouped launch would exceed a launch limit),
 * KDS_E_NOMEM, KDS_E_DEVICE; message in kds_batch_last_error(NULL). */
kds_status kds_batch_create(kds_problem* const* problems, int32_t n, kds_batch** out);

/* n_steps time steps of every member (kds_step semantics), asynchronously.
 * KDS_E_STATE if a member has no state.  Each member's steps_done grows. */
kds_status kds_batch_step(kds_batch* b, int32_t n_steps);

/* Same, then waits; *ms = milliseconds between HIP events recorded on the
 * batch stream around the n_steps graph launches.  For measurement. */
kds_status kds_batch_step_timed(kds_batch* b, int32_t n_steps, double* ms);

/* Average duration of the batch's grouped kernels per step: kernel_ms[0] =
 * sum over the grouped line-sweep launches, kernel_ms[1] = sum over the
 * grouped relaxations (reps back-to-back launches each, HIP events on the
 * batch stream); line-schedule member states are saved and restored (needs
 * their size in free device memory).  For measurement. */
kds_status kds_batch_time_kernels(kds_batch* b, int32_t reps, double* kernel_ms);

/* Launch-shape search for the batch (Sec. 5 subdomain parallelism over many
 * problems): the batched step is timed (reps steps after one untimed, HIP
 * events on the batch stream) with the line-schedule members' bundles widened
 * 1, 2 and 4 times (columns of cells per workgroup, where the member's cells
 * per lane allow it: the same lines and lane arithmetic, so results are
 * unchanged; the members' own plans are untouched), and the fastest is kept.
 * Every member's state and boundary data are saved before and restored after
 * (needs their size in free device memory); step counts do not move.
 * *best_ms (may be NULL) = ms per step of the kept choice.  Errors:
 * KDS_E_INVALID, KDS_E_STATE (a member without state), KDS_E_NOMEM,
 * KDS_E_DEVICE. */
kds_status kds_batch_tune(kds_batch* b, int32_t reps, double* best_ms);

/* Wait for the batch stream. */
kds_status kds_batch_synchronize(kds_batch* b);

/* Release the batch (not its members).  NULL is allowed. */
void kds_batch_destroy(kds_batch* b);

/* Last error message of b, or the thread-local kds_batch_create message if b is NULL. */
const char* kds_batch_last_error(const kds_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* KDS_H */
