// kds_oracle.cpp -- plain FP64 CPU oracle of the kinetic DG time step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
// libkds and its Python binding) may include, link, load or call this file.
// Only tests/, the smoke check and the CPU-baseline leg of bench.py use it.
// It shares no code, header, table or constant with the GPU path.
//
// What it computes (Gerhard, Helluy, Michel-Dansac, Weber, "Parallel kinetic
// schemes for conservation laws, with large time steps", arXiv:2212.11010):
//
//   * kinetic representation W = sum_k F_k, equilibria M_k(W) satisfying the
//     moment conditions (Sec. 2.1, eq:maxwell_def);
//   * one time step = free transport of every F_k for dt, then the
//     over-relaxation F_k <- omega M_k(W) + (1-omega) F_k (Sec. 2.2,
//     eq:over_relaxation);
//   * the transport is the implicit upwind DG scheme (Sec. 3.1, eq:dg_imp),
//     theta-generalised (theta = 1: the implicit Euler form printed in the
//     paper; theta = 1/2: Crank-Nicolson, the form used in practice), with
//     nodal tensor Gauss-Lobatto bases on Cartesian cells and collocated
//     Gauss-Lobatto quadrature;
//   * the implicit system is solved by visiting the cells of each subdomain in a
//     topological order of the velocity-oriented cell graph (Sec. 3.2,
//     "downwind algorithm"), one dense per-cell LU solve per cell;
//   * on an axis that is not periodic, the upwind value at an inflow face of
//     the box is prescribed: the kinetic boundary data f_k = M_k(W_b) of a
//     given boundary state W_b (Dirichlet conditions, Sec. 6.2), at the old
//     and the new time of the theta-scheme;
//   * subdomains are coupled by the iterative algorithm of Sec. 5.1 (eq:ibvp):
//     iterate p takes its upwind interface data from the neighbours' iterate
//     p-1; iterate 0 is the state at the previous time (eq:ibvp2); every
//     subdomain reads iterate p-1 (Jacobi).  Periodic wrap faces always count
//     as interfaces, since the periodic upwind graph is not acyclic.
//
// Deliberately slow and literal: no precomputed inverse, no reordering, no
// blocking.  Every cell system is assembled from the residual definition and
// solved by Gaussian elimination with partial pivoting.
//
// Layouts (all FP64):
//   W   [cell][node][c]           cells x-fastest, nodes x-fastest
//   F   [k][c][cell][node]        oracle-internal kinetic layout
//   W_b [boundary node][c]        boundary nodes: for each non-periodic axis a
//                                 (x, y, z order), the face at the low end,
//                                 then at the high end; on a face, cells over
//                                 the other axes (lower axis fastest), then
//                                 the face nodes of the cell over the other
//                                 axes' node indices (lower axis fastest)
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t dim;
  int32_t n_cells[3];
  int32_t sub_cells[3];
  double box_lo[3];
  double box_hi[3];
  int32_t degree;        // p >= 0 (p = 0 is the finite-volume limit)
  int32_t m;             // number of conserved components
  int32_t law;           // 0 = linear Q^i(W) = A^i W, 1 = Euler
  const double* law_params;
  int32_t n_law_params;
  int32_t n_vel;
  const double* vel;     // n_vel * dim
  const double* eq_a;    // n_vel, or NULL
  const double* eq_b;    // n_vel * dim, or NULL
  double omega;
  double dt;
  double theta;
  int32_t n_iter;        // K >= 1; 0 = iterate to convergence
  const double* source_sigma;  // m damping rates sigma_c >= 0 (may be +inf), or NULL
  const int32_t* periodic;     // 3 flags, or NULL (all periodic); 0 = Dirichlet ends
  const double* bnd_W_old;     // boundary state [boundary node][c] at the step start, or NULL
  const double* bnd_W_new;     // ... at the step end (orc_step: first step; later steps
                               // hold it constant)
} orc_config;

}  // extern "C"

namespace {

int P_of(const orc_config* c) { return c->degree + 1; }
int nn_of(const orc_config* c) {
  int P = P_of(c), n = 1;
  for (int a = 0; a < c->dim; ++a) n *= P;
  return n;
}
long ncell_of(const orc_config* c) {
  long n = 1;
  for (int a = 0; a < c->dim; ++a) n *= c->n_cells[a];
  return n;
}

// Legendre polynomial P_n and its derivative at x in [-1, 1] (three-term
// recurrence).
void legendre(int n, double x, double* Pn, double* dPn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *Pn = 1.0; *dPn = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *Pn = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid off +-1
  if (std::fabs(x) < 1.0)
    *dPn = n * (p0 - x * p1) / (1.0 - x * x);
  else
    *dPn = (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0)) * 0.5 * n * (n + 1.0);
}

}  // namespace

extern "C" {

// Gauss-Lobatto nodes and weights on [0, 1] (p + 1 points: the end points and
// the roots of P_p'); weights sum to one.  p = 0 gives the single midpoint with
// weight one (cell average, finite-volume limit).
int orc_gl(int p, double* xi, double* w) {
  if (p < 0 || p > 8) return 1;
  if (p == 0) { xi[0] = 0.5; w[0] = 1.0; return 0; }
  int n = p + 1;
  std::vector<double> x(n);
  for (int j = 0; j < n; ++j) {
    double xj = -std::cos(M_PI * j / p);
    if (j > 0 && j < p) {
      // Newton on P_p'(x) = 0 using q = (1-x^2) P_p', q' = -p(p+1) P_p
      for (int it = 0; it < 100; ++it) {
        double Pn, dPn;
        legendre(p, xj, &Pn, &dPn);
        double q = (1.0 - xj * xj) * dPn;
        double dq = -p * (p + 1.0) * Pn;
        double step = q / dq;
        xj -= step;
        if (std::fabs(step) < 1e-17) break;
      }
    }
    x[j] = xj;
  }
  for (int j = 0; j < n; ++j) {
    double Pn, dPn;
    legendre(p, x[j], &Pn, &dPn);
    double wj = 2.0 / (p * (p + 1.0) * Pn * Pn);
    xi[j] = 0.5 * (x[j] + 1.0);
    w[j] = 0.5 * wj;
  }
  return 0;
}

// D[b*(p+1) + a] = l_a'(xi_b), derivative of the a-th Lagrange basis
// polynomial on the Gauss-Lobatto nodes of [0, 1], by direct differentiation
// of the product formula.
int orc_deriv(int p, double* D) {
  int n = p + 1;
  std::vector<double> xi(n), w(n);
  if (orc_gl(p, xi.data(), w.data())) return 1;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      double s = 0.0;
      for (int mm = 0; mm < n; ++mm) {
        if (mm == a) continue;
        double term = 1.0 / (xi[a] - xi[mm]);
        for (int l = 0; l < n; ++l) {
          if (l == a || l == mm) continue;
          term *= (xi[b] - xi[l]) / (xi[a] - xi[l]);
        }
        s += term;
      }
      D[b * n + a] = s;
    }
  return 0;
}

// Physical flux Q^i(W), i = 0..dim-1, written Q[i*m + c] (eq:conslaw).
//   law 0: Q^i = A^i W with A^i = law_params[i*m*m ...] row-major.
//   law 1: compressible Euler, W = (rho, rho u_1..rho u_d, E),
//          p = (gamma - 1)(E - rho |u|^2 / 2).
int orc_flux(const orc_config* c, const double* W, double* Q) {
  int d = c->dim, m = c->m;
  if (c->law == 0) {
    if (c->n_law_params < d * m * m) return 1;
    for (int i = 0; i < d; ++i)
      for (int r = 0; r < m; ++r) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += c->law_params[(i * m + r) * m + q] * W[q];
        Q[i * m + r] = s;
      }
    return 0;
  }
  if (c->law == 1) {
    if (m != d + 2 || c->n_law_params < 1) return 1;
    double gamma = c->law_params[0];
    double rho = W[0], E = W[d + 1];
    double u[3] = {0, 0, 0}, ke = 0.0;
    for (int i = 0; i < d; ++i) { u[i] = W[1 + i] / rho; ke += 0.5 * rho * u[i] * u[i]; }
    double pr = (gamma - 1.0) * (E - ke);
    for (int i = 0; i < d; ++i) {
      Q[i * m + 0] = rho * u[i];
      for (int j = 0; j < d; ++j) Q[i * m + 1 + j] = rho * u[i] * u[j] + (i == j ? pr : 0.0);
      Q[i * m + d + 1] = (E + pr) * u[i];
    }
    return 0;
  }
  return 1;
}

// Equilibrium weights: M_k(W) = a_k W + sum_i b_{k,i} Q^i(W).  The moment
// conditions of eq:maxwell_def hold for every W iff
//   sum_k a_k = 1, sum_k V_k^i a_k = 0, sum_k b_{k,j} = 0,
//   sum_k V_k^i b_{k,j} = delta_ij.
// When the caller gives no weights, the minimum-norm solution is used:
// [a | b] = P^T (P P^T)^{-1}, with P = [1 ; V^T] of size (dim+1) x n_vel.
int orc_eq_weights(const orc_config* c, double* a, double* b) {
  int d = c->dim, nv = c->n_vel;
  if (c->eq_a && c->eq_b) {
    for (int k = 0; k < nv; ++k) {
      a[k] = c->eq_a[k];
      for (int i = 0; i < d; ++i) b[k * d + i] = c->eq_b[k * d + i];
    }
    return 0;
  }
  int r = d + 1;
  std::vector<double> Pm(r * nv);
  for (int k = 0; k < nv; ++k) {
    Pm[0 * nv + k] = 1.0;
    for (int i = 0; i < d; ++i) Pm[(1 + i) * nv + k] = c->vel[k * d + i];
  }
  // G = P P^T (r x r); solve G Y = I by Gauss-Jordan
  std::vector<double> G(r * r), Y(r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int k = 0; k < nv; ++k) s += Pm[i * nv + k] * Pm[j * nv + k];
      G[i * r + j] = s;
    }
  for (int i = 0; i < r; ++i) Y[i * r + i] = 1.0;
  for (int col = 0; col < r; ++col) {
    int piv = col;
    for (int i = col + 1; i < r; ++i)
      if (std::fabs(G[i * r + col]) > std::fabs(G[piv * r + col])) piv = i;
    if (std::fabs(G[piv * r + col]) < 1e-300) return 1;
    for (int j = 0; j < r; ++j) {
      std::swap(G[col * r + j], G[piv * r + j]);
      std::swap(Y[col * r + j], Y[piv * r + j]);
    }
    double inv = 1.0 / G[col * r + col];
    for (int j = 0; j < r; ++j) { G[col * r + j] *= inv; Y[col * r + j] *= inv; }
    for (int i = 0; i < r; ++i) {
      if (i == col) continue;
      double f = G[i * r + col];
      for (int j = 0; j < r; ++j) { G[i * r + j] -= f * G[col * r + j]; Y[i * r + j] -= f * Y[col * r + j]; }
    }
  }
  // X = P^T Y  (nv x r)
  for (int k = 0; k < nv; ++k)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int i = 0; i < r; ++i) s += Pm[i * nv + k] * Y[i * r + j];
      if (j == 0) a[k] = s; else b[k * d + (j - 1)] = s;
    }
  return 0;
}

// M[k*m + c] = M_k(W)_c.
int orc_equilibrium(const orc_config* c, const double* W, double* M) {
  int d = c->dim, m = c->m, nv = c->n_vel;
  std::vector<double> a(nv), b(nv * d), Q(d * m);
  if (orc_eq_weights(c, a.data(), b.data())) return 1;
  if (orc_flux(c, W, Q.data())) return 1;
  for (int k = 0; k < nv; ++k)
    for (int r = 0; r < m; ++r) {
      double s = a[k] * W[r];
      for (int i = 0; i < d; ++i) s += b[k * d + i] * Q[i * m + r];
      M[k * m + r] = s;
    }
  return 0;
}

}  // extern "C"

namespace {

struct CellOp {
  // Residual r_i(f; tr) = sum_j L[i][j] f_j + sum_{inflow faces} lift * tr,
  // i.e. the terms of eq:dg_imp after division by the lumped mass h^d w_i:
  //   volume: -(1/w_i) sum_q w_q f_q (V . grad psi_i)(x_q) (GL collocation)
  //   faces : (1/(h w_i^{face normal axis})) [(V.N)_+ f_i + (V.N)_- f_R]
  int dim, P, nn;
  std::vector<double> L;      // nn x nn
  // For node i and face f = 2*axis + side: coefficient multiplying the
  // neighbour trace (zero if i is not on face f or the face is not inflow).
  std::vector<double> lift;   // nn x (2*dim)
};

void node_index(int i, int dim, int P, int* idx) {
  for (int a = 0; a < dim; ++a) { idx[a] = i % P; i /= P; }
}

CellOp build_cell_op(const orc_config* c, const double* V) {
  CellOp op;
  op.dim = c->dim;
  op.P = P_of(c);
  op.nn = nn_of(c);
  int P = op.P, nn = op.nn, d = op.dim, p = c->degree;
  std::vector<double> xi(P), w(P), D(P * P);
  orc_gl(p, xi.data(), w.data());
  if (p > 0) orc_deriv(p, D.data()); else D[0] = 0.0;
  double h[3];
  for (int a = 0; a < d; ++a) h[a] = (c->box_hi[a] - c->box_lo[a]) / c->n_cells[a];
  op.L.assign(nn * nn, 0.0);
  op.lift.assign(nn * 2 * d, 0.0);
  for (int i = 0; i < nn; ++i) {
    int ii[3];
    node_index(i, d, P, ii);
    for (int j = 0; j < nn; ++j) {
      int jj[3];
      node_index(j, d, P, jj);
      for (int ax = 0; ax < d; ++ax) {
        bool same_other = true;
        for (int o = 0; o < d; ++o)
          if (o != ax && ii[o] != jj[o]) same_other = false;
        if (!same_other) continue;
        // -(1/w_i) w_j (V^ax/h_ax) l'_{i_ax}(xi_{j_ax}); tangential weights cancel
        op.L[i * nn + j] += -(V[ax] / h[ax]) * w[jj[ax]] * D[jj[ax] * P + ii[ax]] / w[ii[ax]];
      }
    }
    for (int ax = 0; ax < d; ++ax)
      for (int side = 0; side < 2; ++side) {
        int face_idx = side ? p : 0;
        if (ii[ax] != face_idx) continue;
        double VN = side ? V[ax] : -V[ax];
        double coef = VN / (h[ax] * w[ii[ax]]);
        if (VN > 0) op.L[i * nn + i] += coef;
        else if (VN < 0) op.lift[i * 2 * d + 2 * ax + side] = coef;
      }
  }
  return op;
}

// Dense solve A x = b (n x n) by Gaussian elimination with partial pivoting.
int lu_solve(int n, std::vector<double>& A, std::vector<double>& b) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int i = col + 1; i < n; ++i)
      if (std::fabs(A[i * n + col]) > std::fabs(A[piv * n + col])) piv = i;
    if (A[piv * n + col] == 0.0) return 1;
    if (piv != col) {
      for (int j = 0; j < n; ++j) std::swap(A[col * n + j], A[piv * n + j]);
      std::swap(b[col], b[piv]);
    }
    for (int i = col + 1; i < n; ++i) {
      double f = A[i * n + col] / A[col * n + col];
      if (f == 0.0) continue;
      for (int j = col; j < n; ++j) A[i * n + j] -= f * A[col * n + j];
      b[i] -= f * b[col];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  return 0;
}

struct Grid {
  int d, N[3], S[3];
  bool per[3];
  long ncell;
  long cell_of(const int* cc) const {
    long id = 0, mul = 1;
    for (int a = 0; a < d; ++a) { id += cc[a] * mul; mul *= N[a]; }
    return id;
  }
  void coords(long id, int* cc) const {
    for (int a = 0; a < d; ++a) { cc[a] = (int)(id % N[a]); id /= N[a]; }
  }
};

Grid make_grid(const orc_config* c) {
  Grid g;
  g.d = c->dim;
  for (int a = 0; a < 3; ++a) { g.N[a] = a < c->dim ? c->n_cells[a] : 1; g.S[a] = a < c->dim ? c->sub_cells[a] : 1; }
  g.ncell = ncell_of(c);
  for (int a = 0; a < 3; ++a) g.per[a] = !(c->periodic && a < c->dim && c->periodic[a] == 0);
  return g;
}

// Boundary nodes of the face (axis ax): cells over the other axes times the
// face nodes of a cell.
long face_nodes(const orc_config* c, int ax) {
  long n = 1;
  for (int a = 0; a < c->dim; ++a)
    if (a != ax) n *= (long)c->n_cells[a] * P_of(c);
  return n;
}

// Offset of face (ax, side) in the boundary-node numbering, -1 if ax is periodic.
long face_offset(const orc_config* c, int ax, int side) {
  Grid g = make_grid(c);
  if (g.per[ax]) return -1;
  long off = 0;
  for (int a = 0; a < ax; ++a)
    if (!g.per[a]) off += 2 * face_nodes(c, a);
  return off + side * face_nodes(c, ax);
}

long n_boundary_nodes(const orc_config* c) {
  Grid g = make_grid(c);
  long n = 0;
  for (int a = 0; a < c->dim; ++a)
    if (!g.per[a]) n += 2 * face_nodes(c, a);
  return n;
}

// Index on face ax of the boundary node matching node i of cell cc.
long face_index(const orc_config* c, const int* cc, int ax, int i) {
  int P = P_of(c);
  int ii[3];
  node_index(i, c->dim, P, ii);
  long cell = 0, cmul = 1, node = 0, nmul = 1;
  for (int a = 0; a < c->dim; ++a) {
    if (a == ax) continue;
    cell += cc[a] * cmul;
    cmul *= c->n_cells[a];
    node += ii[a] * nmul;
    nmul *= P;
  }
  return cell * nmul + node;
}

// Neighbour across face (ax, side): returns its cell id and whether the face is
// interior to one subdomain (no periodic wrap, same subdomain index on ax).
// On a non-periodic axis a face of the box has no neighbour: returns -1.
long neighbour(const Grid& g, const int* cc, int ax, int side, bool* internal) {
  int nc[3] = {cc[0], cc[1], cc[2]};
  bool wrapped = false;
  if (side) { nc[ax] += 1; if (nc[ax] == g.N[ax]) { nc[ax] = 0; wrapped = true; } }
  else { nc[ax] -= 1; if (nc[ax] < 0) { nc[ax] = g.N[ax] - 1; wrapped = true; } }
  *internal = !wrapped && (cc[ax] / g.S[ax] == nc[ax] / g.S[ax]);
  if (wrapped && !g.per[ax]) return -1;
  return g.cell_of(nc);
}

// Neighbour node matching node i across face (ax, side): same indices on the
// other axes, opposite face index on ax.
int matching_node(int i, int dim, int P, int ax, int side) {
  int ii[3];
  node_index(i, dim, P, ii);
  ii[ax] = side ? 0 : P - 1;
  int j = 0, mul = 1;
  for (int a = 0; a < dim; ++a) { j += ii[a] * mul; mul *= P; }
  return j;
}

// One transport step dt for a single scalar field f (one velocity, one
// component): theta-scheme DG, subdomain sweeps, K Jacobi iterations.
// fb_old / fb_new: kinetic boundary values of this field at the boundary
// nodes (NULL: zero inflow at the faces of non-periodic axes).
int transport_scalar(const orc_config* c, const CellOp& op, const double* V,
                     const double* f_old, double* f_new, const double* fb_old,
                     const double* fb_new) {
  Grid g = make_grid(c);
  int d = c->dim, P = op.P, nn = op.nn, K = c->n_iter;
  double dt = c->dt, th = c->theta;
  long total = g.ncell * nn;
  std::vector<double> prev(f_old, f_old + total), cur(total, 0.0);
  std::vector<char> done(g.ncell, 0);
  std::vector<double> A(nn * nn), rhs(nn), rold(nn);
  int nsub[3];
  for (int a = 0; a < 3; ++a) nsub[a] = g.N[a] / g.S[a];
  // K = 0: iterate until the iterates stop changing (the limit K -> infinity,
  // the fully implicit solve): the change falls to rounding level, or stops
  // decreasing for 20 iterates; cap 10000 iterates
  const bool converge = K == 0;
  const int kmax = converge ? 10000 : K;
  double best_diff = 1e300;
  int stalled = 0;
  for (int it = 1; it <= kmax; ++it) {
    std::fill(done.begin(), done.end(), 0);
    for (int s2 = 0; s2 < nsub[2]; ++s2)
      for (int s1 = 0; s1 < nsub[1]; ++s1)
        for (int s0 = 0; s0 < nsub[0]; ++s0) {
          int sidx[3] = {s0, s1, s2};
          // lexicographic order inside the subdomain, each axis traversed in
          // the direction of V (a topological order of the oriented graph)
          long cnt = 1;
          for (int a = 0; a < d; ++a) cnt *= g.S[a];
          for (long t = 0; t < cnt; ++t) {
            int cc[3] = {0, 0, 0};
            long rem = t;
            for (int a = 0; a < d; ++a) {
              int loc = (int)(rem % g.S[a]);
              rem /= g.S[a];
              if (V[a] < 0) loc = g.S[a] - 1 - loc;
              cc[a] = sidx[a] * g.S[a] + loc;
            }
            long cell = g.cell_of(cc);
            const double* fo = f_old + cell * nn;
            // old-time residual r(f^{n-1}; tr^{n-1})
            for (int i = 0; i < nn; ++i) {
              double s = 0.0;
              for (int j = 0; j < nn; ++j) s += op.L[i * nn + j] * fo[j];
              rold[i] = s;
            }
            for (int i = 0; i < nn; ++i) rhs[i] = fo[i] / dt - (1.0 - th) * rold[i];
            for (int ax = 0; ax < d; ++ax)
              for (int side = 0; side < 2; ++side) {
                bool internal;
                long nb = neighbour(g, cc, ax, side, &internal);
                if (nb < 0) {
                  // face of the box on a Dirichlet axis: prescribed inflow
                  const long off = face_offset(c, ax, side);
                  for (int i = 0; i < nn; ++i) {
                    double lc = op.lift[i * 2 * d + 2 * ax + side];
                    if (lc == 0.0) continue;
                    const long b = off + face_index(c, cc, ax, i);
                    const double bo = fb_old ? fb_old[b] : 0.0;
                    const double bn = fb_new ? fb_new[b] : 0.0;
                    rhs[i] -= (1.0 - th) * lc * bo + th * lc * bn;
                  }
                  continue;
                }
                const double* tr_new;
                if (internal) {
                  bool any_lift = false;
                  for (int i = 0; i < nn; ++i) if (op.lift[i * 2 * d + 2 * ax + side] != 0.0) any_lift = true;
                  if (any_lift && !done[nb]) {
                    std::fprintf(stderr, "oracle: sweep order is not topological\n");
                    return 2;
                  }
                  tr_new = cur.data() + nb * nn;
                } else {
                  tr_new = prev.data() + nb * nn;
                }
                const double* tr_old = f_old + nb * nn;
                for (int i = 0; i < nn; ++i) {
                  double lc = op.lift[i * 2 * d + 2 * ax + side];
                  if (lc == 0.0) continue;
                  int j = matching_node(i, d, P, ax, side);
                  rhs[i] -= (1.0 - th) * lc * tr_old[j] + th * lc * tr_new[j];
                }
              }
            for (int i = 0; i < nn; ++i)
              for (int j = 0; j < nn; ++j) A[i * nn + j] = (i == j ? 1.0 / dt : 0.0) + th * op.L[i * nn + j];
            if (lu_solve(nn, A, rhs)) return 3;
            for (int i = 0; i < nn; ++i) cur[cell * nn + i] = rhs[i];
            done[cell] = 1;
          }
        }
    if (converge) {
      double diff = 0.0, scale = 0.0;
      for (long i = 0; i < total; ++i) {
        diff = std::max(diff, std::fabs(cur[i] - prev[i]));
        scale = std::max(scale, std::fabs(cur[i]));
      }
      prev.swap(cur);
      if (diff <= 2e-16 * scale) break;
      if (diff < best_diff) { best_diff = diff; stalled = 0; }
      else if (++stalled >= 20 && diff <= 1e-12 * scale) break;
    } else {
      prev.swap(cur);
    }
  }
  std::memcpy(f_new, prev.data(), total * sizeof(double));
  return 0;
}

int validate(const orc_config* c) {
  if (!c || c->dim < 1 || c->dim > 3 || c->degree < 0 || c->degree > 5) return 1;
  if (c->periodic)
    for (int a = 0; a < c->dim; ++a)
      if (c->periodic[a] != 0 && c->periodic[a] != 1) return 1;
  if (c->m < 1 || c->n_vel < 1 || c->n_iter < 0 || !(c->dt > 0)) return 1;
  for (int a = 0; a < c->dim; ++a) {
    if (c->n_cells[a] < 1 || c->sub_cells[a] < 1) return 1;
    if (c->n_cells[a] % c->sub_cells[a]) return 1;
  }
  return 0;
}

}  // namespace

extern "C" {

// Residual of one cell for velocity V: r[i] = (L f)_i + sum_faces lift * tr,
// with tr[(2*axis + side)*nn + i] the neighbour value matching node i on that
// face (ignored where node i is not on an inflow face).  Used by the pins.
int orc_cell_residual(const orc_config* c, const double* V, const double* f,
                      const double* tr, double* r) {
  if (validate(c)) return 1;
  CellOp op = build_cell_op(c, V);
  int nn = op.nn, d = c->dim;
  for (int i = 0; i < nn; ++i) {
    double s = 0.0;
    for (int j = 0; j < nn; ++j) s += op.L[i * nn + j] * f[j];
    for (int fce = 0; fce < 2 * d; ++fce) s += op.lift[i * 2 * d + fce] * tr[fce * nn + i];
    r[i] = s;
  }
  return 0;
}

// Transport of one scalar field (velocity k) over dt; f layout [cell][node];
// fb_old / fb_new: its boundary values at the boundary nodes (or NULL).
int orc_transport(const orc_config* c, int k, const double* f_old, double* f_new,
                  const double* fb_old, const double* fb_new) {
  if (validate(c) || k < 0 || k >= c->n_vel) return 1;
  const double* V = c->vel + k * c->dim;
  CellOp op = build_cell_op(c, V);
  return transport_scalar(c, op, V, f_old, f_new, fb_old, fb_new);
}

// Transport of n_lines independent scalar fields of the 1-D problem c
// (dim = 1, periodic): line l is f[l][cell][node], carried at velocity
// v[l]; each line is exactly orc_transport of a one-velocity copy of c.  A
// test helper for the sampled full-size checks, where the transport along
// every grid line through the sampled cells is needed (an axis-aligned
// velocity transports each node line on its own); OpenMP over the lines
// (n_threads > 0), no change of arithmetic.
int orc_transport_lines(const orc_config* c, int n_lines, const double* v, const double* f_old,
                        double* f_new, int n_threads) {
  if (validate(c) || c->dim != 1 || n_lines < 0 || !v) return 1;
  if (c->periodic && c->periodic[0] != 1) return 1;
  const long len = (long)c->n_cells[0] * P_of(c);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
  for (int l = 0; l < n_lines; ++l) {
    orc_config cl = *c;
    cl.n_vel = 1;
    cl.vel = v + l;
    CellOp op = build_cell_op(&cl, cl.vel);
    err |= transport_scalar(&cl, op, cl.vel, f_old + l * len, f_new + l * len, nullptr, nullptr);
  }
  return err;
}

// Number of boundary nodes (faces of the non-periodic axes).
long orc_n_boundary_nodes(const orc_config* c) {
  if (validate(c)) return -1;
  return n_boundary_nodes(c);
}

// F[k][c][cell][node] = M_k(W)_c, W[cell][node][c]  (Sec. 2.2: F_k = M_k(W_0)).
int orc_init(const orc_config* c, const double* W, double* F) {
  if (validate(c)) return 1;
  long nc = ncell_of(c);
  int nn = nn_of(c), m = c->m, nv = c->n_vel;
  std::vector<double> M(nv * m);
  for (long cell = 0; cell < nc; ++cell)
    for (int i = 0; i < nn; ++i) {
      if (orc_equilibrium(c, W + (cell * nn + i) * m, M.data())) return 1;
      for (int k = 0; k < nv; ++k)
        for (int r = 0; r < m; ++r) F[((long)(k * m + r) * nc + cell) * nn + i] = M[k * m + r];
    }
  return 0;
}

// W[cell][node][c] = sum_k F_k.
int orc_moments(const orc_config* c, const double* F, double* W) {
  if (validate(c)) return 1;
  long nc = ncell_of(c);
  int nn = nn_of(c), m = c->m, nv = c->n_vel;
  for (long cell = 0; cell < nc; ++cell)
    for (int i = 0; i < nn; ++i)
      for (int r = 0; r < m; ++r) {
        double s = 0.0;
        for (int k = 0; k < nv; ++k) s += F[((long)(k * m + r) * nc + cell) * nn + i];
        W[(cell * nn + i) * m + r] = s;
      }
  return 0;
}

// Relaxation at every node (eq:over_relaxation):
//   W = sum_k F_k;  F_k <- omega M_k(W) + (1 - omega) F_k.
// With a source S(W) = -sigma_c W_c (per component), step 3 of the kinetic
// algorithm (Sec. 2.3) first replaces W by the Crank-Nicolson solution of
// dW/dt = S(W) over dt (eq:source_term_application_to_W):
//   W+_c = mu_c W_c,  mu_c = (1 - sigma_c dt/2) / (1 + sigma_c dt/2)
// (mu_c = -1 for sigma_c = +inf, the perfect-conductor limit), and the kinetic
// data follow the equilibrium part of that change, F_k += M_k(W+) - M_k(W),
// so that sum_k F_k = W+ before the relaxation towards M_k(W+).
int orc_relax(const orc_config* c, double* F) {
  if (validate(c)) return 1;
  long nc = ncell_of(c);
  int nn = nn_of(c), m = c->m, nv = c->n_vel;
  std::vector<double> W(m), Wp(m), M(nv * m), Mp(nv * m), mu(m, 1.0);
  double om = c->omega;
  bool src = c->source_sigma != nullptr;
  if (src)
    for (int r = 0; r < m; ++r) {
      double sg = c->source_sigma[r];
      mu[r] = std::isinf(sg) ? -1.0 : (1.0 - 0.5 * sg * c->dt) / (1.0 + 0.5 * sg * c->dt);
    }
  for (long cell = 0; cell < nc; ++cell)
    for (int i = 0; i < nn; ++i) {
      for (int r = 0; r < m; ++r) {
        double s = 0.0;
        for (int k = 0; k < nv; ++k) s += F[((long)(k * m + r) * nc + cell) * nn + i];
        W[r] = s;
        Wp[r] = mu[r] * s;
      }
      if (orc_equilibrium(c, Wp.data(), Mp.data())) return 1;
      if (src && orc_equilibrium(c, W.data(), M.data())) return 1;
      for (int k = 0; k < nv; ++k)
        for (int r = 0; r < m; ++r) {
          double& f = F[((long)(k * m + r) * nc + cell) * nn + i];
          if (src) f += Mp[k * m + r] - M[k * m + r];
          f = om * Mp[k * m + r] + (1.0 - om) * f;
        }
    }
  return 0;
}

// n_steps full time steps (Sec. 2.2): transport of every (k, c) field, then
// relaxation.  The (k, c) transports are independent; n_threads > 1 runs them
// concurrently (OpenMP) without changing any arithmetic.  Boundary data: the
// first step goes from bnd_W_old to bnd_W_new, later steps hold bnd_W_new.
int orc_step(const orc_config* c, double* F, int n_steps, int n_threads) {
  if (validate(c) || n_steps < 0) return 1;
  long nc = ncell_of(c);
  int nn = nn_of(c), m = c->m, nv = c->n_vel;
  long slab = nc * nn;
  std::vector<CellOp> ops;
  for (int k = 0; k < nv; ++k) ops.push_back(build_cell_op(c, c->vel + k * c->dim));
  // kinetic boundary data f_k = M_k(W_b) [k][c][boundary node], old and new
  const long nb = n_boundary_nodes(c);
  std::vector<double> fbo(nv * m * nb, 0.0), fbn(nv * m * nb, 0.0), Mb(nv * m);
  auto kinetic = [&](const double* Wb, std::vector<double>& fb) -> int {
    if (!Wb) return 0;
    for (long b = 0; b < nb; ++b) {
      if (orc_equilibrium(c, Wb + b * m, Mb.data())) return 1;
      for (int kc = 0; kc < nv * m; ++kc) fb[kc * nb + b] = Mb[kc];
    }
    return 0;
  };
  if (nb > 0 && (kinetic(c->bnd_W_old, fbo) || kinetic(c->bnd_W_new, fbn))) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  for (int s = 0; s < n_steps; ++s) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int kc = 0; kc < nv * m; ++kc) {
      int k = kc / m;
      std::vector<double> out(slab);
      double* f = F + (long)kc * slab;
      const double* bo = nb > 0 ? fbo.data() + kc * nb : nullptr;
      const double* bn = nb > 0 ? fbn.data() + kc * nb : nullptr;
      err |= transport_scalar(c, ops[k], c->vel + k * c->dim, f, out.data(), bo, bn);
      std::memcpy(f, out.data(), slab * sizeof(double));
    }
    if (err) return err;
    fbo = fbn;  // later steps: the boundary state stays at its end value
    if (orc_relax(c, F)) return 1;
  }
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
