// kds_setup.cpp -- one-time FP64 host setup of libkds: Gauss-Lobatto basis,
// the 1-D cell operator of the implicit upwind DG transport and its local
// inverse, equilibrium weights.
#include <algorithm>
#include <cmath>

#include "kds_internal.h"

namespace kds {

namespace {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence; P_n' from the
// recurrence P_n' = n P_{n-1} + x P_{n-1}'.
void legendre_pd(int n, double x, double& Pn, double& dPn) {
  double pm1 = 1.0, dpm1 = 0.0;  // P_0
  if (n == 0) { Pn = 1.0; dPn = 0.0; return; }
  double p = x, dp = 1.0;        // P_1
  for (int k = 2; k <= n; ++k) {
    double pk = ((2 * k - 1) * x * p - (k - 1) * pm1) / k;
    double dpk = k * p + x * dp;
    pm1 = p; dpm1 = dp;
    p = pk; dp = dpk;
  }
  (void)dpm1;
  Pn = p;
  dPn = dp;
}

}  // namespace

// Gauss-Lobatto points on [0, 1]: the end points and the zeros of P_p'.  The
// interior zeros are found by Newton's method on P_p' with P_p'' taken from
// Legendre's equation (1 - x^2) P'' = 2 x P' - p (p + 1) P.
// Weights 2 / (p (p + 1) P_p(x_j)^2) on [-1, 1], halved on [0, 1].
Basis1D make_basis(int degree) {
  Basis1D b;
  int P = degree + 1;
  b.P = P;
  b.xi.assign(P, 0.0);
  b.w.assign(P, 0.0);
  b.D.assign(P * P, 0.0);
  if (P == 1) {  // cell average, finite-volume limit
    b.xi[0] = 0.5;
    b.w[0] = 1.0;
    return b;
  }
  int p = degree;
  std::vector<double> x(P);
  x[0] = -1.0;
  x[P - 1] = 1.0;
  for (int j = 1; j < p; ++j) {
    double z = -std::cos(M_PI * j / p);  // Chebyshev-Lobatto point as initial guess
    for (int it = 0; it < 60; ++it) {
      double Pp, dP;
      legendre_pd(p, z, Pp, dP);
      double d2P = (2.0 * z * dP - p * (p + 1.0) * Pp) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * (1.0 + std::fabs(z))) break;
    }
    x[j] = z;
  }
  for (int j = 0; j < P; ++j) {
    double Pp, dP;
    legendre_pd(p, x[j], Pp, dP);
    b.w[j] = 1.0 / (p * (p + 1.0) * Pp * Pp);  // (2 / (...)) / 2
    b.xi[j] = 0.5 * (1.0 + x[j]);
  }
  // barycentric differentiation matrix on the [0, 1] points
  std::vector<double> lam(P, 1.0);
  for (int j = 0; j < P; ++j)
    for (int k = 0; k < P; ++k)
      if (k != j) lam[j] /= (b.xi[j] - b.xi[k]);
  for (int r = 0; r < P; ++r) {
    double diag = 0.0;
    for (int a = 0; a < P; ++a) {
      if (a == r) continue;
      double v = (lam[a] / lam[r]) / (b.xi[r] - b.xi[a]);
      b.D[r * P + a] = v;
      diag -= v;
    }
    b.D[r * P + r] = diag;
  }
  return b;
}

namespace {

// In-place inverse of an n x n matrix (Gauss-Jordan, partial pivoting).
bool invert(int n, std::vector<double>& A) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    double inv = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= inv; I[c * n + k] *= inv; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  A.swap(I);
  return true;
}

}  // namespace

// 1-D operator along the velocity, in downwind node order (node 0 on the
// inflow face, node P-1 on the outflow face).  Dividing eq:dg_imp by the
// lumped mass h w_a, the residual per node is (|V|/h) [(L f)_a - l_a t] with
//   L_ab = -(w_b / w_a) l_a'(xi_b) + delta_{a,P-1} delta_{b,P-1} / w_{P-1}
//   l_a  = delta_{a,0} / w_0,
// so the theta-scheme (I + theta nu L) f^n = (I - (1-theta) nu L) f^{n-1}
// + nu l (theta t^n + (1-theta) t^{n-1}) gives C = A^{-1} B, e = nu A^{-1} l.
LineOp make_line_op(const Basis1D& b, double nu, double theta) {
  int P = b.P;
  LineOp op;
  op.P = P;
  op.nu = nu;
  std::vector<double> L(P * P, 0.0), l(P, 0.0);
  for (int a = 0; a < P; ++a)
    for (int c = 0; c < P; ++c) L[a * P + c] = -(b.w[c] / b.w[a]) * b.D[c * P + a];
  L[(P - 1) * P + (P - 1)] += 1.0 / b.w[P - 1];
  l[0] += 1.0 / b.w[0];
  std::vector<double> A(P * P), B(P * P);
  for (int i = 0; i < P * P; ++i) {
    double id = (i / P == i % P) ? 1.0 : 0.0;
    A[i] = id + theta * nu * L[i];
    B[i] = id - (1.0 - theta) * nu * L[i];
  }
  invert(P, A);
  op.C.assign(P * P, 0.0);
  op.e.assign(P, 0.0);
  for (int r = 0; r < P; ++r) {
    for (int c = 0; c < P; ++c) {
      double s = 0.0;
      for (int k = 0; k < P; ++k) s += A[r * P + k] * B[k * P + c];
      op.C[r * P + c] = s;
    }
    double s = 0.0;
    for (int k = 0; k < P; ++k) s += A[r * P + k] * l[k];
    op.e[r] = nu * s;
  }
  return op;
}

// Equilibrium weights.  The moment conditions of eq:maxwell_def hold for all
// W iff  sum_k a_k = 1, sum_k V_k^i a_k = 0, sum_k b_kj = 0,
// sum_k V_k^i b_kj = delta_ij,  i.e.  R [a | b] = I with R = [1 ; V^T]
// ((d+1) x n_vel).  Minimum-norm solution: [a | b] = R^T (R R^T)^{-1},
// computed with a Cholesky factorisation of the Gram matrix R R^T.
bool eq_weights(int dim, int nv, const double* vel, const double* eq_a, const double* eq_b,
                std::vector<double>& a, std::vector<double>& b, std::string& err) {
  a.assign(nv, 0.0);
  b.assign(nv * dim, 0.0);
  if (eq_a && eq_b) {
    for (int k = 0; k < nv; ++k) {
      a[k] = eq_a[k];
      for (int i = 0; i < dim; ++i) b[k * dim + i] = eq_b[k * dim + i];
    }
    return true;
  }
  if (eq_a || eq_b) { err = "eq_a and eq_b must both be given or both be NULL"; return false; }
  int r = dim + 1;
  auto R = [&](int row, int k) { return row == 0 ? 1.0 : vel[k * dim + row - 1]; };
  std::vector<double> G(r * r, 0.0), Lc(r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      for (int k = 0; k < nv; ++k) G[i * r + j] += R(i, k) * R(j, k);
  for (int j = 0; j < r; ++j) {
    double s = G[j * r + j];
    for (int k = 0; k < j; ++k) s -= Lc[j * r + k] * Lc[j * r + k];
    if (!(s > 1e-14 * (1.0 + G[j * r + j]))) {
      err = "kinetic velocities do not span the moment conditions (eq:maxwell_def has no solution)";
      return false;
    }
    Lc[j * r + j] = std::sqrt(s);
    for (int i = j + 1; i < r; ++i) {
      double t = G[i * r + j];
      for (int k = 0; k < j; ++k) t -= Lc[i * r + k] * Lc[j * r + k];
      Lc[i * r + j] = t / Lc[j * r + j];
    }
  }
  // Ginv columns by forward/back substitution
  std::vector<double> Gi(r * r, 0.0);
  for (int c = 0; c < r; ++c) {
    std::vector<double> y(r, 0.0);
    for (int i = 0; i < r; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= Lc[i * r + k] * y[k];
      y[i] = t / Lc[i * r + i];
    }
    for (int i = r - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < r; ++k) t -= Lc[k * r + i] * Gi[k * r + c];
      Gi[i * r + c] = t / Lc[i * r + i];
    }
  }
  for (int k = 0; k < nv; ++k)
    for (int c = 0; c < r; ++c) {
      double s = 0.0;
      for (int i = 0; i < r; ++i) s += R(i, k) * Gi[i * r + c];
      if (c == 0) a[k] = s; else b[k * dim + c - 1] = s;
    }
  return true;
}

}  // namespace kds

namespace kds {

// Eigenvalues of a symmetric n x n matrix (row-major), by cyclic Jacobi
// rotations: each rotation zeroes one off-diagonal pair; sweeps until the
// off-diagonal mass is negligible.
void sym_eigenvalues(int n, std::vector<double> A, std::vector<double>& ev) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * (tot + 1e-300)) break;
    for (int pq = 0; pq < n * n; ++pq) {
      const int pp = pq / n, q = pq % n;
      if (q <= pp || A[pp * n + q] == 0.0) continue;
      // the angle that zeroes A[pp][q]
      const double tau = (A[q * n + q] - A[pp * n + pp]) / (2.0 * A[pp * n + q]);
      const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
      const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
      for (int k = 0; k < n; ++k) {  // columns pp, q
        const double akp = A[k * n + pp], akq = A[k * n + q];
        A[k * n + pp] = c * akp - sn * akq;
        A[k * n + q] = sn * akp + c * akq;
      }
      for (int k = 0; k < n; ++k) {  // rows pp, q
        const double apk = A[pp * n + k], aqk = A[q * n + k];
        A[pp * n + k] = c * apk - sn * aqk;
        A[q * n + k] = sn * apk + c * aqk;
      }
    }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
}

// Checks of a linear law's kinetic model (warnings; the problem still runs).
//   * Sub-characteristic condition (Sec. 2.1): the kinetic speeds must
//     exceed the largest wave speed, max over directions of |eig(sum_i N_i A^i)|;
//     with symmetric A^i that is at most max_i rho(A^i) times sqrt(d) and at
//     least max_i rho(A^i) -- the check uses the coordinate directions,
//     max_i rho(A^i).
//   * Monotonicity of the equilibrium (the bound lambda must satisfy so that
//     the relaxation keeps the kinetic entropy argument of Sec. 2.2): every
//     dM_k/dW = a_k I + sum_i b_{k,i} A^i positive semidefinite.
// Both need symmetric A^i (then the eigenvalues are real and the Jacobi
// method applies); otherwise checked = false.
EqChecks check_linear_law(int dim, int m, int nv, const std::vector<double>& A,
                          const std::vector<double>& a, const std::vector<double>& b) {
  EqChecks r;
  const double scale = [&] {
    double s = 0.0;
    for (double x : A) s = std::max(s, std::fabs(x));
    return s + 1.0;
  }();
  for (int i = 0; i < dim; ++i)
    for (int u = 0; u < m; ++u)
      for (int v = 0; v < u; ++v)
        if (std::fabs(A[(size_t)i * m * m + u * m + v] - A[(size_t)i * m * m + v * m + u]) >
            1e-12 * scale)
          return r;
  r.checked = true;
  std::vector<double> ev;
  for (int i = 0; i < dim; ++i) {
    sym_eigenvalues(m, std::vector<double>(A.begin() + (size_t)i * m * m, A.begin() + (size_t)(i + 1) * m * m), ev);
    for (double e : ev) r.wave_speed = std::max(r.wave_speed, std::fabs(e));
  }
  r.min_eig = 1e300;
  for (int k = 0; k < nv; ++k) {
    std::vector<double> D(m * m, 0.0);
    for (int u = 0; u < m; ++u) D[u * m + u] = a[k];
    for (int i = 0; i < dim; ++i)
      for (int u = 0; u < m * m; ++u) D[u] += b[k * dim + i] * A[(size_t)i * m * m + u];
    sym_eigenvalues(m, D, ev);
    for (double e : ev) r.min_eig = std::min(r.min_eig, e);
  }
  return r;
}

// Dense cell operator for a velocity V in any direction (Sec. 3.1, eq:dg_imp
// on a Cartesian cell with the tensor Gauss-Lobatto basis).  Per axis a with
// V^a != 0 the residual has the 1-D part (|V^a|/h_a) (L_a f - l_a t_a), applied
// along axis a (downwind node order along a is physical order for V^a > 0 and
// reversed for V^a < 0).  With A = I + theta dt sum_a L_a and
// B = I - (1 - theta) dt sum_a L_a:
//   f^n = A^{-1} B f^{n-1} + sum_a A^{-1} lift_a (theta t_a^n + (1-theta) t_a^{n-1}),
// lift_a mapping the P^{d-1} face values of the upwind neighbour across the
// inflow face of axis a onto the nodes of that face.
// Result: Wop = [C | E_0 | E_1 | E_2], nn x (nn + 3 nf), row-major, with
// E_a = 0 for axes where V^a = 0; face node q enumerates the other axes'
// node indices (x fastest), the neighbour's matching node has the outflow
// index on axis a.
bool make_dense_op(const Basis1D& b, int dim, const double* V, const double* h, double dt,
                   double theta, std::vector<double>& Wop, int& nn, int& nf) {
  const int P = b.P;
  nn = 1;
  for (int a = 0; a < dim; ++a) nn *= P;
  nf = nn / P;
  // 1-D operator in physical node order for a positive velocity, and its mirror
  std::vector<double> Lp(P * P, 0.0);
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) Lp[r * P + c] = -(b.w[c] / b.w[r]) * b.D[c * P + r];
  Lp[(P - 1) * P + (P - 1)] += 1.0 / b.w[P - 1];
  std::vector<double> Lfull(nn * nn, 0.0), A(nn * nn), B(nn * nn);
  auto idx = [&](int i, int a) { for (int t = 0; t < a; ++t) i /= P; return i % P; };
  for (int a = 0; a < dim; ++a) {
    if (V[a] == 0.0) continue;
    const double s = std::fabs(V[a]) / h[a];
    for (int i = 0; i < nn; ++i)
      for (int j = 0; j < nn; ++j) {
        bool same = true;
        for (int o = 0; o < dim; ++o)
          if (o != a && idx(i, o) != idx(j, o)) same = false;
        if (!same) continue;
        int ri = idx(i, a), rj = idx(j, a);
        if (V[a] < 0) { ri = P - 1 - ri; rj = P - 1 - rj; }  // mirror to downwind order
        Lfull[i * nn + j] += s * Lp[ri * P + rj];
      }
  }
  for (int i = 0; i < nn * nn; ++i) {
    const double id = (i / nn == i % nn) ? 1.0 : 0.0;
    A[i] = id + theta * dt * Lfull[i];
    B[i] = id - (1.0 - theta) * dt * Lfull[i];
  }
  std::vector<double> Ai = A;
  if (!invert(nn, Ai)) return false;
  const int K = nn + 3 * nf;
  Wop.assign((size_t)nn * K, 0.0);
  for (int i = 0; i < nn; ++i)
    for (int j = 0; j < nn; ++j) {
      double acc = 0.0;
      for (int t = 0; t < nn; ++t) acc += Ai[i * nn + t] * B[t * nn + j];
      Wop[(size_t)i * K + j] = acc;
    }
  for (int a = 0; a < dim; ++a) {
    if (V[a] == 0.0) continue;
    const int in_idx = V[a] > 0 ? 0 : P - 1;        // inflow face node index on axis a
    const double lift = dt * (std::fabs(V[a]) / h[a]) / b.w[in_idx];
    for (int q = 0; q < nf; ++q) {
      // cell node on the inflow face with the other-axis indices of q
      int node = 0, mul = 1, rem = q;
      for (int o = 0; o < dim; ++o) {
        int io;
        if (o == a) io = in_idx;
        else { io = rem % P; rem /= P; }
        node += io * mul;
        mul *= P;
      }
      for (int i = 0; i < nn; ++i)
        Wop[(size_t)i * K + nn + a * nf + q] = Ai[i * nn + node] * lift;
    }
  }
  return true;
}

}  // namespace kds
