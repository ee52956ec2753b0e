// Host driver of the sanitizer test (tests/test_sanitize_cpu.py): runs the
// library's FP64 setup routines -- Gauss-Lobatto basis, 1-D and dense cell
// operators, equilibrium weights, the linear-law stability checks -- over the
// degrees, dimensions and velocity sets the library accepts, built with
// AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 when every
// routine returned what it should and every output is finite.
#include <cmath>
#include <cstdio>
#include <vector>

#include "kds_internal.h"

using namespace kds;

static int bad = 0;
static double sum = 0.0;

static void take(const std::vector<double>& v, const char* what) {
  for (double x : v) {
    if (!std::isfinite(x)) {
      std::printf("non-finite output of %s\n", what);
      ++bad;
      return;
    }
    sum += x;
  }
}

int main() {
  for (int degree = 1; degree < kMaxP; ++degree) {
    const Basis1D b = make_basis(degree);
    take(b.xi, "make_basis xi");
    take(b.w, "make_basis w");
    take(b.D, "make_basis D");
    for (double nu : {0.25, 1.79, 5.0, 11.0})
      for (double theta : {0.5, 1.0}) {
        const LineOp op = make_line_op(b, nu, theta);
        take(op.C, "make_line_op C");
        take(op.e, "make_line_op e");
      }
    const double h[3] = {0.125, 0.25, 0.0625};
    const double vels[][3] = {{1, 0, 0}, {0, -2, 0}, {0, 0, 3}, {1.7, 1.7, 1.7}, {1.7, -1.7, -1.7},
                              {-1.7, 1.7, -1.7}, {-1, -1, 1}, {0.5, -0.25, 0}};
    for (int dim = 2; dim <= 3; ++dim)
      for (const auto& V : vels) {
        if (dim == 2 && V[2] != 0.0) continue;
        std::vector<double> W;
        int nn = 0, nf = 0;
        if (!make_dense_op(b, dim, V, h, 0.3, 0.5, W, nn, nf)) {
          std::printf("make_dense_op refused degree %d dim %d\n", degree, dim);
          ++bad;
        }
        take(W, "make_dense_op");
      }
  }
  // velocity sets: D1Q2, D2Q4, D3Q6, D3Q4, and one that cannot satisfy the
  // moment conditions (all velocities along x in 2-D)
  const double l = 2.0, s = std::sqrt(3.0);
  const std::vector<std::vector<double>> sets = {
      {l, -l},
      {l, 0, -l, 0, 0, l, 0, -l},
      {l, 0, 0, -l, 0, 0, 0, l, 0, 0, -l, 0, 0, 0, l, 0, 0, -l},
      {s, s, s, s, -s, -s, -s, s, -s, -s, -s, s}};
  const int dims[] = {1, 2, 3, 3};
  for (size_t i = 0; i < sets.size(); ++i) {
    const int dim = dims[i], nv = (int)sets[i].size() / dim;
    std::vector<double> a, bw;
    std::string err;
    if (!eq_weights(dim, nv, sets[i].data(), nullptr, nullptr, a, bw, err)) {
      std::printf("eq_weights refused set %zu: %s\n", i, err.c_str());
      ++bad;
      continue;
    }
    take(a, "eq_weights a");
    take(bw, "eq_weights b");
    // a symmetric law (acoustics-like) and a non-symmetric one
    const int m = dim + 1;
    std::vector<double> A((size_t)dim * m * m, 0.0), An = A;
    for (int d = 0; d < dim; ++d) {
      A[(size_t)d * m * m + 0 * m + (d + 1)] = A[(size_t)d * m * m + (d + 1) * m + 0] = 1.0;
      An[(size_t)d * m * m + 0 * m + (d + 1)] = 2.0;
      An[(size_t)d * m * m + (d + 1) * m + 0] = 0.5;
    }
    const EqChecks c1 = check_linear_law(dim, m, nv, A, a, bw);
    const EqChecks c2 = check_linear_law(dim, m, nv, An, a, bw);
    if (!c1.checked || c2.checked || !std::isfinite(c1.min_eig) || std::fabs(c1.wave_speed - 1.0) > 1e-13) {
      std::printf("check_linear_law set %zu: checked %d/%d speed %g\n", i, c1.checked, c2.checked,
                  c1.wave_speed);
      ++bad;
    }
    sum += c1.min_eig;
  }
  {
    const double V[] = {1, 0, 2, 0};  // 2-D, both along x: no solution
    std::vector<double> a, bw;
    std::string err;
    if (eq_weights(2, 2, V, nullptr, nullptr, a, bw, err)) {
      std::printf("eq_weights accepted a degenerate set\n");
      ++bad;
    }
  }
  std::vector<double> ev;
  sym_eigenvalues(4, {4, 1, 0, 0, 1, 3, 1, 0, 0, 1, 2, 1, 0, 0, 1, 1}, ev);
  take(ev, "sym_eigenvalues");
  std::printf("checksum %.17g, failures %d\n", sum, bad);
  return bad == 0 ? 0 : 1;
}
