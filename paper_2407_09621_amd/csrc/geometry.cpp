// Host side of the general-geometry operator: the 1D data of the mapped
// apply and the per-face penalties of a level of trilinear hexahedra
// (Sec. 2: gamma_e = k(k+1)(1/h+ + 1/h-), with h of each side read as the
// cell volume over the face area).  Plain C++ (no HIP), so that the CPU
// tests can compile it on its own.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "tables.h"

namespace sipg {

namespace {

// dx_i / dxi_d of the trilinear map through X (vertex a + 2b + 4c at
// X[3 (a + 2b + 4c) + i]) at the reference point (x0, x1, x2)
void trilinear_jacobian(const double* X, double x0, double x1, double x2, double J[3][3]) {
  const double a0 = 1.0 - x0, a1 = 1.0 - x1, a2 = 1.0 - x2;
  for (int i = 0; i < 3; ++i) {
    J[i][0] = (X[3 + i] - X[i]) * a1 * a2 + (X[9 + i] - X[6 + i]) * x1 * a2 +
              (X[15 + i] - X[12 + i]) * a1 * x2 + (X[21 + i] - X[18 + i]) * x1 * x2;
    J[i][1] = (X[6 + i] - X[i]) * a0 * a2 + (X[9 + i] - X[3 + i]) * x0 * a2 +
              (X[18 + i] - X[12 + i]) * a0 * x2 + (X[21 + i] - X[15 + i]) * x0 * x2;
    J[i][2] = (X[12 + i] - X[i]) * a0 * a1 + (X[15 + i] - X[3 + i]) * x0 * a1 +
              (X[18 + i] - X[6 + i]) * a0 * x1 + (X[21 + i] - X[9 + i]) * x0 * x1;
  }
}

// cofactor matrix C (J^{-T} = C / det J) and the determinant
double cofactor(const double J[3][3], double C[3][3]) {
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
}

}  // namespace

std::vector<double> mapped_table(int k) {
  const int N = k + 1;
  const Tables1D t = make_tables_1d(k);
  std::vector<double> g, w, S, D;
  gauss_legendre(N, g, w);
  lagrange_eval(t.nodes, g, S, &D);
  std::vector<double> out;
  out.insert(out.end(), S.begin(), S.end());
  out.insert(out.end(), D.begin(), D.end());
  out.insert(out.end(), w.begin(), w.end());
  out.insert(out.end(), g.begin(), g.end());
  out.insert(out.end(), t.d0.begin(), t.d0.end());
  out.insert(out.end(), t.d1.begin(), t.d1.end());
  return out;
}

std::vector<double> quad_table(int k, int nq) {
  const Tables1D t = make_tables_1d(k);
  std::vector<double> g, w, V;
  gauss_legendre(nq, g, w);
  lagrange_eval(t.nodes, g, V, nullptr);
  std::vector<double> out(V);
  out.insert(out.end(), w.begin(), w.end());
  out.insert(out.end(), g.begin(), g.end());
  return out;
}

bool mapped_penalties(int k, int n, const double* V, double penalty_scale,
                      std::vector<double>& gam, std::string& err) {
  const int N = k + 1;
  std::vector<double> g, w;
  gauss_legendre(N, g, w);
  const size_t n1 = (size_t)n + 1;
  const int nc = n * n * n;
  auto cell_x = [&](int c, double* X) {
    const int p[3] = {c % n, (c / n) % n, c / (n * n)};
    for (int v = 0; v < 8; ++v)
      for (int i = 0; i < 3; ++i)
        X[3 * v + i] = V[(((size_t)(p[2] + (v >> 2)) * n1 + p[1] + ((v >> 1) & 1)) * n1 + p[0] +
                          (v & 1)) * 3 + i];
  };
  // |e| of face xi_d = side by the N x N Gauss rule: sum w |C[:, d]|
  auto area = [&](const double* X, int d, int side) {
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    double a = 0.0;
    for (int q2 = 0; q2 < N; ++q2)
      for (int q1 = 0; q1 < N; ++q1) {
        double xi[3], J[3][3], C[3][3];
        xi[d] = side;
        xi[d1] = g[q1];
        xi[d2] = g[q2];
        trilinear_jacobian(X, xi[0], xi[1], xi[2], J);
        cofactor(J, C);
        a += w[q1] * w[q2] * std::sqrt(C[0][d] * C[0][d] + C[1][d] * C[1][d] + C[2][d] * C[2][d]);
      }
    return a;
  };
  std::vector<double> vol(nc);
  std::vector<int> bad(nc, 0);
  const int nthreads = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  auto volumes = [&](int t0) {
    for (int c = t0; c < nc; c += nthreads) {
      double X[24], J[3][3], C[3][3];
      cell_x(c, X);
      double s = 0.0;
      for (int qz = 0; qz < N; ++qz)
        for (int qy = 0; qy < N; ++qy)
          for (int qx = 0; qx < N; ++qx) {
            trilinear_jacobian(X, g[qx], g[qy], g[qz], J);
            const double det = cofactor(J, C);
            if (!(det > 0.0)) bad[c] = 1;
            s += w[qx] * w[qy] * w[qz] * det;
          }
      for (int v = 0; v < 8; ++v) {
        trilinear_jacobian(X, v & 1, (v >> 1) & 1, v >> 2, J);
        if (!(cofactor(J, C) > 0.0)) bad[c] = 1;
      }
      vol[c] = s;
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(volumes, t);
    for (auto& t : th) t.join();
  }
  for (int c = 0; c < nc; ++c)
    if (bad[c]) {
      err = "cell " + std::to_string(c) +
            " has a non-positive Jacobian determinant (inverted or degenerate cell)";
      return false;
    }
  gam.assign((size_t)nc * 6, 0.0);
  const double kk = (double)k * (k + 1) * penalty_scale;
  auto faces = [&](int t0) {
    for (int c = t0; c < nc; c += nthreads) {
      const int p[3] = {c % n, (c / n) % n, c / (n * n)};
      const int st[3] = {1, n, n * n};
      double X[24];
      cell_x(c, X);
      for (int d = 0; d < 3; ++d) {
        if (p[d] == 0) gam[(size_t)c * 6 + 2 * d] = 2.0 * kk * area(X, d, 0) / vol[c];
        const double a = area(X, d, 1);  // the lower cell's side of the face, as seen from it
        if (p[d] == n - 1) {
          gam[(size_t)c * 6 + 2 * d + 1] = 2.0 * kk * a / vol[c];
        } else {
          const int cn = c + st[d];
          const double ge = kk * (a / vol[c] + a / vol[cn]);
          gam[(size_t)c * 6 + 2 * d + 1] = ge;
          gam[(size_t)cn * 6 + 2 * d] = ge;  // written by this cell only
        }
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(faces, t);
    for (auto& t : th) t.join();
  }
  return true;
}

}  // namespace sipg
