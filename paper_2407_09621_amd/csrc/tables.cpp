// Host construction of the 1D data (Sec. 2: Lagrange basis on Gauss-Lobatto
// points; Sec. 2.1: 1D mass and stiffness matrices, face evaluators S_f,
// D_f) and of the fast-diagonalization pairs of the vertex-patch and coarse
// 1D matrices.
#include "tables.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace sipg {

namespace {

// Legendre P_n(t) and P_{n-1}(t) by the three-term recurrence.
void legendre(int n, double t, double& pn, double& pn1) {
  double p0 = 1.0, p1 = t;
  if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// Gauss-Lobatto points of degree k on [-1,1]: the endpoints and the roots
// of P_k', found by Newton's method with P_k'' from Legendre's equation.
std::vector<double> gll_points_pm1(int k) {
  std::vector<double> t(k + 1);
  t[0] = -1.0;
  t[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double x = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre(k, x, p, pm);
      double dp = k * (x * p - pm) / (x * x - 1.0);
      double d2p = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = x;
  }
  return t;
}

std::vector<double> barycentric_weights(const std::vector<double>& x) {
  const int n = (int)x.size();
  std::vector<double> w(n, 1.0);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (a != b) w[a] /= (x[a] - x[b]);
  return w;
}

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre(n, t, p, pm);
      dp = n * (t * p - pm) / (t * t - 1.0);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p, pm;
    legendre(n, t, p, pm);
    dp = n * (t * p - pm) / (t * t - 1.0);
    // map [-1,1] -> [0,1]
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) halved
  }
}

// Values (and optionally derivatives) of the Lagrange basis of `nodes` at
// the points x, row-major [x.size() x N].  Values by the barycentric formula,
// derivatives through the nodal differentiation matrix (phi_a' is a
// polynomial of degree k-1 and is reproduced by its nodal interpolant).
void lagrange_eval(const std::vector<double>& nodes, const std::vector<double>& x,
                   std::vector<double>& val, std::vector<double>* der) {
  const int N = (int)nodes.size();
  const int Q = (int)x.size();
  std::vector<double> bw = barycentric_weights(nodes);
  val.assign((size_t)Q * N, 0.0);
  for (int q = 0; q < Q; ++q) {
    int hit = -1;
    for (int a = 0; a < N; ++a)
      if (x[q] == nodes[a]) hit = a;
    if (hit >= 0) {
      val[(size_t)q * N + hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int a = 0; a < N; ++a) den += bw[a] / (x[q] - nodes[a]);
    for (int a = 0; a < N; ++a) val[(size_t)q * N + a] = bw[a] / (x[q] - nodes[a]) / den;
  }
  if (der) {
    // Dn[b][a] = phi_a'(x_b)
    std::vector<double> Dn((size_t)N * N, 0.0);
    for (int b = 0; b < N; ++b) {
      double diag = 0.0;
      for (int a = 0; a < N; ++a) {
        if (a == b) continue;
        double v = (bw[a] / bw[b]) / (nodes[b] - nodes[a]);
        Dn[(size_t)b * N + a] = v;
        diag -= v;
      }
      Dn[(size_t)b * N + b] = diag;
    }
    der->assign((size_t)Q * N, 0.0);
    for (int q = 0; q < Q; ++q)
      for (int a = 0; a < N; ++a) {
        double s = 0.0;
        for (int b = 0; b < N; ++b) s += val[(size_t)q * N + b] * Dn[(size_t)b * N + a];
        (*der)[(size_t)q * N + a] = s;
      }
  }
}

Tables1D make_tables_1d(int k, double penalty_scale) {
  if (k < 1 || k > kMaxN - 1) throw std::invalid_argument("degree out of range");
  Tables1D t;
  t.k = k;
  const int N = k + 1;
  t.N = N;
  std::vector<double> tp = gll_points_pm1(k);
  t.nodes.resize(N);
  for (int a = 0; a < N; ++a) t.nodes[a] = 0.5 * (tp[a] + 1.0);
  t.nodes[0] = 0.0;
  t.nodes[N - 1] = 1.0;

  std::vector<double> xq, wq, V, D;
  gauss_legendre(N, xq, wq);
  lagrange_eval(t.nodes, xq, V, &D);
  t.mass.assign(N * N, 0.0);
  t.stiff.assign(N * N, 0.0);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      double m = 0.0, s = 0.0;
      for (int q = 0; q < N; ++q) {
        m += wq[q] * V[q * N + a] * V[q * N + b];
        s += wq[q] * D[q * N + a] * D[q * N + b];
      }
      t.mass[a * N + b] = m;
      t.stiff[a * N + b] = s;
    }

  std::vector<double> ends = {0.0, 1.0}, Ve, De;
  lagrange_eval(t.nodes, ends, Ve, &De);
  t.d0.assign(De.begin(), De.begin() + N);
  t.d1.assign(De.begin() + N, De.end());
  const double g = 2.0 * k * (k + 1) * penalty_scale;
  t.gamma_hat = g;

  // 1D face terms (from the SIPG face integral on a point face with jump
  // u_left - u_right and the average of the two one-sided derivatives;
  // boundary points use the outward normal).  s0 = e_0, s1 = e_{N-1}.
  auto e = [&](int a, int b) { return a == b ? 1.0 : 0.0; };
  const int L = N - 1;
  std::vector<double> LL(N * N), RR(N * N), B0(N * N), B1(N * N);
  t.lr.assign(N * N, 0.0);
  t.rl.assign(N * N, 0.0);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      double s1a = e(a, L), s1b = e(b, L), s0a = e(a, 0), s0b = e(b, 0);
      LL[a * N + b] = g * s1a * s1b - 0.5 * (s1a * t.d1[b] + t.d1[a] * s1b);
      RR[a * N + b] = g * s0a * s0b + 0.5 * (s0a * t.d0[b] + t.d0[a] * s0b);
      t.lr[a * N + b] = -g * s1a * s0b - 0.5 * s1a * t.d0[b] + 0.5 * t.d1[a] * s0b;
      t.rl[a * N + b] = -g * s0a * s1b + 0.5 * s0a * t.d1[b] - 0.5 * t.d0[a] * s1b;
      B0[a * N + b] = g * s0a * s0b + (s0a * t.d0[b] + t.d0[a] * s0b);
      B1[a * N + b] = g * s1a * s1b - (s1a * t.d1[b] + t.d1[a] * s1b);
    }
  for (int v = 0; v < 4; ++v) t.lcell[v] = t.stiff;
  for (int i = 0; i < N * N; ++i) {
    t.lcell[0][i] += RR[i] + LL[i];  // interior: left face and right face
    t.lcell[1][i] += B0[i] + LL[i];  // at x = 0
    t.lcell[2][i] += RR[i] + B1[i];  // at x = 1
    t.lcell[3][i] += B0[i] + B1[i];  // single cell
  }
  return t;
}

bool generalized_eig(int n, const std::vector<double>& Lm, const std::vector<double>& Mm,
                     std::vector<double>& S, std::vector<double>& lam) {
  // Cholesky M = C C^T
  std::vector<double> C((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = Mm[j * n + j];
    for (int p = 0; p < j; ++p) s -= C[j * n + p] * C[j * n + p];
    if (s <= 0.0) return false;
    C[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = Mm[i * n + j];
      for (int p = 0; p < j; ++p) t -= C[i * n + p] * C[j * n + p];
      C[i * n + j] = t / C[j * n + j];
    }
  }
  // Ci = C^{-1} (lower triangular)
  std::vector<double> Ci((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Ci[j * n + j] = 1.0 / C[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int p = j; p < i; ++p) s += C[i * n + p] * Ci[p * n + j];
      Ci[i * n + j] = -s / C[i * n + i];
    }
  }
  // B = Ci L Ci^T
  std::vector<double> T((size_t)n * n, 0.0), B((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Ci[i * n + p] * Lm[p * n + j];
      T[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += T[i * n + p] * Ci[j * n + p];
      B[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      double a = 0.5 * (B[i * n + j] + B[j * n + i]);
      B[i * n + j] = B[j * n + i] = a;
    }
  // cyclic Jacobi: B = Q diag Q^T
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += B[i * n + j] * B[i * n + j];
        if (i != j) off += B[i * n + j] * B[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = B[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (B[q * n + q] - B[p * n + p]) / (2.0 * apq);
        double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int r = 0; r < n; ++r) {  // B <- B J
          double bp = B[r * n + p], bq = B[r * n + q];
          B[r * n + p] = c * bp - s * bq;
          B[r * n + q] = s * bp + c * bq;
        }
        for (int r = 0; r < n; ++r) {  // B <- J^T B
          double bp = B[p * n + r], bq = B[q * n + r];
          B[p * n + r] = c * bp - s * bq;
          B[q * n + r] = s * bp + c * bq;
        }
        for (int r = 0; r < n; ++r) {  // Q <- Q J
          double qp = Q[r * n + p], qq = Q[r * n + q];
          Q[r * n + p] = c * qp - s * qq;
          Q[r * n + q] = s * qp + c * qq;
        }
      }
  }
  lam.assign(n, 0.0);
  for (int i = 0; i < n; ++i) lam[i] = B[i * n + i];
  // S = Ci^T Q
  S.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Ci[p * n + i] * Q[p * n + j];
      S[i * n + j] = s;
    }
  return true;
}

namespace {

// Global 1D stiffness-plus-face matrix of `cells` consecutive cells whose
// first cell is (or is not) at the low boundary and whose last cell is (or is
// not) at the high boundary; mass is blockdiag(Mh).
void line_matrices(const Tables1D& t, int cells, bool low_bdry, bool high_bdry,
                   std::vector<double>& Lm, std::vector<double>& Mm) {
  const int N = t.N, G = cells * N;
  Lm.assign((size_t)G * G, 0.0);
  Mm.assign((size_t)G * G, 0.0);
  for (int c = 0; c < cells; ++c) {
    bool lo = (c == 0) && low_bdry, hi = (c == cells - 1) && high_bdry;
    int v = (lo ? 1 : 0) + (hi ? 2 : 0);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        Lm[(size_t)(c * N + a) * G + c * N + b] = t.lcell[v][a * N + b];
        Mm[(size_t)(c * N + a) * G + c * N + b] = t.mass[a * N + b];
        if (c + 1 < cells) {
          Lm[(size_t)(c * N + a) * G + (c + 1) * N + b] = t.lr[a * N + b];
          Lm[(size_t)((c + 1) * N + a) * G + c * N + b] = t.rl[a * N + b];
        }
      }
  }
}

}  // namespace

// Even-odd (mirror-pair) blocks of the degree-7 1D operators.  The GLL
// nodes are symmetric about the cell centre, so the reversal J (node a ->
// N-1-a) maps the mass matrix and the interior cell block of Lh onto
// themselves, the coupling to the upper neighbour onto the coupling to the
// lower one (L_{c,c+1} = J L_{c+1,c} J), and the boundary correction at x = 1
// onto the one at x = 0.  With node index idx(h, a) = h ? N-1-a : a
// (a = 0..3) a vector splits into halves v_0, v_1 (h = 0, 1) and into
// E = v_0 + v_1, O = v_0 - v_1.  A J-symmetric Q maps E to (Q00 + Q01) E and
// O to (Q00 - Q01) O (blocks Qhh'[a][c] = Q[idx(h,a)][idx(h',c)]): one 4 x 4
// block per half instead of two.  For a coupling B and its mirror J B J
// acting on neighbours m and p, with S = v_m + J v_p and D = v_m - J v_p:
// E(B v_m + J B J v_p) = (B00 + B10) S_0 + (B01 + B11) S_1 and
// O(...) = (B00 - B10) D_0 + (B01 - B11) D_1.
// Blocks (row-major 4 x 4): 0-1 mass even/odd, 2-3 interior cell block
// even/odd, 4-7 lower coupling L_{c+1,c} as (e0, e1, o0, o1), 8-11 the
// boundary correction at x = 0, Lcell[1] - Lcell[0], in the same form.
// Returns false (blocks unusable) if a symmetry fails beyond rounding.
bool even_odd_blocks(const Tables1D& t, double* out) {
  const int N = t.N;
  if (N != 8) return false;
  auto at = [&](const std::vector<double>& q, int i, int j) { return q[i * N + j]; };
  std::vector<double> dlt(N * N), dhi(N * N), dboth(N * N);
  for (int i = 0; i < N * N; ++i) {
    dlt[i] = t.lcell[1][i] - t.lcell[0][i];
    dhi[i] = t.lcell[2][i] - t.lcell[0][i];
    dboth[i] = t.lcell[3][i] - t.lcell[0][i];
  }
  double scale = 0.0, dev = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const int mi = N - 1 - i, mj = N - 1 - j;
      scale = std::max(scale, std::fabs(at(t.lcell[0], i, j)) + std::fabs(at(t.rl, i, j)));
      dev = std::max(dev, std::fabs(at(t.mass, i, j) - at(t.mass, mi, mj)));
      dev = std::max(dev, std::fabs(at(t.lcell[0], i, j) - at(t.lcell[0], mi, mj)));
      dev = std::max(dev, std::fabs(at(t.lr, i, j) - at(t.rl, mi, mj)));
      dev = std::max(dev, std::fabs(at(dhi, i, j) - at(dlt, mi, mj)));
      dev = std::max(dev, std::fabs(at(dboth, i, j) - at(dlt, i, j) - at(dlt, mi, mj)));
    }
  if (!(dev <= 1e-12 * scale)) return false;
  auto idx = [&](int h, int a) { return h ? N - 1 - a : a; };
  auto sym = [&](const std::vector<double>& q, double* e, double* o) {
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        e[a * 4 + c] = at(q, idx(0, a), idx(0, c)) + at(q, idx(0, a), idx(1, c));
        o[a * 4 + c] = at(q, idx(0, a), idx(0, c)) - at(q, idx(0, a), idx(1, c));
      }
  };
  auto cpl = [&](const std::vector<double>& q, double* b) {
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        const double b00 = at(q, idx(0, a), idx(0, c)), b01 = at(q, idx(0, a), idx(1, c));
        const double b10 = at(q, idx(1, a), idx(0, c)), b11 = at(q, idx(1, a), idx(1, c));
        b[0 * 16 + a * 4 + c] = b00 + b10;
        b[1 * 16 + a * 4 + c] = b01 + b11;
        b[2 * 16 + a * 4 + c] = b00 - b10;
        b[3 * 16 + a * 4 + c] = b01 - b11;
      }
  };
  sym(t.mass, out + 0 * 16, out + 1 * 16);
  sym(t.lcell[0], out + 2 * 16, out + 3 * 16);
  cpl(t.rl, out + 4 * 16);
  cpl(dlt, out + 8 * 16);
  return true;
}

// Even-odd half-blocks of an N x N matrix Q with Q[N-1-a][N-1-b] = Q[a][b]
// (true of the mass matrix and the interior cell block: the GLL nodes are
// symmetric about the cell centre and the two faces of an interior cell
// enter alike): QE[a][b] = (Q[a][b] + Q[a][N-1-b]) / 2 for b < N/2 and
// Q[a][mid] / 2 in the middle column of odd N, QO[a][b] = (Q[a][b] -
// Q[a][N-1-b]) / 2, rows a < (N+1)/2 and a < N/2.  Written to out as QE then
// QO.  Returns false if the symmetry fails beyond rounding.
bool half_blocks(const std::vector<double>& Q, int N, double* out) {
  const int P = N / 2, PE = (N + 1) / 2;
  double scale = 0.0, dev = 0.0;
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      scale = std::max(scale, std::fabs(Q[a * N + b]));
      dev = std::max(dev, std::fabs(Q[a * N + b] - Q[(N - 1 - a) * N + N - 1 - b]));
    }
  if (!(dev <= 1e-12 * scale)) return false;
  double* QE = out;
  double* QO = out + PE * PE;
  for (int a = 0; a < PE; ++a)
    for (int b = 0; b < PE; ++b)
      QE[a * PE + b] = (b == N - 1 - b) ? 0.5 * Q[a * N + b] : 0.5 * (Q[a * N + b] + Q[a * N + N - 1 - b]);
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b) QO[a * P + b] = 0.5 * (Q[a * N + b] - Q[a * N + N - 1 - b]);
  return true;
}

// Window matrices of the patch-wise evaluation (Sec. 2.1, Fig. patch_int):
// the 2N x 2N stiffness-plus-face matrix of a window of two cells a, b
// (h-free) holds the whole interior face between them, the boundary face of
// a cell that ends the line, and the cell stiffness times the cell's share
// (1 for the first and last cell of the line, which lie in one window, 1/2
// otherwise):
//   [[w_a K + F_aa (+ B_0), F_ab], [F_ba, w_b K + F_bb (+ B_1)]]
// with the face blocks of the interior face (as in the global 1D matrix).
// Summed over the windows of a line this is the global 1D matrix.
void window_matrices(const Tables1D& t, double* out) {
  const int N = t.N, G = 2 * N;
  const double g = t.gamma_hat;
  auto e0 = [&](int i) { return i == 0 ? 1.0 : 0.0; };
  auto e1 = [&](int i) { return i == N - 1 ? 1.0 : 0.0; };
  for (int type = 0; type < 4; ++type) {
    const bool lo = type & 1, hi = type & 2;
    const double wa = lo ? 1.0 : 0.5, wb = hi ? 1.0 : 0.5;
    double* W = out + type * G * G;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const double K = t.stiff[i * N + j];
        // right face of the lower cell a, left face of the upper cell b
        const double faa = g * e1(i) * e1(j) - 0.5 * (e1(i) * t.d1[j] + t.d1[i] * e1(j));
        const double fbb = g * e0(i) * e0(j) + 0.5 * (e0(i) * t.d0[j] + t.d0[i] * e0(j));
        const double b0 = g * e0(i) * e0(j) + (e0(i) * t.d0[j] + t.d0[i] * e0(j));
        const double b1 = g * e1(i) * e1(j) - (e1(i) * t.d1[j] + t.d1[i] * e1(j));
        W[i * G + j] = wa * K + faa + (lo ? b0 : 0.0);
        W[(N + i) * G + N + j] = wb * K + fbb + (hi ? b1 : 0.0);
        W[i * G + N + j] = t.lr[i * N + j];
        W[(N + i) * G + j] = t.rl[i * N + j];
      }
  }
}

// Even-odd form of the fast diagonalization of a G x G patch pencil (L, M)
// that is symmetric under the reversal J of its G nodes: the eigenvectors
// split into J-even ones, s = P y with P = [I; J] / sqrt 2, and J-odd ones,
// s = Q y with Q = [I; -J] / sqrt 2, where y solves the H x H pencil
// (P^T L P, P^T M P) (entries L[a][b] + L[a][G-1-b]) or (Q^T L Q, Q^T M Q)
// (L[a][b] - L[a][G-1-b]).  Stores YE / sqrt 2, YO / sqrt 2, lamE, lamO.
// Returns false when the pencil is not reversal-symmetric (to 1e-12).
bool fd_even_odd(int G, const std::vector<double>& Lm, const std::vector<double>& Mm,
                 double* out) {
  const int H = G / 2;
  double scale = 0.0;
  for (double v : Lm) scale = std::max(scale, std::fabs(v));
  for (int i = 0; i < G; ++i)
    for (int j = 0; j < G; ++j) {
      const int ri = G - 1 - i, rj = G - 1 - j;
      if (std::fabs(Lm[ri * G + rj] - Lm[i * G + j]) > 1e-12 * scale ||
          std::fabs(Mm[ri * G + rj] - Mm[i * G + j]) > 1e-12)
        return false;
    }
  std::vector<double> LE(H * H), ME(H * H), LO(H * H), MO(H * H), Y, lam;
  for (int a = 0; a < H; ++a)
    for (int b = 0; b < H; ++b) {
      LE[a * H + b] = Lm[a * G + b] + Lm[a * G + G - 1 - b];
      LO[a * H + b] = Lm[a * G + b] - Lm[a * G + G - 1 - b];
      ME[a * H + b] = Mm[a * G + b] + Mm[a * G + G - 1 - b];
      MO[a * H + b] = Mm[a * G + b] - Mm[a * G + G - 1 - b];
    }
  const double r2 = 1.0 / std::sqrt(2.0);
  if (!generalized_eig(H, LE, ME, Y, lam)) return false;
  for (int i = 0; i < H * H; ++i) out[i] = Y[i] * r2;
  for (int i = 0; i < H; ++i) out[2 * H * H + i] = lam[i];
  if (!generalized_eig(H, LO, MO, Y, lam)) return false;
  for (int i = 0; i < H * H; ++i) out[H * H + i] = Y[i] * r2;
  for (int i = 0; i < H; ++i) out[2 * H * H + H + i] = lam[i];
  return true;
}

std::vector<double> build_device_table(int k, int n0, TableLayout& lay, double penalty_scale) {
  Tables1D t = make_tables_1d(k, penalty_scale);
  const int N = t.N, G = 2 * N, Gc = (n0 >= 1 && n0 <= 3) ? n0 * N : 0;
  lay = TableLayout();
  lay.N = N;
  lay.G = G;
  lay.Gc = Gc;
  int off = 0;
  auto take = [&](int count) { int o = off; off += count; return o; };
  lay.mass = take(N * N);
  lay.lcell = take(4 * N * N);
  lay.d0 = take(N);
  lay.d1 = take(N);
  lay.gam = take(2);
  lay.fd_s = take(4 * G * G);
  lay.fd_l = take(4 * G);
  lay.fdc_s = take(Gc * Gc);
  lay.fdc_l = take(Gc);
  lay.p1 = take(2 * N * N);
  lay.lr = take(N * N);
  lay.rl = take(N * N);
  lay.eo = take(N == 8 ? 12 * 16 : 0);
  lay.fd_eo = take(2 * (G / 2) * (G / 2) + G);
  lay.pw_l = take(4 * G * G);
  lay.sym = take(2 * (((N + 1) / 2) * ((N + 1) / 2) + (N / 2) * (N / 2)));
  lay.total = off;
  std::vector<double> tab(off, 0.0);
  for (int i = 0; i < N * N; ++i) tab[lay.mass + i] = t.mass[i];
  for (int v = 0; v < 4; ++v)
    for (int i = 0; i < N * N; ++i) tab[lay.lcell + v * N * N + i] = t.lcell[v][i];
  for (int a = 0; a < N; ++a) {
    tab[lay.d0 + a] = t.d0[a];
    tab[lay.d1 + a] = t.d1[a];
  }
  for (int i = 0; i < N * N; ++i) {
    tab[lay.lr + i] = t.lr[i];
    tab[lay.rl + i] = t.rl[i];
  }
  tab[lay.gam] = t.gamma_hat;
  std::vector<double> Lm, Mm, S, lam;
  for (int type = 0; type < 4; ++type) {
    line_matrices(t, 2, type & 1, type & 2, Lm, Mm);
    if (!generalized_eig(G, Lm, Mm, S, lam)) throw std::runtime_error("patch mass not SPD");
    for (int i = 0; i < G * G; ++i) tab[lay.fd_s + type * G * G + i] = S[i];
    for (int i = 0; i < G; ++i) tab[lay.fd_l + type * G + i] = lam[i];
    if (type == 0) lay.fd_eo_ok = fd_even_odd(G, Lm, Mm, &tab[lay.fd_eo]) ? 1 : 0;
  }
  if (Gc > 0) {  // exact coarse solve only for 1, 2 or 3 coarse cells per direction
    line_matrices(t, n0, true, true, Lm, Mm);
    if (!generalized_eig(Gc, Lm, Mm, S, lam)) throw std::runtime_error("coarse mass not SPD");
    for (int i = 0; i < Gc * Gc; ++i) tab[lay.fdc_s + i] = S[i];
    for (int i = 0; i < Gc; ++i) tab[lay.fdc_l + i] = lam[i];
  }
  // P1[(c, a), b] = phi_b((x_a + c) / 2): coarse basis at the fine nodes
  std::vector<double> pts(2 * N), val;
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < N; ++a) pts[c * N + a] = 0.5 * (t.nodes[a] + c);
  lagrange_eval(t.nodes, pts, val, nullptr);
  for (int i = 0; i < 2 * N * N; ++i) tab[lay.p1 + i] = val[i];
  if (N == 8) lay.eo_ok = even_odd_blocks(t, &tab[lay.eo]) ? 1 : 0;
  window_matrices(t, &tab[lay.pw_l]);
  if (!half_blocks(t.mass, N, &tab[lay.sym]) ||
      !half_blocks(t.lcell[0], N, &tab[lay.sym] + ((N + 1) / 2) * ((N + 1) / 2) + (N / 2) * (N / 2)))
    throw std::runtime_error("1D mass or interior block not symmetric under reversal");
  return tab;
}

}  // namespace sipg
