// Host-side 1D data of the SIPG discretization and the layout of the
// per-degree device table that every kernel reads.
//
// All tables are h-free: on a uniform Cartesian level with cell size h the
// operator is A = h * (Mh (x) Mh (x) Lh + Mh (x) Lh (x) Mh + Lh (x) Mh (x) Mh)
// (Sec. 2.1, eq. tensorproduct_3d, with the 1D mass scaling as h and the 1D
// stiffness-plus-face matrix as 1/h), so one table serves every level.
#pragma once
#include <vector>

namespace sipg {

constexpr int kMaxN = 8;  // degree 7

// Offsets (in doubles) of the pieces of the device table for one degree.
struct TableLayout {
  int N = 0;      // nodes per direction, k + 1
  int G = 0;      // patch size per direction, 2N
  int Gc = 0;     // coarse-grid size per direction, n0 * N
  int mass = 0;   // Mh [N x N], row-major
  int lcell = 0;  // Lh cell blocks [4][N x N]: 0 interior, 1 at x=0, 2 at x=1, 3 both
  int d0 = 0;     // phi'(0) [N]
  int d1 = 0;     // phi'(1) [N]
  int gam = 0;    // h-free penalty 2k(k+1) [1]
  int fd_s = 0;   // patch eigenvectors S [4][G x G] (types: bit0 lower cell at
                  // the low boundary, bit1 upper cell at the high boundary)
  int fd_l = 0;   // patch eigenvalues [4][G]
  int fdc_s = 0;  // coarse eigenvectors [Gc x Gc]
  int fdc_l = 0;  // coarse eigenvalues [Gc]
  int p1 = 0;     // 1D prolongation [2N x N]: row (child c, node a), column b
  int lr = 0;     // Lh off-diagonal block L_{c,c+1} [N x N] (coupling to the upper cell)
  int rl = 0;     // Lh off-diagonal block L_{c+1,c} [N x N] (coupling to the lower cell)
  int eo = 0;     // N = 8 only: even-odd blocks [12][4 x 4] of the mirror-pair form (see
                  // build_device_table); eo_ok = 1 when the symmetries they rest on hold
  int eo_ok = 0;
  int sym = 0;    // even-odd half-blocks of Mh and of the interior Lh block:
                  // ME [PE x PE], MO [P x P], LE, LO (P = N/2, PE = (N+1)/2)
  int fd_eo = 0;  // patch fast diagonalization of the interior type 0 in even-odd form
                  // (H = G/2): YE, YO [H x H] (row = node a < H, column = eigenvector,
                  // scaled by 1/sqrt 2), lamE [H], lamO [H]; fd_eo_ok = 1 when the
                  // type-0 patch matrices are symmetric under reversal
  int fd_eo_ok = 0;
  int pw_l = 0;   // patch-wise evaluation: window stiffness-plus-face matrices [4][G x G]
                  // by window type (bit0: lower cell first of the line, bit1: upper
                  // cell last); the window mass is the cell mass times 1/2 or 1
  int mass_f = 0; // float copies for the FP32 path start here (same order)
  int total = 0;
};

struct Tables1D {
  int k = 0, N = 0;
  std::vector<double> nodes;       // GLL points on [0,1]
  std::vector<double> mass, stiff; // Mh, Kh [N x N]
  std::vector<double> lcell[4];    // Lh diagonal blocks by boundary type
  std::vector<double> lr, rl;      // Lh off-diagonal blocks L_{c,c+1}, L_{c+1,c}
  std::vector<double> d0, d1;
  double gamma_hat = 0;
};

// penalty_scale multiplies the h-free penalty 2k(k+1) (1 = the paper's gamma).
Tables1D make_tables_1d(int k, double penalty_scale = 1.0);

// Generalized eigenpairs L S = M S diag(lam), S^T M S = I for symmetric L and
// SPD M of size n (row-major).  Returns false if M is not SPD.
bool generalized_eig(int n, const std::vector<double>& L, const std::vector<double>& M,
                     std::vector<double>& S, std::vector<double>& lam);

// 1D Lagrange basis (values / derivatives) of the GLL nodes at points x.
void lagrange_eval(const std::vector<double>& nodes, const std::vector<double>& x,
                   std::vector<double>& val, std::vector<double>* der);

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Full device table for degree k and coarse size n0; fills `layout`.
std::vector<double> build_device_table(int k, int n0, TableLayout& layout,
                                       double penalty_scale = 1.0);

}  // namespace sipg
