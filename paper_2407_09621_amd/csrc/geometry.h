// Host-side data of the general-geometry (trilinear hexahedra) operator.
#pragma once
#include <string>
#include <vector>

namespace sipg {

// 1D data of the mapped apply: S [N x N], D [N x N] (GLL basis and its
// derivative at the N Gauss points, row = point), Gauss weights [N],
// points [N], phi'(0) [N], phi'(1) [N].
std::vector<double> mapped_table(int k);

// The nq-point Gauss rule on [0, 1] with the GLL basis of degree k there:
// values [nq x N] (row = point), weights [nq], points [nq].
std::vector<double> quad_table(int k, int nq);

// Face penalties k(k+1) s (1/h- + 1/h+), h = cell volume / face area (both by
// the N-point Gauss rules; boundary faces 2k(k+1) s / h-) of the n^3-cell
// level with host vertex array V ((n+1)^3 x 3, [vz][vy][vx][xyz]); gam gets
// n^3 x 6 values, face 2 d + side.  Returns false (and a message) when a
// cell has a non-positive Jacobian determinant at a Gauss point or corner.
bool mapped_penalties(int k, int n, const double* V, double penalty_scale,
                      std::vector<double>& gam, std::string& err);

}  // namespace sipg
