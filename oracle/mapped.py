"""The SIPG Laplacian on a mesh of trilinear hexahedra (general geometry).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2: every cell K is the image of the reference cube [0, 1]^3 under a map
F_K, the shape functions are phi_{K,i} = phi_i o F_K^{-1}, and Sec. 2.1 turns
the cell integral into an integral over the reference cube with the per-point
Jacobian J of F_K:

    A^K_ij = int grad_xi phi_i^T J^{-1} J^{-T} |J| grad_xi phi_j dxi,

evaluated by tensor quadrature (A^K = G_phi^T W G_phi, W holding the
Jacobian terms and the weights).  The face terms of eq. bilinear_form use
the physical normal and surface measure of each face.

Readings:
* Geometry: the mesh is the structured grid of (n+1)^3 vertices; each cell
  is the trilinear map of its 8 vertices, so two cells that share a face see
  the same bilinear surface with the same parametrization.
* Quadrature: N-point Gauss per direction on cells and N x N on faces (the
  rule of the Cartesian operator), so an affine mesh gives the exact
  integrals.  On non-affine cells the integrands are rational and the rule
  defines the discrete operator.
* Penalty: gamma_e = k(k+1)(1/h+ + 1/h-) with h of each side the cell volume
  over the face area (both by the same Gauss rules); boundary faces use
  2k(k+1)/h-.  On a uniform Cartesian mesh h is the cell size, as in
  ``oracle.sipg``.
* With n dsigma = det(J) J^{-T} n_hat dA on the reference face, every face
  term is an integral over the reference face.

Vertex array: V[vz, vy, vx, :] = (x, y, z); cell (cx, cy, cz) has vertex
(a, b, c) in {0, 1}^3 at V[cz + c, cy + b, cx + a], numbered a + 2b + 4c.
Degree-of-freedom layout as in ``oracle.sipg``.
"""
import functools

import numpy as np
import scipy.sparse as sp

from . import basis1d
from .sipg import _coo_block, _face_points, _tensor_basis_at, n_dofs


def cell_vertices(V, cx, cy, cz):
    """The 8 vertices [8, 3] of cell (cx, cy, cz), vertex a + 2b + 4c."""
    return np.array([V[cz + c, cy + b, cx + a] for c in (0, 1) for b in (0, 1) for a in (0, 1)])


def trilinear(X, xi):
    """Positions x [Q, 3] and Jacobians J [Q, 3, 3], J[q, i, d] = dx_i/dxi_d,
    of the trilinear map with vertices X [8, 3] at reference points xi [Q, 3]."""
    xi = np.asarray(xi, dtype=np.float64)
    ell = (1.0 - xi, xi)              # ell[a][:, d]: the 1D hat of corner a
    dell = (-1.0, 1.0)
    x = np.zeros((len(xi), 3))
    J = np.zeros((len(xi), 3, 3))
    for v in range(8):
        a, b, c = v & 1, (v >> 1) & 1, v >> 2
        la, lb, lc = ell[a][:, 0], ell[b][:, 1], ell[c][:, 2]
        x += (la * lb * lc)[:, None] * X[v]
        J[:, :, 0] += (dell[a] * lb * lc)[:, None] * X[v]
        J[:, :, 1] += (la * dell[b] * lc)[:, None] * X[v]
        J[:, :, 2] += (la * lb * dell[c])[:, None] * X[v]
    return x, J


def _cell_rule(k):
    N = k + 1
    x, w = basis1d.gauss_rule(N)
    P = np.array([(a, b, c) for c in x for b in x for a in x])
    W = np.array([wa * wb * wc for wc in w for wb in w for wa in w])
    return P, W


@functools.lru_cache(maxsize=None)
def _cell_basis(k):
    """Gauss points, weights and the reference basis (values, gradients)
    there; the same for every cell."""
    P, W = _cell_rule(k)
    v, g = _tensor_basis_at(k, P, 1.0)
    return P, W, v, g


@functools.lru_cache(maxsize=None)
def _face_basis(k, d, side):
    pts, wq = _face_points(k, d, float(side))
    v, g = _tensor_basis_at(k, pts, 1.0)
    return pts, wq, v, g


def _physical(gref, J):
    """Physical gradients grad phi = J^{-T} grad_xi phi: [Q, N^3, 3]."""
    Jinv = np.linalg.inv(J)                       # [Q, d, i]
    return np.einsum("qdi,qId->qIi", Jinv, gref)


def cell_volume(k, X):
    """|K| = sum_q w_q det J(xi_q) with the N^3-point Gauss rule."""
    P, W = _cell_rule(k)
    _, J = trilinear(X, P)
    return float(W @ np.linalg.det(J))


def face_area(k, X, d, side):
    """|e| of the face xi_d = side of the cell with vertices X, by the N x N
    Gauss rule: dsigma = |det(J) J^{-T} e_d| dA."""
    pts, wq = _face_points(k, d, float(side))
    _, J = trilinear(X, pts)
    nu = np.linalg.det(J)[:, None] * np.linalg.inv(J)[:, d, :]   # det J * (J^{-T} e_d)
    return float(wq @ np.linalg.norm(nu, axis=1))


def cell_matrix_mapped(k, X):
    """int_K grad phi_I . grad phi_J dx on the trilinear cell X (Sec. 2.1)."""
    P, W, _, gref = _cell_basis(k)
    _, J = trilinear(X, P)
    g = _physical(gref, J)
    wd = W * np.linalg.det(J)
    gi = [np.ascontiguousarray(g[:, :, i]) for i in range(3)]
    return sum(gi[i].T @ (wd[:, None] * gi[i]) for i in range(3))


def _face_side(k, X, d, side):
    """Values, physical gradients and positions of the basis of the cell X on
    its face xi_d = side, and n dsigma / dA there (outward)."""
    pts, wq, v, gref = _face_basis(k, d, side)
    x, J = trilinear(X, pts)
    g = _physical(gref, J)
    sign = 1.0 if side == 1 else -1.0
    nu = sign * np.linalg.det(J)[:, None] * np.linalg.inv(J)[:, d, :]
    return v, g, x, nu, wq


def interior_face_blocks_mapped(k, Xm, Xp, d, penalty_scale=1.0):
    """The four blocks of the interior-face form on the face between K- (its
    side xi_d = 1, vertices Xm) and K+ (its side xi_d = 0, vertices Xp):
    block[(t, s)][I, J] = a_e(phi_J on K_s, phi_I on K_t)."""
    vm, gm, xm, nu, wq = _face_side(k, Xm, d, 1)
    vp, gp, xp, _, _ = _face_side(k, Xp, d, 0)
    if not np.allclose(xm, xp, rtol=0, atol=1e-12 * max(1.0, np.abs(xm).max())):
        raise ValueError("the two cells do not share the face")
    ds = np.linalg.norm(nu, axis=1)
    n_minus = nu / ds[:, None]
    area = float(wq @ ds)
    hm = cell_volume(k, Xm) / area
    hp = cell_volume(k, Xp) / area
    gamma = penalty_scale * k * (k + 1) * (1.0 / hm + 1.0 / hp)
    w = wq * ds
    side = {'-': (vm, gm, n_minus), '+': (vp, gp, -n_minus)}
    blocks = {}
    for t in '-+':
        vt, gt, nt = side[t]
        for s in '-+':
            vs, gs, ns = side[s]
            # sum over the face points q of w_q times
            #   gamma [[phi_J]].[[phi_I]] - {grad phi_J}.[[phi_I]] - [[phi_J]].{grad phi_I}
            # written as products over q (rows I: test functions on K_t)
            nn = np.einsum("qi,qi->q", ns, nt)
            gs_nt = np.einsum("qJi,qi->qJ", gs, nt)
            gt_ns = np.einsum("qIi,qi->qI", gt, ns)
            blocks[(t, s)] = (gamma * vt.T @ ((w * nn)[:, None] * vs)
                              - 0.5 * vt.T @ (w[:, None] * gs_nt)
                              - 0.5 * gt_ns.T @ (w[:, None] * vs))
    return blocks


def boundary_face_block_mapped(k, X, d, side, penalty_scale=1.0):
    """Boundary face xi_d = side of the cell X: {v} = v, [[v]] = v n,
    gamma = 2k(k+1)/h with h = |K| / |e|."""
    v, g, _, nu, wq = _face_side(k, X, d, side)
    ds = np.linalg.norm(nu, axis=1)
    n = nu / ds[:, None]
    h = cell_volume(k, X) / float(wq @ ds)
    gamma = penalty_scale * 2.0 * k * (k + 1) / h
    gn = np.einsum("qIi,qi->qI", g, n)
    w = wq * ds
    # sum over q of w_q (gamma phi_I phi_J - phi_I dn phi_J - dn phi_I phi_J)
    return (gamma * v.T @ (w[:, None] * v) - v.T @ (w[:, None] * gn)
            - gn.T @ (w[:, None] * v))


def _check(V, n):
    V = np.asarray(V, dtype=np.float64)
    if V.shape != (n + 1, n + 1, n + 1, 3):
        raise ValueError("vertex array must have shape (n+1, n+1, n+1, 3)")
    return V


def assemble_mapped(n, k, V, boundary_terms=True, penalty_scale=1.0):
    """Sparse CSR matrix of the SIPG form on the trilinear mesh V: cell loop,
    interior-face loop and boundary-face loop of the matrix-free skeleton in
    Sec. 2.1, each local integral by quadrature with per-point Jacobians."""
    V = _check(V, n)
    nb = (k + 1) ** 3
    R, C, D = [], [], []

    def add(r, c, blk):
        rr, cc, dd = _coo_block(np.array([r * nb]), np.array([c * nb]), blk)
        R.append(rr)
        C.append(cc)
        D.append(dd)

    idx = lambda cx, cy, cz: cx + n * cy + n * n * cz
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                c = idx(cx, cy, cz)
                X = cell_vertices(V, cx, cy, cz)
                add(c, c, cell_matrix_mapped(k, X))
                pos = (cx, cy, cz)
                for d in range(3):
                    if pos[d] < n - 1:
                        q = list(pos)
                        q[d] += 1
                        cp = idx(*q)
                        blocks = interior_face_blocks_mapped(k, X, cell_vertices(V, *q), d,
                                                             penalty_scale)
                        add(c, c, blocks[('-', '-')])
                        add(c, cp, blocks[('-', '+')])
                        add(cp, c, blocks[('+', '-')])
                        add(cp, cp, blocks[('+', '+')])
                    if boundary_terms and pos[d] == 0:
                        add(c, c, boundary_face_block_mapped(k, X, d, 0, penalty_scale))
                    if boundary_terms and pos[d] == n - 1:
                        add(c, c, boundary_face_block_mapped(k, X, d, 1, penalty_scale))
    A = sp.coo_matrix((np.concatenate(D), (np.concatenate(R), np.concatenate(C))),
                      shape=(n_dofs(n, k),) * 2).tocsr()
    A.sum_duplicates()
    return A


def apply_cells_mapped(u, n, k, V, cells, penalty_scale=1.0):
    """(A u) restricted to the listed cells, from each cell's own blocks and
    its six faces only (for sampled checks on meshes too large to assemble).
    Returns an array [len(cells), N^3]."""
    V = _check(V, n)
    nb = (k + 1) ** 3
    u = np.asarray(u, dtype=np.float64)
    ublk = lambda c: u[c * nb:(c + 1) * nb]
    out = []
    for c in cells:
        c = int(c)
        pos = [c % n, (c // n) % n, c // (n * n)]
        X = cell_vertices(V, *pos)
        v = cell_matrix_mapped(k, X) @ ublk(c)
        for d in range(3):
            stride = [1, n, n * n][d]
            if pos[d] < n - 1:     # this cell is K- of its upper face
                q = list(pos)
                q[d] += 1
                b = interior_face_blocks_mapped(k, X, cell_vertices(V, *q), d, penalty_scale)
                v += b[('-', '-')] @ ublk(c) + b[('-', '+')] @ ublk(c + stride)
            else:
                v += boundary_face_block_mapped(k, X, d, 1, penalty_scale) @ ublk(c)
            if pos[d] > 0:         # this cell is K+ of its lower face
                q = list(pos)
                q[d] -= 1
                b = interior_face_blocks_mapped(k, cell_vertices(V, *q), X, d, penalty_scale)
                v += b[('+', '+')] @ ublk(c) + b[('+', '-')] @ ublk(c - stride)
            else:
                v += boundary_face_block_mapped(k, X, d, 0, penalty_scale) @ ublk(c)
        out.append(v)
    return np.array(out)


def node_positions(n, k, V):
    """Physical positions [n_dofs, 3] of the GLL nodes of every cell
    (cell-blocked order), through each cell's trilinear map."""
    V = _check(V, n)
    nodes = basis1d.gll_nodes(k)
    P = np.array([(a, b, c) for c in nodes for b in nodes for a in nodes])
    out = []
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                x, _ = trilinear(cell_vertices(V, cx, cy, cz), P)
                out.append(x)
    return np.concatenate(out)


def min_jacobian(n, k, V):
    """Smallest det J over the cell Gauss points and the corners of all cells
    (positive for a valid mesh)."""
    V = _check(V, n)
    P, _ = _cell_rule(k)
    corners = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], float)
    pts = np.concatenate([P, corners])
    m = np.inf
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                _, J = trilinear(cell_vertices(V, cx, cy, cz), pts)
                m = min(m, float(np.linalg.det(J).min()))
    return m


def _mapped_cell_rule(k, nq, X):
    """Physical points [Q, 3] and weights w_q det J [Q] of the nq-point Gauss
    rule per direction on the trilinear cell X, and the reference basis
    values there [Q, N^3]."""
    N = k + 1
    xq, wq = basis1d.gauss_rule(nq)
    P = np.array([(a, b, c) for c in xq for b in xq for a in xq])
    W = np.array([wa * wb * wc for wc in wq for wb in wq for wa in wq])
    x, J = trilinear(X, P)
    Vq = basis1d.lagrange_values(basis1d.gll_nodes(k), xq)
    qi = np.arange(nq ** 3)
    a, b, c = qi % nq, (qi // nq) % nq, qi // (nq * nq)
    loc = np.arange(N ** 3)
    i, j, l = loc % N, (loc // N) % N, loc // (N * N)
    Phi = Vq[a][:, i] * Vq[b][:, j] * Vq[c][:, l]
    return x, W * np.linalg.det(J), Phi


def rhs_mapped(problem, n, k, V):
    """b_I = int_K f phi_I dx on every trilinear cell, (k+2)-point Gauss rule
    per direction with the per-point det J (the Cartesian rule of
    ``oracle.rhs`` on the mapped cells); cell-blocked order."""
    V = _check(V, n)
    out = []
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                x, w, Phi = _mapped_cell_rule(k, k + 2, cell_vertices(V, cx, cy, cz))
                out.append((problem.f(x[:, 0], x[:, 1], x[:, 2]) * w) @ Phi)
    return np.concatenate(out)


def l2_error_mapped(problem, uh, n, k, V):
    """||u - u_h||_L2 over the mapped mesh, (k+3)-point Gauss rule per
    direction with the per-point det J."""
    V = _check(V, n)
    N3 = (k + 1) ** 3
    uh = np.asarray(uh).reshape(n ** 3, N3)
    s = 0.0
    c = 0
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                x, w, Phi = _mapped_cell_rule(k, k + 3, cell_vertices(V, cx, cy, cz))
                e = problem.u(x[:, 0], x[:, 1], x[:, 2]) - Phi @ uh[c]
                s += float(w @ (e * e))
                c += 1
    return float(np.sqrt(s))


def level_vertices(V, n, n_level):
    """Vertices of the level with n_level cells per direction: every
    (n / n_level)-th vertex of the finest level's array."""
    s = n // n_level
    return np.ascontiguousarray(np.asarray(V)[::s, ::s, ::s])


class MappedHierarchy:
    """The V-cycle (Alg. v_cycle) on trilinear cells.  Reading: the residuals
    use the mapped operator of each level (its vertices every 2^j-th fine
    vertex), while the vertex-patch solves and the coarse solve keep the
    exact inverses of the Cartesian operator's patch and coarse matrices,
    which are then approximate inverses; the transfers are the Cartesian
    ones (reference-space embedding of the nested Q_k spaces)."""

    def __init__(self, n, k, V):
        from . import multigrid
        self.H = multigrid.Hierarchy(n, k)       # Cartesian patch factors and coarse solve
        self.A = [assemble_mapped(lev.n, k, level_vertices(V, n, lev.n)) for lev in self.H.levels]

    def _smooth(self, l, x, b, sweeps):
        from . import multigrid
        from scipy.linalg import cho_solve
        lev = self.H.levels[l]
        x = np.array(x, dtype=np.float64, copy=True)
        for _ in range(sweeps):
            for colour in range(8):
                r = b - self.A[l] @ x
                for v, c in lev.patches:
                    if c != colour:
                        continue
                    idx = multigrid.patch_dofs(lev.n, lev.k, v)
                    x[idx] += cho_solve(lev.patch_factor(v), r[idx])
        return x

    def vcycle(self, l, x, b):
        if l == 0:
            return self.H.coarse.solve(b)
        x = self._smooth(l, x, b, self.H.nu_pre)
        r = b - self.A[l] @ x
        rc = self.H.P[l].T @ r
        ec = self.vcycle(l - 1, np.zeros(rc.shape), rc)
        x = x + self.H.P[l] @ ec
        return self._smooth(l, x, b, self.H.nu_post)
