"""Geometric multigrid with a multiplicative vertex-patch smoother
(Sec. 7.1, Alg. v_cycle), FP64, on assembled sparse matrices.

Readings of points the paper leaves open (the smoother is only named
"multiplicative vertex-patch", with references):
* Levels: level 0 is the coarsest; every level is rediscretized with its own
  h (the operator form of Sec. 2 on n_l^3 cells), n_{l-1} = n_l / 2.
* Transfers: the canonical embedding of the nested spaces (coarse function
  evaluated at the fine nodes) for prolongation, its transpose for
  restriction.
* Smoother: one vertex patch per interior vertex (the 2x2x2 cells sharing
  it).  Patches are coloured by the parity of the vertex coordinates
  (8 colours, same-colour patches share no cell).  One sweep visits colours
  0..7 in order; for each colour the residual r = b - A x is formed once and
  every patch of that colour adds its exact local correction
  x_P += A_PP^{-1} r_P, with A_PP the principal submatrix of A on the patch.
  Pre- and post-smoothing use the same order (so the preconditioner is not
  symmetric, as the paper notes for the parallel multiplicative smoother).
* V(2, 2): two pre- and two post-sweeps.  Coarse solve: exact.
* Additive variant (for the comparison the paper draws when it explains why
  the multiplicative smoother makes the preconditioner non-symmetric): one
  residual per sweep, every patch's exact local correction summed, the sum
  damped by omega (1/8 by default: every cell lies in 8 vertex patches).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis1d, sipg


# ---------------------------------------------------------------------------
# Transfers
# ---------------------------------------------------------------------------

def _child_embedding(k, o):
    """E[I, J] = coarse basis phi_J evaluated at fine node I of the child
    with offset o = (ox, oy, oz) in {0,1}^3 inside its parent."""
    N = k + 1
    x = basis1d.gll_nodes(k)
    loc = np.arange(N ** 3)
    i, j, l = loc % N, (loc // N) % N, loc // (N * N)
    pts = np.stack([(o[0] + x[i]) / 2, (o[1] + x[j]) / 2, (o[2] + x[l]) / 2], axis=1)
    val, _ = sipg._tensor_basis_at(k, pts, 1.0)
    return val


def prolongation(nc, k):
    """Sparse P: coarse level (nc^3 cells) -> fine level ((2nc)^3 cells)."""
    nf = 2 * nc
    N3 = (k + 1) ** 3
    R, C, D = [], [], []
    cc = np.arange(nc ** 3)
    cx, cy, cz = cc % nc, (cc // nc) % nc, cc // (nc * nc)
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                E = _child_embedding(k, (ox, oy, oz))
                fc = (2 * cx + ox) + nf * (2 * cy + oy) + nf * nf * (2 * cz + oz)
                r, c, d = sipg._coo_block(fc * N3, cc * N3, E)
                R.append(r)
                C.append(c)
                D.append(d)
    P = sp.coo_matrix((np.concatenate(D), (np.concatenate(R), np.concatenate(C))),
                      shape=(nf ** 3 * N3, nc ** 3 * N3)).tocsr()
    P.eliminate_zeros()
    return P


# ---------------------------------------------------------------------------
# Vertex patches
# ---------------------------------------------------------------------------

def vertex_patches(n):
    """Interior vertices (vx, vy, vz) in {1..n-1}^3 with their colour
    (vx mod 2) + 2 (vy mod 2) + 4 (vz mod 2)."""
    out = []
    for vz in range(1, n):
        for vy in range(1, n):
            for vx in range(1, n):
                out.append(((vx, vy, vz), (vx % 2) + 2 * (vy % 2) + 4 * (vz % 2)))
    return out


def patch_dofs(n, k, v):
    """Global DoF indices of the 8 cells around vertex v, cells ordered
    (dz, dy, dx) lexicographic, then the local index."""
    N3 = (k + 1) ** 3
    idx = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c = (v[0] - 1 + dx) + n * (v[1] - 1 + dy) + n * n * (v[2] - 1 + dz)
                idx.append(np.arange(c * N3, (c + 1) * N3))
    return np.concatenate(idx)


def patch_type(n, v):
    """Boundary configuration of a patch per direction: whether its lower
    cell touches x_d = 0 and whether its upper cell touches x_d = 1."""
    return tuple((v[d] == 1, v[d] == n - 1) for d in range(3))


class Level:
    def __init__(self, n, k, penalty_scale=1.0):
        self.n = n
        self.k = k
        self.A = sipg.assemble(n, k, penalty_scale=penalty_scale)
        self.patches = vertex_patches(n)
        self._chol = {}

    def patch_factor(self, v):
        """Cholesky factor of A_PP.  A_PP depends only on the patch type
        (translation invariance on a uniform mesh), so it is cached per
        type; tests check the cached factor against a direct extraction."""
        t = patch_type(self.n, v)
        if t not in self._chol:
            idx = patch_dofs(self.n, self.k, v)
            App = self.A[idx][:, idx].toarray()
            self._chol[t] = sla.cho_factor(App, lower=True)
        return self._chol[t]


def smooth(level, x, b, sweeps):
    """Multiplicative vertex-patch sweeps (reading in the module docstring)."""
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(sweeps):
        for colour in range(8):
            r = b - level.A @ x
            for v, c in level.patches:
                if c != colour:
                    continue
                idx = patch_dofs(level.n, level.k, v)
                x[idx] += sla.cho_solve(level.patch_factor(v), r[idx])
    return x


def smooth_additive(level, x, b, sweeps, damping=0.125):
    """Additive vertex-patch sweeps: x += omega sum_P R_P^T A_PP^{-1} R_P (b - A x)."""
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(sweeps):
        r = b - level.A @ x
        c = np.zeros_like(x)
        for v, _colour in level.patches:
            idx = patch_dofs(level.n, level.k, v)
            c[idx] += sla.cho_solve(level.patch_factor(v), r[idx])
        x = x + damping * c
    return x


class Hierarchy:
    """Levels 0 (coarsest, n0 cells per direction) .. L-1 (finest, n)."""

    def __init__(self, n, k, n_levels=None, coarsest=None, smoother="multiplicative",
                 damping=0.125, penalty_scale=1.0):
        if coarsest is None:
            # halve while even and above 3: 2 for n = 2^L, 3 for n = 3 * 2^L
            m = n
            while m % 2 == 0 and m > 3:
                m //= 2
            coarsest = m
        ns = [n]
        while ns[-1] > coarsest:
            if ns[-1] % 2:
                raise ValueError("mesh size not reachable by halving")
            ns.append(ns[-1] // 2)
        ns = ns[::-1]
        if n_levels is not None:
            ns = ns[len(ns) - n_levels:]
        self.k = k
        self.smoother = smoother
        self.damping = damping
        self.levels = [Level(m, k, penalty_scale) for m in ns]
        self.P = [None] + [prolongation(ns[i - 1], k) for i in range(1, len(ns))]
        self.coarse = spla.splu(self.levels[0].A.tocsc())
        self.nu_pre = 2
        self.nu_post = 2

    def vcycle(self, l, x, b):
        """Alg. v_cycle on level l."""
        if l == 0:
            return self.coarse.solve(b)
        lev = self.levels[l]
        x = self.smooth(lev, x, b, self.nu_pre)
        r = b - lev.A @ x
        rc = self.P[l].T @ r
        ec = self.vcycle(l - 1, np.zeros(rc.shape), rc)
        x = x + self.P[l] @ ec
        return self.smooth(lev, x, b, self.nu_post)

    def smooth(self, lev, x, b, sweeps):
        if self.smoother == "additive":
            return smooth_additive(lev, x, b, sweeps, self.damping)
        return smooth(lev, x, b, sweeps)

    def precondition(self, v):
        """z = V-cycle on the finest level with zero initial guess."""
        L = len(self.levels) - 1
        return self.vcycle(L, np.zeros(v.shape), v)
