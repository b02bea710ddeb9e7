"""Right-hand sides and L2 errors by tensor Gauss quadrature on every cell.

Sec. 7.2: Poisson problem with the manufactured solution
u = sin(pi x) sin(pi y) sin(pi z) on the unit cube (f = -Laplace u, g = 0).
We also use sums of sine modes u = sum_m a_m sin(p_m pi x) sin(q_m pi y)
sin(r_m pi z) with integer wavenumbers (so g = 0), and the Q2 polynomial
x(1-x) y(1-y) z(1-z) for the exact-reproduction pin.

b_I = int_K f phi_I with the (k+2)-point Gauss rule per direction;
||u - u_h||_L2 with the (k+3)-point rule per direction.
"""
import numpy as np

from . import basis1d


class SineModes:
    """u = sum_m a_m sin(p_m pi x) sin(q_m pi y) sin(r_m pi z)."""

    def __init__(self, amps, pqr):
        self.amps = np.asarray(amps, dtype=np.float64).reshape(-1)
        self.pqr = np.asarray(pqr, dtype=np.float64).reshape(-1, 3)

    def u(self, X, Y, Z):
        out = np.zeros(np.broadcast(X, Y, Z).shape)
        for a, (p, q, r) in zip(self.amps, self.pqr):
            out += a * np.sin(p * np.pi * X) * np.sin(q * np.pi * Y) * np.sin(r * np.pi * Z)
        return out

    def f(self, X, Y, Z):
        """-Laplace u."""
        out = np.zeros(np.broadcast(X, Y, Z).shape)
        for a, (p, q, r) in zip(self.amps, self.pqr):
            lam = np.pi ** 2 * (p * p + q * q + r * r)
            out += lam * a * np.sin(p * np.pi * X) * np.sin(q * np.pi * Y) * np.sin(r * np.pi * Z)
        return out


def single_sine():
    """The paper's manufactured solution sin(pi x) sin(pi y) sin(pi z)."""
    return SineModes([1.0], [[1, 1, 1]])


class BubbleQ2:
    """u = x(1-x) y(1-y) z(1-z) in Q2, zero on the boundary."""

    @staticmethod
    def u(X, Y, Z):
        return X * (1 - X) * Y * (1 - Y) * Z * (1 - Z)

    @staticmethod
    def f(X, Y, Z):
        a, b, c = X * (1 - X), Y * (1 - Y), Z * (1 - Z)
        return 2.0 * (b * c + a * c + a * b)


def _cell_quadrature(n, k, nq):
    """Physical quadrature points of all cells [ncell, Q] (x, y, z), weights
    [Q] (times h^3) and the basis table phi [Q, N^3]."""
    h = 1.0 / n
    N = k + 1
    xq, wq = basis1d.gauss_rule(nq)
    V = basis1d.lagrange_values(basis1d.gll_nodes(k), xq)      # [nq, N]
    qi = np.arange(nq ** 3)
    a, b, c = qi % nq, (qi // nq) % nq, qi // (nq * nq)
    W = wq[a] * wq[b] * wq[c] * h ** 3
    loc = np.arange(N ** 3)
    i, j, l = loc % N, (loc // N) % N, loc // (N * N)
    Phi = V[a][:, i] * V[b][:, j] * V[c][:, l]                  # [Q, N^3]
    cells = np.arange(n ** 3)
    cx, cy, cz = cells % n, (cells // n) % n, cells // (n * n)
    X = (cx[:, None] + xq[a][None, :]) * h
    Y = (cy[:, None] + xq[b][None, :]) * h
    Z = (cz[:, None] + xq[c][None, :]) * h
    return X, Y, Z, W, Phi


def rhs(problem, n, k):
    """b_I = int f phi_I, cell-blocked order."""
    X, Y, Z, W, Phi = _cell_quadrature(n, k, k + 2)
    F = problem.f(X, Y, Z) * W[None, :]
    return (F @ Phi).reshape(-1)


def l2_error(problem, uh, n, k):
    """||u - u_h||_L2(Omega)."""
    X, Y, Z, W, Phi = _cell_quadrature(n, k, k + 3)
    N3 = (k + 1) ** 3
    Uh = np.asarray(uh).reshape(n ** 3, N3) @ Phi.T
    E = problem.u(X, Y, Z) - Uh
    return float(np.sqrt(np.sum(E * E * W[None, :])))


def interpolate(problem, n, k):
    """Nodal interpolant: u at every DoF's GLL node."""
    from .sipg import node_coordinates
    P = node_coordinates(n, k)
    return problem.u(P[:, 0], P[:, 1], P[:, 2])
