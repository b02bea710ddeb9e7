"""1D reference data on [0, 1] (Sec. 2 and Sec. 2.1 of the paper).

The shape functions are Lagrange polynomials of degree k on the N = k + 1
Gauss-Lobatto (GLL) points (Sec. 2).  Local 1D matrices are integrated with
the N-point Gauss-Legendre rule, which is exact for the mass matrix (degree
2k) and the stiffness matrix (degree 2k - 2).  Reading: the paper's remark
that quadrature points "align" with the nodes could suggest GLL collocation
(a lumped mass matrix); we integrate exactly instead, because the paper's
sum factorization multiplies with dense 1D mass matrices (Sec. 2.1,
eq. tensorproduct_3d and Appendix A).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k):
    """GLL points of degree k on [0, 1]: the endpoints plus the roots of
    P_k' (Legendre), mapped from [-1, 1].  Sec. 2 (Gauss-Lobatto points)."""
    if k < 1:
        raise ValueError("k >= 1 required")
    c = np.zeros(k + 1)
    c[k] = 1.0
    inner = np.sort(npleg.Legendre(c).deriv().roots().real) if k > 1 else np.array([])
    t = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (t + 1.0)


def gauss_rule(n):
    """n-point Gauss-Legendre rule on [0, 1] (points, weights)."""
    t, w = npleg.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """phi_a(x_q) for every node a and point x_q: array [len(x), N].

    Plain product formula phi_a(x) = prod_{b != a} (x - x_b) / (x_a - x_b)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    N = len(nodes)
    out = np.ones((len(x), N))
    for a in range(N):
        for b in range(N):
            if b != a:
                out[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
    return out


def lagrange_derivs(nodes, x):
    """phi_a'(x_q): array [len(x), N].

    Product rule: phi_a'(x) = sum_{m != a} 1/(x_a - x_m)
    * prod_{b != a, m} (x - x_b)/(x_a - x_b)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    N = len(nodes)
    out = np.zeros((len(x), N))
    for a in range(N):
        for m in range(N):
            if m == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[m]))
            for b in range(N):
                if b != a and b != m:
                    term = term * (x - nodes[b]) / (nodes[a] - nodes[b])
            out[:, a] += term
    return out


def mass_stiffness(k):
    """h-free 1D mass Mhat_ab = int_0^1 phi_a phi_b and stiffness
    Khat_ab = int_0^1 phi_a' phi_b' (exact N-point Gauss)."""
    nodes = gll_nodes(k)
    xq, wq = gauss_rule(k + 1)
    V = lagrange_values(nodes, xq)
    D = lagrange_derivs(nodes, xq)
    M = V.T @ (wq[:, None] * V)
    K = D.T @ (wq[:, None] * D)
    return M, K


def end_vectors(k):
    """Trace vectors of the 1D basis at the two ends of [0, 1]:
    s0 = phi(0), s1 = phi(1), d0 = phi'(0), d1 = phi'(1).  These are the
    1 x N face evaluators S_f and D_f of Sec. 2.1."""
    nodes = gll_nodes(k)
    s = lagrange_values(nodes, [0.0, 1.0])
    d = lagrange_derivs(nodes, [0.0, 1.0])
    return s[0], s[1], d[0], d[1]
