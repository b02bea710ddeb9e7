"""Pins of the oracle's SIPG operator (Sec. 2, eq. bilinear_form; Sec. 2.1,
eq. tensorproduct_3d) and its right-hand side / L2 error (Sec. 7.2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import rhs, sipg
from paper_2407_09621_amd import inputs


def _interp(fun, n, k):
    P = sipg.node_coordinates(n, k)
    return fun(P[:, 0], P[:, 1], P[:, 2])


@pytest.mark.parametrize("k,n", [(1, 1), (1, 3), (2, 2), (3, 2), (4, 2), (2, 4)])
def test_symmetric_positive_definite(k, n):
    A = sipg.assemble(n, k).toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    if A.shape[0] <= 2000:
        assert np.linalg.eigvalsh(A).min() > 0
    np.linalg.cholesky(A)


@pytest.mark.parametrize("k,n", [(1, 3), (2, 2), (3, 3), (5, 2), (7, 1)])
def test_constants_annihilated_without_boundary_faces(k, n):
    A = sipg.assemble(n, k, boundary_terms=False)
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() <= 1e-13 * abs(A).max()


@pytest.mark.parametrize("k,n,s", [(1, 1, 1.0), (1, 4, 1.0), (2, 3, 1.0), (3, 2, 1.0),
                                   (4, 2, 1.0), (2, 3, 2.5), (3, 2, 7.0)])
def test_energy_closed_forms(k, n, s):
    """Exact values of the form for globally smooth functions (no interior
    jumps), gamma = s 2k(k+1) n (s the penalty scale):  a(1,1) = 6 gamma,
    a(x,x) = 7 gamma/3 - 1, a(x,y) = 3 gamma/2 (only boundary faces carry
    jumps: int_dOmega 1 = 6, int_dOmega x^2 = 7/3, int x dn x = 1,
    int_dOmega x y = 3/2, int y dn x + x dn y = 3/2 - 3/2 = 0 ... computed
    from the six faces of the unit cube)."""
    A = sipg.assemble(n, k, penalty_scale=s)
    g = s * 2 * k * (k + 1) * n
    one = np.ones(A.shape[0])
    X = _interp(lambda x, y, z: x, n, k)
    Y = _interp(lambda x, y, z: y, n, k)
    assert abs(one @ (A @ one) - 6 * g) < 1e-10 * g
    assert abs(X @ (A @ X) - (7 * g / 3 - 1)) < 1e-10 * g
    assert abs(Y @ (A @ X) - 1.5 * g) < 1e-10 * g


@pytest.mark.parametrize("k,n,s", [(1, 2, 1.0), (2, 3, 1.0), (3, 3, 1.0), (4, 2, 1.0),
                                   (5, 2, 1.0), (7, 2, 1.0), (3, 3, 3.0)])
def test_quadrature_assembly_equals_kronecker_sum(k, n, s):
    A = sipg.assemble(n, k, penalty_scale=s)
    u = inputs.uniform_vector(A.shape[0], seed=100 + k)
    v = A @ u
    w = sipg.kron_apply(u, n, k, penalty_scale=s)
    assert np.linalg.norm(v - w) <= 1e-13 * np.linalg.norm(v)
    if s == 1.0:
        rows = np.random.default_rng(k).choice(A.shape[0], 40, replace=False)
        np.testing.assert_allclose(sipg.apply_rows(u, n, k, rows), v[rows],
                                   rtol=0, atol=1e-12 * np.abs(v).max())


@pytest.mark.parametrize("k", [2, 3])
def test_q2_solution_reproduced_exactly(k):
    """u = x(1-x)y(1-y)z(1-z) lies in V_h for k >= 2 and SIPG is consistent,
    so the discrete solution equals its nodal interpolant."""
    n = 3
    A = sipg.assemble(n, k)
    b = rhs.rhs(rhs.BubbleQ2, n, k)
    x = spla.spsolve(A.tocsc(), b)
    assert np.abs(x - rhs.interpolate(rhs.BubbleQ2, n, k)).max() < 1e-13
    assert rhs.l2_error(rhs.BubbleQ2, x, n, k) < 1e-14


@pytest.mark.parametrize("k,ns", [(1, (2, 4, 8)), (2, (2, 4, 8)), (3, (2, 4, 6))])
def test_l2_convergence_order(k, ns):
    errs = []
    for n in ns:
        A = sipg.assemble(n, k)
        b = rhs.rhs(rhs.single_sine(), n, k)
        x = spla.spsolve(A.tocsc(), b)
        errs.append(rhs.l2_error(rhs.single_sine(), x, n, k))
    rate = np.log(errs[-2] / errs[-1]) / np.log(ns[-1] / ns[-2])
    assert abs(rate - (k + 1)) < 0.35, (errs, rate)


@pytest.mark.parametrize("k,n,tol", [(1, 2, 5e-4), (3, 2, 1e-6), (5, 2, 1e-9)])
def test_l2_error_absolute_scale(k, n, tol):
    """||u - 0||_L2 of u = sin(pi x) sin(pi y) sin(pi z) is sqrt(1/8) (each
    factor has mean square 1/2), and of two orthogonal modes
    a1 s(1,1,1) + a2 s(2,1,3) it is sqrt((a1^2 + a2^2) / 8).  The (k+3)-point
    rule is not exact for sines; the bound is its quadrature error, which
    falls with k (the symmetric single mode is integrated to rounding)."""
    zero = np.zeros(sipg.n_dofs(n, k))
    assert abs(rhs.l2_error(rhs.single_sine(), zero, n, k) - np.sqrt(1 / 8)) < 1e-12
    two = rhs.SineModes([0.7, -1.3], [(1, 1, 1), (2, 1, 3)])
    assert abs(rhs.l2_error(two, zero, n, k) - np.sqrt((0.49 + 1.69) / 8)) < tol


def test_rhs_and_l2_of_polynomials():
    n, k = 2, 3
    # interpolant of a Q_k polynomial has zero L2 error
    class Poly:
        u = staticmethod(lambda x, y, z: x ** 3 * y - 2 * z ** 2 * x + 1)
        f = staticmethod(lambda x, y, z: 0 * x + 1.0)
    assert rhs.l2_error(Poly, rhs.interpolate(Poly, n, k), n, k) < 1e-14
    # f = 1: sum of b_I is the volume, b_I is the integral of phi_I
    b = rhs.rhs(Poly, n, k)
    assert abs(b.sum() - 1.0) < 1e-14
    # sine: the total load is int f = 3 pi^2 (2/pi)^3 up to quadrature error
    b = rhs.rhs(rhs.single_sine(), 8, 3)
    assert abs(b.sum() - 3 * np.pi ** 2 * (2 / np.pi) ** 3) < 1e-6


def test_cell_blocked_tensor_permutation_roundtrip():
    n, k = 3, 2
    u = inputs.uniform_vector(sipg.n_dofs(n, k), 5)
    assert np.array_equal(sipg.from_tensor(sipg.to_tensor(u, n, k), n, k), u)
    # GLL node coordinates are monotone along the global tensor axes
    P = sipg.node_coordinates(n, k)
    X = sipg.to_tensor(P[:, 0], n, k)
    assert np.all(np.diff(X, axis=2) >= 0) and np.all(np.diff(X, axis=1) == 0)


@pytest.mark.parametrize("n,k,pen", [(2, 1, 1.0), (3, 2, 1.0), (3, 3, 2.5), (4, 1, 1.0), (2, 4, 1.0)])
def test_patchwise_apply_equals_assembled(n, k, pen):
    """The paper's patch-wise evaluation (Sec. 2.1, Fig. patch_int): the
    sum over all interior-vertex patches of each patch's own Kronecker sum
    of window matrices is the quadrature-assembled SIPG operator (interior,
    boundary and corner patches; a scaled penalty)."""
    u = np.random.default_rng(10 * n + k).uniform(-1, 1, sipg.n_dofs(n, k))
    ref = sipg.assemble(n, k, penalty_scale=pen) @ u
    v = sipg.patchwise_apply(u, n, k, penalty_scale=pen)
    assert np.linalg.norm(v - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k", [(2, 2), (5, 3)])
def test_windows_sum_to_the_line_matrices(n, k):
    """Every window carries its interior face once and each cell's mass and
    stiffness with weights that add up to 1 over the windows containing the
    cell: the windows summed along a line give the 1D matrices.  A window
    alone is not the principal 2N x 2N block of the line (the cell integrals
    are split), except for n = 2."""
    N = k + 1
    M, L = sipg.global_1d(n, k)
    Ms, Ls = np.zeros_like(M), np.zeros_like(L)
    for w in range(1, n):
        Mw, Lw = sipg.patch_1d(n, k, w)
        sl = slice((w - 1) * N, (w + 1) * N)
        Ms[sl, sl] += Mw
        Ls[sl, sl] += Lw
    np.testing.assert_allclose(Ms, M, atol=1e-14 * np.abs(M).max())
    np.testing.assert_allclose(Ls, L, atol=1e-12 * np.abs(L).max())
    Mw, Lw = sipg.patch_1d(n, k, 1)
    principal = np.allclose(Lw, L[:2 * N, :2 * N])
    assert principal == (n == 2)
    with pytest.raises(ValueError):
        sipg.patch_1d(n, k, 0)
