"""Pins of the oracle's SIPG operator on trilinear hexahedra (Sec. 2 with the
mapped cell integral of Sec. 2.1, A^K = G_phi^T W G_phi with per-point
Jacobians).  Each pin rests on something other than the mapped assembly
itself: the Cartesian oracle (3D quadrature and the Kronecker sum), the
invariance of the Laplacian under rigid motions, and the consistency of SIPG
for harmonic polynomials that the mapped space reproduces exactly."""
import numpy as np
import pytest

from oracle import mapped, sipg
from paper_2407_09621_amd import inputs


def _interior_rows(n, k):
    N3 = (k + 1) ** 3
    c = np.arange(n ** 3)
    cx, cy, cz = c % n, (c // n) % n, c // (n * n)
    inner = (cx > 0) & (cx < n - 1) & (cy > 0) & (cy < n - 1) & (cz > 0) & (cz < n - 1)
    return np.concatenate([np.arange(i * N3, (i + 1) * N3) for i in c[inner]])


@pytest.mark.parametrize("k,n", [(1, 3), (2, 3), (3, 2), (5, 2)])
def test_identity_mesh_is_the_cartesian_operator(k, n):
    A = mapped.assemble_mapped(n, k, inputs.mesh_vertices(n))
    B = sipg.assemble(n, k)
    assert abs(A - B).max() <= 1e-13 * abs(B).max()


@pytest.mark.parametrize("k,n,s", [(1, 3, 1.7), (2, 3, 0.6), (3, 2, 2.5)])
def test_rigid_motion_and_scaling(k, n, s):
    """The Laplacian is invariant under rotations and translations; under
    x -> s x every term of the form scales by s in 3D (grad . grad dx by
    s^{-2} s^3, the penalty 1/h times the face measure by s^{-1} s^2, the
    normal-derivative terms likewise)."""
    V = inputs.mesh_vertices(n, affine=s * inputs.rotation(7 + k), shift=[0.3, -1.0, 2.0])
    A = mapped.assemble_mapped(n, k, V)
    B = sipg.assemble(n, k)
    assert abs(A - s * B).max() <= 1e-13 * s * abs(B).max()


@pytest.mark.parametrize("k,n", [(1, 3), (2, 2), (3, 2)])
def test_rotated_box_cells_match_the_anisotropic_kronecker_sum(k, n):
    """Cells of size (a/n, b/n, c/n), rotated: the operator is the Kronecker
    sum with per-direction 1D matrices M_d = s_d M, L_d = L / s_d of the
    Cartesian 1D data (penalty 2k(k+1) n / s_d on faces normal to d, which is
    the volume-over-area reading of h).  Catches a transposed Jacobian or a
    mixed-up normal direction, which an isotropic scaling hides."""
    s = np.array([0.7, 1.3, 2.1])
    V = inputs.mesh_vertices(n, affine=inputs.rotation(3) @ np.diag(s))
    A = mapped.assemble_mapped(n, k, V)
    M, L = sipg.global_1d(n, k)
    al = sipg._along
    u = inputs.uniform_vector(sipg.n_dofs(n, k), 11)
    U = sipg.to_tensor(u, n, k)
    W = al(al(al(U, L / s[0], 2), s[1] * M, 1), s[2] * M, 0)
    W += al(al(al(U, s[0] * M, 2), L / s[1], 1), s[2] * M, 0)
    W += al(al(al(U, s[0] * M, 2), s[1] * M, 1), L / s[2], 0)
    ref = sipg.from_tensor(W, n, k)
    got = A @ u
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def _jittered(n, seed, amp=0.2):
    V = inputs.mesh_vertices(n, "jitter", amp, seed=seed)
    return V


@pytest.mark.parametrize("k", [1, 2, 3])
def test_linear_functions_consistency_on_trilinear_cells(k):
    """A linear u = a.x + c composed with a trilinear map is trilinear in the
    reference coordinates, so the space holds it exactly; it is harmonic with
    no jumps, and the N-point Gauss rules integrate every term exactly (the
    cofactors of J are of degree <= 2 per variable).  Integration by parts
    then makes (A u)_i vanish on every cell without a boundary face."""
    n = 4
    V = _jittered(n, 5)
    assert mapped.min_jacobian(n, k, V) > 0
    A = mapped.assemble_mapped(n, k, V)
    x = mapped.node_positions(n, k, V)
    u = x @ np.array([0.3, -1.2, 0.7]) + 0.4
    r = A @ u
    rows = _interior_rows(n, k)
    scale = abs(A).max() * np.abs(u).max()
    assert np.abs(r[rows]).max() <= 1e-13 * scale
    assert np.abs(r).max() >= 1e-3 * scale   # boundary rows carry the Nitsche terms


@pytest.mark.parametrize("k", [2, 3])
def test_quadratic_harmonic_consistency_on_trilinear_cells(k):
    """u = x^2 - y^2 + xz / 2 is harmonic and quadratic; on trilinear cells it
    is of degree 2 per reference variable (in the space for k >= 2) and the
    integrands stay within the Gauss rules' exactness for k >= 2."""
    n = 4
    V = _jittered(n, 9)
    A = mapped.assemble_mapped(n, k, V)
    x = mapped.node_positions(n, k, V)
    u = x[:, 0] ** 2 - x[:, 1] ** 2 + 0.5 * x[:, 0] * x[:, 2]
    r = A @ u
    assert np.abs(r[_interior_rows(n, k)]).max() <= 1e-13 * abs(A).max() * np.abs(u).max()


@pytest.mark.parametrize("k,n,kind", [(1, 3, "jitter"), (2, 3, "smooth"), (3, 2, "jitter")])
def test_symmetric_positive_definite_and_constants(k, n, kind):
    V = inputs.mesh_vertices(n, kind, 0.2 if kind == "jitter" else 0.08, seed=2)
    A = mapped.assemble_mapped(n, k, V)
    D = A.toarray()
    assert np.abs(D - D.T).max() <= 1e-14 * np.abs(D).max()
    assert np.linalg.eigvalsh(D).min() > 0
    A0 = mapped.assemble_mapped(n, k, V, boundary_terms=False)
    assert np.abs(A0 @ np.ones(A0.shape[0])).max() <= 1e-13 * abs(A0).max()


def test_sampled_cells_match_the_assembled_matrix():
    n, k = 4, 2
    V = _jittered(n, 4)
    A = mapped.assemble_mapped(n, k, V)
    u = inputs.uniform_vector(A.shape[0], 1)
    v = A @ u
    cells = [0, 5, 21, 42, 63]
    got = mapped.apply_cells_mapped(u, n, k, V, cells)
    N3 = (k + 1) ** 3
    for row, c in zip(got, cells):
        ref = v[c * N3:(c + 1) * N3]
        assert np.abs(row - ref).max() <= 1e-13 * np.abs(v).max()


def test_volume_and_area_of_a_sheared_cell():
    """Closed forms for an affine cell: |K| = |det B|, face areas |B e_i x B e_j|."""
    B = np.array([[1.0, 0.3, 0.1], [0.0, 0.8, -0.2], [0.1, 0.0, 1.4]])
    X = np.array([B @ np.array([a, b, c], float) for c in (0, 1) for b in (0, 1) for a in (0, 1)])
    assert abs(mapped.cell_volume(2, X) - abs(np.linalg.det(B))) <= 1e-14
    for d in range(3):
        t = [a for a in range(3) if a != d]
        ref = np.linalg.norm(np.cross(B[:, t[0]], B[:, t[1]]))
        for side in (0, 1):
            assert abs(mapped.face_area(2, X, d, side) - ref) <= 1e-14


def test_identity_mesh_rhs_and_l2_match_the_cartesian_oracle():
    from oracle import rhs
    n, k = 3, 2
    V = inputs.mesh_vertices(n)
    prob = rhs.SineModes(*inputs.sine_modes(3))
    b = mapped.rhs_mapped(prob, n, k, V)
    assert np.abs(b - rhs.rhs(prob, n, k)).max() <= 1e-14 * np.abs(b).max()
    u = inputs.uniform_vector(sipg.n_dofs(n, k), 5)
    assert abs(mapped.l2_error_mapped(prob, u, n, k, V) - rhs.l2_error(prob, u, n, k)) <= 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_solution_on_deformed_meshes_converges_at_rate_k_plus_1(k):
    """The sine solution vanishes on the cube's boundary, which the smooth
    interior deformation keeps in place: the SIPG solution on the trilinear
    meshes of n = 2, 4, 8 cells converges in L2 at the rate k + 1 of the
    method, which a wrong face term, penalty or right-hand side would spoil."""
    import scipy.sparse.linalg as spla
    from oracle import rhs
    prob = rhs.single_sine()
    errs = []
    for n in (2, 4, 8):
        V = inputs.mesh_vertices(n, "smooth", 0.08, seed=1)
        A = mapped.assemble_mapped(n, k, V)
        u = spla.spsolve(A.tocsc(), mapped.rhs_mapped(prob, n, k, V))
        errs.append(mapped.l2_error_mapped(prob, u, n, k, V))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > k + 1 - 0.3, (errs, rates)


def test_mapped_vcycle_on_the_identity_mesh_is_the_cartesian_vcycle():
    """With identity vertices the mapped V-cycle (mapped residuals, Cartesian
    patch and coarse inverses) is the Cartesian V-cycle of the oracle."""
    from oracle import multigrid
    n, k = 4, 2
    H = multigrid.Hierarchy(n, k)
    M = mapped.MappedHierarchy(n, k, inputs.mesh_vertices(n))
    b = inputs.uniform_vector(sipg.n_dofs(n, k), 3)
    L = len(H.levels) - 1
    x0 = np.zeros_like(b)
    ref = H.vcycle(L, x0, b)
    got = M.vcycle(L, x0, b)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mapped_vcycle_contracts_on_a_deformed_mesh():
    """The Cartesian inverses stay good approximate inverses on a mildly
    deformed mesh: the V-cycle iteration's error contracts."""
    import scipy.sparse.linalg as spla
    n, k = 4, 2
    V = inputs.mesh_vertices(n, "smooth", 0.08, seed=1)
    M = mapped.MappedHierarchy(n, k, V)
    A = M.A[-1]
    b = inputs.uniform_vector(A.shape[0], 4)
    xs = spla.spsolve(A.tocsc(), b)
    x = np.zeros_like(b)
    errs = []
    for _ in range(4):
        x = x + M.vcycle(len(M.A) - 1, np.zeros_like(b), b - A @ x)
        errs.append(np.linalg.norm(x - xs))
    assert errs[-1] < 0.05 * errs[0] and all(errs[i + 1] < errs[i] for i in range(3))


def test_mapped_vcycle_diverges_on_a_strongly_jittered_mesh():
    """The limit of the Cartesian inverses (reading R20 of the design): on
    8^3 cells with interior vertices moved by up to 0.2 h the V-cycle with
    Cartesian patch and coarse inverses amplifies the error; recorded so the
    limitation stays visible."""
    import scipy.sparse.linalg as spla
    n, k = 8, 2
    V = inputs.mesh_vertices(n, "jitter", 0.2, seed=8)
    M = mapped.MappedHierarchy(n, k, V)
    A = M.A[-1]
    b = inputs.uniform_vector(A.shape[0], 14)
    xs = spla.spsolve(A.tocsc(), b)
    x = M.vcycle(len(M.A) - 1, np.zeros_like(b), b)
    assert np.linalg.norm(x - xs) > np.linalg.norm(xs)


def test_mapped_vcycle_contracts_on_a_moderately_jittered_mesh():
    """The other side of that limit: with interior vertices moved by up to
    0.1 h on the same 8^3 cells the Cartesian inverses still contract the
    error by more than 100 per cycle."""
    import scipy.sparse.linalg as spla
    n, k = 8, 2
    V = inputs.mesh_vertices(n, "jitter", 0.1, seed=8)
    M = mapped.MappedHierarchy(n, k, V)
    A = M.A[-1]
    b = inputs.uniform_vector(A.shape[0], 14)
    xs = spla.spsolve(A.tocsc(), b)
    x = np.zeros_like(b)
    errs = []
    for _ in range(2):
        x = x + M.vcycle(len(M.A) - 1, np.zeros_like(b), b - A @ x)
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert errs[0] < 1e-2 and errs[1] < 1e-2 * errs[0], errs
