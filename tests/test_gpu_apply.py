"""GPU parity of the FP64 operator apply (Sec. 2.1, eq. tensorproduct_3d)
against the oracle: element-wise on small meshes that span several
workgroups with a ragged tail, and at the full benchmark sizes (64^3 cells
of degree 3, 40^3 of degree 5, 32^3 of degree 7) against the oracle's
Kronecker apply plus sampled rows from the quadrature matrices.
Tolerance: 1e-12 relative in l2 (FP64; the two sides differ only in the
rounding order of the same sums)."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, to_cpu, to_gpu
from oracle import sipg
from paper_2407_09621_amd import inputs

pytestmark = pytest.mark.gpu

SMALL = [(k, n) for k in range(1, 8) for n in (1, 2, 3, 5)]


@pytest.mark.parametrize("k,n", SMALL)
def test_apply_matches_assembled_matrix(k, n):
    from paper_2407_09621_amd import Problem
    if k >= 6 and n == 5:
        n = 4
    announce("apply", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=1000 + 10 * k + n)
    v = to_cpu(P.apply(to_gpu(u)))
    ref = sipg.assemble(n, k) @ u
    assert rel_l2(v, ref) < 1e-12
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("k,n", [(2, 3), (3, 5), (4, 6), (5, 6), (6, 4), (7, 3)])
def test_residual_matches(k, n):
    from paper_2407_09621_amd import Problem
    announce("residual", k, n)
    P = Problem(k, n, n_levels=1)
    x = inputs.uniform_vector(P.n_dofs(), seed=2)
    b = inputs.uniform_vector(P.n_dofs(), seed=3)
    r = to_cpu(P.residual(to_gpu(b), to_gpu(x)))
    ref = b - sipg.assemble(n, k) @ x
    assert rel_l2(r, ref) < 1e-12


def test_apply_edge_cases():
    import torch
    from paper_2407_09621_amd import Problem, SipgError
    announce("apply edge cases")
    P = Problem(2, 2, n_levels=1)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    assert torch.count_nonzero(P.apply(u)) == 0
    with pytest.raises(SipgError):
        P.apply(u, u)  # aliasing is rejected
    with pytest.raises(TypeError):
        P.apply(u.float())
    # constants: A 1 = boundary terms only; interior rows vanish without them
    one = torch.ones_like(u)
    v = to_cpu(P.apply(one))
    ref = sipg.assemble(2, 2) @ np.ones(P.n_dofs())
    assert rel_l2(v, ref) < 1e-13


@pytest.mark.parametrize("k,n", [(3, 64), (5, 40), (7, 32)])
def test_apply_full_size(k, n):
    """The benchmark configurations, same launch as the benchmark."""
    from paper_2407_09621_amd import Problem
    announce("apply full size", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=2 + k)
    v = to_cpu(P.apply(to_gpu(u)))
    ref = sipg.kron_apply(u, n, k)
    assert rel_l2(v, ref) < 1e-12
    rows = np.random.default_rng(k).choice(P.n_dofs(), 64, replace=False)
    # include the first and last cells (boundary faces) explicitly
    rows = np.concatenate([rows, [0, P.n_dofs() - 1]])
    samp = sipg.apply_rows(u, n, k, rows)
    np.testing.assert_allclose(v[rows], samp, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("k,n", [(5, 64), (4, 64)])
def test_apply_vectors_ending_on_a_page_boundary(k, n):
    """Regression: the idle lanes of the last workgroup tile (64^3 cells do
    not fill whole 7- or 10-cell tiles) must load inside one cell.  At k = 5
    the FP64 vector is exactly 216 x 2 MiB, so a load past its end leaves
    the allocation.  Apply and residual form, sampled rows including the
    last cells, against the oracle's row formula."""
    import torch
    from paper_2407_09621_amd import Problem
    announce("apply ending on a page boundary", k, n)
    P = Problem(k, n, n_levels=1)
    nd = P.n_dofs()
    u = inputs.uniform_vector(nd, seed=7 + k)
    ug = to_gpu(u)
    v = P.apply(ug)
    b = torch.ones_like(ug)
    r = P.residual(b, ug)
    torch.cuda.synchronize()
    N3 = (k + 1) ** 3
    rng = np.random.default_rng(k)
    rows = np.concatenate([rng.choice(nd, 48, replace=False), np.arange(nd - 2 * N3, nd, 37)])
    samp = sipg.apply_rows(u, n, k, rows)
    scale = np.abs(samp).max()
    np.testing.assert_allclose(to_cpu(v)[rows], samp, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(to_cpu(r)[rows], 1.0 - samp, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("k,n", [(3, 3), (3, 9), (7, 2), (7, 5), (5, 4), (1, 6)])
def test_apply_units_match_assembled_matrix(k, n):
    """sipg_apply_units: the FP64 vector-unit kernel (every degree) and the
    matrix-core kernel (degrees 3 and 7) give the oracle's A u; 9 cells per
    row at k = 3 leave a ragged tile of the 8-cell matrix-core rows."""
    from paper_2407_09621_amd import Problem, SipgError
    announce("apply units", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=3000 + 10 * k + n)
    ref = sipg.assemble(n, k) @ u
    units = ["vector", "matrix"] if k in (3, 7) else ["vector"]
    for un in units:
        v = to_cpu(P.apply(to_gpu(u), units=un))
        assert rel_l2(v, ref) < 1e-12, un
        np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    if k not in (3, 7):
        with pytest.raises(SipgError, match="k = 3 and 7"):
            P.apply(to_gpu(u), units="matrix")


@pytest.mark.parametrize("k,n", [(3, 64), (7, 32)])
def test_apply_vector_units_full_size(k, n):
    """The vector-unit kernel at the benchmark sizes of the two matrix-core
    degrees (the launch the benchmark's vector-unit rows time)."""
    from paper_2407_09621_amd import Problem
    announce("apply vector units full size", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=2 + k)
    v = to_cpu(P.apply(to_gpu(u), units="vector"))
    assert rel_l2(v, sipg.kron_apply(u, n, k)) < 1e-12


@pytest.mark.parametrize("k,n", [(1, 2), (2, 3), (3, 5), (4, 4), (5, 3), (6, 2), (7, 3)])
def test_apply_patchwise_matches_assembled_matrix(k, n):
    """sipg_apply_patchwise (the paper's patch-wise evaluation, every colour
    of vertex patches, boundary and corner window types) gives the oracle's
    A u; odd n leaves colours with fewer patches per direction."""
    from paper_2407_09621_amd import Problem, SipgError
    announce("apply patchwise", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=5000 + 10 * k + n)
    v = to_cpu(P.apply_patchwise(to_gpu(u)))
    ref = sipg.assemble(n, k) @ u
    assert rel_l2(v, ref) < 1e-12
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    P1 = Problem(k, 1, n_levels=1)
    with pytest.raises(SipgError, match="n >= 2"):
        P1.apply_patchwise(to_gpu(inputs.uniform_vector(P1.n_dofs(), 1)))


@pytest.mark.parametrize("k,n", [(3, 64), (7, 32)])
def test_apply_patchwise_full_size(k, n):
    """The patch-wise evaluation at the benchmark sizes against the oracle's
    Kronecker apply (the launch the benchmark's patch-wise rows time)."""
    from paper_2407_09621_amd import Problem
    announce("apply patchwise full size", k, n)
    P = Problem(k, n, n_levels=1)
    u = inputs.uniform_vector(P.n_dofs(), seed=2 + k)
    v = to_cpu(P.apply_patchwise(to_gpu(u)))
    assert rel_l2(v, sipg.kron_apply(u, n, k)) < 1e-12
