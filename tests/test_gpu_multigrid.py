"""GPU parity of the multigrid pieces (Sec. 7.1, Alg. v_cycle) against the
oracle: fast-diagonalization patch corrections (exact local solves, so equal
to the oracle's dense Cholesky solves up to rounding), smoothing sweeps,
transfers, the exact coarse solve and whole V-cycles.  Tolerances are
relative l2 and derive from FP64 rounding of O(100)-term sums through a few
dozen dependent steps."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from gpu_util import announce, rel_l2, to_cpu, to_gpu
from oracle import multigrid, sipg
from paper_2407_09621_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n", [(1, 4), (2, 5), (3, 4), (3, 7), (3, 8), (5, 3), (7, 2), (2, 2)])
def test_patch_correction_matches_dense_solves(k, n):
    from paper_2407_09621_amd import Problem
    announce("patch", k, n)
    P = Problem(k, n, n_levels=1)
    lev = multigrid.Level(n, k)
    r = inputs.uniform_vector(P.n_dofs(), 20 + k)
    x0 = inputs.uniform_vector(P.n_dofs(), 30 + k)
    for colour in range(8):
        x = to_gpu(x0)
        P.patch_correct(colour, to_gpu(r), x)
        ref = x0.copy()
        for v, c in lev.patches:
            if c == colour:
                idx = multigrid.patch_dofs(n, k, v)
                ref[idx] += sla.cho_solve(lev.patch_factor(v), r[idx])
        assert rel_l2(to_cpu(x), ref) < 1e-12, colour


@pytest.mark.parametrize("k,n,sweeps", [(2, 4, 1), (3, 4, 2), (1, 6, 2), (4, 3, 1)])
def test_smoother_matches(k, n, sweeps):
    from paper_2407_09621_amd import Problem
    announce("smooth", k, n, sweeps)
    P = Problem(k, n, n_levels=1)
    lev = multigrid.Level(n, k)
    b = inputs.uniform_vector(P.n_dofs(), 40 + k)
    x0 = inputs.uniform_vector(P.n_dofs(), 50 + k)
    x = to_gpu(x0)
    P.smooth(x, to_gpu(b), sweeps)
    ref = multigrid.smooth(lev, x0, b, sweeps)
    assert rel_l2(to_cpu(x), ref) < 1e-11


@pytest.mark.parametrize("k,nc", [(1, 1), (2, 2), (3, 3), (7, 2), (4, 5)])
def test_transfers_match(k, nc):
    import torch
    from paper_2407_09621_amd import Problem
    announce("transfer", k, nc)
    P = Problem(k, 2 * nc, n_levels=2)
    Pm = multigrid.prolongation(nc, k)
    rf = inputs.uniform_vector(P.n_dofs(1), 60 + k)
    ec = inputs.uniform_vector(P.n_dofs(0), 61 + k)
    xf0 = inputs.uniform_vector(P.n_dofs(1), 62 + k)
    rc = to_cpu(P.restrict(to_gpu(rf), level=1))
    assert rel_l2(rc, Pm.T @ rf) < 1e-13
    xf = to_gpu(xf0)
    P.prolongate_add(to_gpu(ec), xf, level=1)
    assert rel_l2(to_cpu(xf), xf0 + Pm @ ec) < 1e-13


@pytest.mark.parametrize("k,n0", [(1, 1), (2, 2), (3, 2), (7, 2), (2, 3), (5, 3), (7, 3)])
def test_coarse_solve_exact(k, n0):
    from paper_2407_09621_amd import Problem
    announce("coarse", k, n0)
    P = Problem(k, n0, n_levels=1)
    A = sipg.assemble(n0, k)
    b = inputs.uniform_vector(P.n_dofs(0), 70 + k)
    x = to_cpu(P.coarse_solve(to_gpu(b)))
    ref = spla.spsolve(A.tocsc(), b)
    assert rel_l2(x, ref) < 1e-11
    assert np.linalg.norm(A @ x - b) < 1e-12 * np.linalg.norm(b) * 100


@pytest.mark.parametrize("k,n", [(2, 8), (3, 4), (1, 6), (5, 4)])
def test_vcycle_matches(k, n):
    from paper_2407_09621_amd import Problem
    announce("vcycle", k, n)
    P = Problem(k, n)
    H = multigrid.Hierarchy(n, k)
    assert P.num_levels == len(H.levels)
    b = inputs.uniform_vector(P.n_dofs(), 80 + k)
    x0 = inputs.uniform_vector(P.n_dofs(), 81 + k)
    x = to_gpu(x0)
    P.vcycle(x, to_gpu(b))
    ref = H.vcycle(len(H.levels) - 1, x0, b)
    assert rel_l2(to_cpu(x), ref) < 1e-10


@pytest.mark.parametrize("k,n", [(2, 5), (3, 4), (3, 5), (5, 3), (7, 2), (1, 3), (6, 4)])
def test_fused_and_separate_smoothers_match_oracle(k, n):
    """Both forms of the multiplicative smoother: the separate residual per
    colour (the default) and the fused colour step (new patch values = local
    solve of b_P minus the outside neighbours' face couplings, written to a
    second vector, uncovered layers copied), against the oracle's sweeps; odd and
    even n (different uncovered layers per colour), n = 2 (colours without
    patches), two sweeps."""
    from paper_2407_09621_amd import Problem
    announce("smooth fused/separate", k, n)
    lev = multigrid.Level(n, k)
    b = inputs.uniform_vector(sipg.n_dofs(n, k), 80 + k)
    x0 = inputs.uniform_vector(sipg.n_dofs(n, k), 90 + k)
    ref = multigrid.smooth(lev, x0, b, 2)
    for form in ("multiplicative", "multiplicative_fused"):
        P = Problem(k, n, n_levels=1, smoother=form)
        x = to_gpu(x0)
        P.smooth(x, to_gpu(b), 2)
        assert rel_l2(to_cpu(x), ref) < 1e-11, form


@pytest.mark.parametrize("k,n", [(2, 8), (3, 8), (5, 4)])
def test_fused_smoother_in_fp32_vcycle(k, n):
    """The FP32 V-cycle with the fused colour steps against the FP32 V-cycle
    with a separate residual per colour: both are FP32 roundings of the same
    exact cycle (bound 8 u32 relative to the FP64 V-cycle), so they differ by
    a few u32."""
    import torch
    from paper_2407_09621_amd import Problem
    announce("fp32 vcycle fused/separate", k, n)
    b = torch.from_numpy(inputs.uniform_vector(sipg.n_dofs(n, k), 11)).cuda()
    x64 = torch.zeros_like(b)
    Problem(k, n).vcycle(x64, b)
    for form in ("multiplicative", "multiplicative_fused"):
        x = torch.zeros_like(b)
        Problem(k, n, mg_precision="f32", smoother=form).vcycle(x, b)
        assert rel_l2(to_cpu(x), to_cpu(x64)) < 64 * 2.0 ** -24, form
