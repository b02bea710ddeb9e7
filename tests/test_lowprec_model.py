"""CPU pins of the reduced-precision model (tests/lowprec_model.py) and what
it shows about the low-precision V-cycle (Sec. 5.2, Alg. matmul, Sec. 7.1).

The model explains a GPU finding: with BF16 operands and no correction the
FGMRES iteration preconditioned by the V-cycle stalls at degrees 5 and 7,
while splitting only the constant matrix operand (the paper's option of
refining one of the two matrices) restores fast convergence.  The cause is
the rounded 1D operator itself: with 8 significand bits its cell blocks move
the lowest eigenvalue of the discrete Laplacian by many times its size.
The patch eigenvector transforms are not the cause (their rounding errors
stay at a few units of roundoff)."""
import numpy as np
import pytest
import scipy.linalg as sla

import lowprec_model as lm
from oracle import fgmres, rhs, sipg


def test_bf16_rounding_matches_torch_and_ties_go_to_even():
    import torch
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lm.round_bf16(x), ref)
    assert lm.round_bf16(1 + 2.0 ** -8) == 1.0                    # tie: even mantissa 0
    assert lm.round_bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6      # tie: up to the even one
    assert lm.round_bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_split_reconstructs_to_second_order(fmt):
    x = np.random.default_rng(2).uniform(-1, 1, 5000)
    hi, lo = lm.split(x, fmt)
    u = lm.UNIT[fmt]
    assert np.all(np.abs(hi - x) <= u * np.abs(x) * 1.0001)
    assert np.all(np.abs(hi + lo / lm.SPLIT[fmt] - x) <= 2 * u * u * np.abs(x) + 1e-300)


@pytest.mark.parametrize("k", [2, 5, 7])
@pytest.mark.parametrize("fmt,ec", [("f16", 0), ("bf16", 0), ("bf16", 2), ("bf16", 1)])
def test_patch_transforms_stay_at_unit_roundoff(k, fmt, ec):
    """The fast-diagonalization patch solve in model arithmetic against the
    dense solve: a few units of roundoff, not amplified by the patch
    condition number (up to ~5e3 at k = 7)."""
    n = 4
    lev = lm.Level(n, k, fmt, ec)
    exact = lm.Level(n, k, "f32", 0)
    nd = sipg.n_dofs(n, k)
    r = lm.round_f32(np.random.default_rng(k).uniform(-1, 1, nd))
    from oracle import multigrid
    olev = multigrid.Level(n, k) if k < 7 else None
    z = lev.patch_correct(0, r, np.zeros(nd))
    ref = exact.patch_correct(0, r, np.zeros(nd))
    if olev is not None:   # the FP32 model itself equals the dense solve
        dense = np.zeros(nd)
        for v, c in olev.patches:
            if c == 0:
                idx = multigrid.patch_dofs(n, k, v)
                dense[idx] += sla.cho_solve(olev.patch_factor(v), r[idx])
        assert np.linalg.norm(ref - dense) < 1e-5 * np.linalg.norm(dense)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    assert err < 8 * lm.data_unit(fmt, ec), err


@pytest.mark.slow
def test_bf16_without_correction_stalls_and_matrix_split_recovers():
    n, k = 8, 5
    b = rhs.rhs(rhs.single_sine(), n, k)
    A = lambda q: sipg.kron_apply(q, n, k)
    plain = lm.Hierarchy(n, k, "bf16", 0)
    _, i0 = fgmres.fgmres(A, b, plain.precondition, rtol=1e-10, max_iters=12)
    split = lm.Hierarchy(n, k, "bf16", 2)
    _, i2 = fgmres.fgmres(A, b, split.precondition, rtol=1e-10, max_iters=12)
    assert not i0["converged"] and i0["rel_res_true"] > 1e-8
    assert i2["converged"] and i2["iterations"] <= 9
    # the rounded operator's lowest mode moves by more than its eigenvalue
    assert lm.lowest_eigen_shift(32, 5, "bf16", 0) > 5.0
    assert lm.lowest_eigen_shift(32, 5, "bf16", 2) < 0.1
