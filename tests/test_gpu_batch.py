"""GPU checks of batched solves over problems of uneven size and degree:
every batched stage (operator apply, V-cycle, FGMRES with Sec. 7.1's
multigrid preconditioner) gives each problem the result it gets when solved
alone, and the solves agree with the oracle.  The batched launches run the
same per-problem arithmetic in the same order as the one-problem calls, so
the comparisons with those are at rounding level (tolerance 1e-12 relative,
equality expected); captured-graph replays are checked against eager runs
with other GPU work and synchronisations between the replays."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, to_cpu, to_gpu
from oracle import fgmres as ofg
from oracle import multigrid, sipg
from paper_2407_09621_amd import inputs

pytestmark = pytest.mark.gpu

# (k, n): several degrees (two problems each of N = 3 and 4), meshes from 2
# to 24 cells, depths 1..4, single-level problems of 2 and 3 cells
MIXED = [(2, 4), (3, 6), (2, 24), (5, 3), (3, 8), (1, 12), (7, 2), (3, 3), (2, 16)]


def _vectors(B, seed):
    return [to_gpu(inputs.uniform_vector(m, seed + i)) for i, m in enumerate(B.sizes)]


def test_batch_shapes_and_rejections():
    from paper_2407_09621_amd import Batch, SipgError
    announce("batch shapes")
    B = Batch(MIXED)
    assert B.sizes == [n ** 3 * (k + 1) ** 3 for k, n in MIXED]
    with pytest.raises(SipgError, match="coarsest"):
        Batch([(2, 4), (2, 5)])  # 5 cells cannot be halved to a coarse grid of <= 3
    with pytest.raises(ValueError):
        B.apply(_vectors(B, 1)[:-1])


def test_batch_apply_matches_single_and_oracle():
    from paper_2407_09621_amd import Batch, Problem
    announce("batch apply")
    B = Batch(MIXED)
    us = _vectors(B, 10)
    vs = B.apply(us)
    for (k, n), u, v in zip(MIXED, us, vs):
        ref = Problem(k, n, n_levels=1).apply(u)
        assert rel_l2(to_cpu(v), to_cpu(ref)) < 1e-12, (k, n)
        assert rel_l2(to_cpu(v), sipg.kron_apply(to_cpu(u), n, k)) < 1e-13, (k, n)


@pytest.mark.parametrize("probs", [
    [(7, 1), (7, 2), (7, 3), (7, 4)],        # degree 7 on the matrix cores, one cell per wave
    [(3, 8), (3, 16)],                        # degree 3, 8 cells per wave
    [(3, 16), (3, 4), (3, 2), (3, 1), (3, 3)],  # degree 3, the batch falls back to 1 cell per wave
])
def test_batch_apply_matrix_core_degrees(probs):
    """Several mesh sizes of one matrix-core degree in one launch, plain and
    residual form."""
    from paper_2407_09621_amd import Batch, Problem
    announce("batch apply matrix cores", probs)
    B = Batch(probs)
    us = _vectors(B, 60)
    vs = B.apply(us)
    for (k, n), u, v in zip(probs, us, vs):
        assert rel_l2(to_cpu(v), sipg.kron_apply(to_cpu(u), n, k)) < 1e-13, (k, n)
    for (k, n), u in zip(probs, us):
        b = to_gpu(inputs.uniform_vector(n ** 3 * (k + 1) ** 3, 70 + n))
        r = to_cpu(Problem(k, n, n_levels=1).residual(b, u))
        ref = to_cpu(b) - sipg.kron_apply(to_cpu(u), n, k)
        assert rel_l2(r, ref) < 1e-12, (k, n)


def test_batch_apply_more_than_one_launch_per_degree():
    """20 problems of one degree: two launches of at most 16 problems."""
    from paper_2407_09621_amd import Batch
    announce("batch apply 20")
    probs = [(2, (2, 3, 4, 6)[i % 4]) for i in range(20)]
    B = Batch(probs)
    us = _vectors(B, 40)
    vs = B.apply(us)
    for (k, n), u, v in zip(probs, us, vs):
        assert rel_l2(to_cpu(v), sipg.kron_apply(to_cpu(u), n, k)) < 1e-13


@pytest.mark.parametrize("prec,ec", [("f64", 0), ("f32", 0), ("f16", 1)])
def test_batch_vcycle_matches_single(prec, ec):
    from paper_2407_09621_amd import Batch, Problem
    announce("batch vcycle", prec, ec)
    import torch
    B = Batch(MIXED, mg_precision=prec, error_correction=bool(ec))
    bs = _vectors(B, 60)
    xs = [torch.zeros_like(b) for b in bs]
    B.vcycle(xs, bs)
    for (k, n), b, x in zip(MIXED, bs, xs):
        P = Problem(k, n, mg_precision=prec, error_correction=bool(ec))
        x1 = torch.zeros_like(b)
        P.vcycle(x1, b)
        assert rel_l2(to_cpu(x), to_cpu(x1)) < 1e-12, (k, n)


def test_batch_vcycle_matches_oracle():
    from paper_2407_09621_amd import Batch
    announce("batch vcycle oracle")
    import torch
    probs = [(2, 4), (3, 6), (1, 8)]
    B = Batch(probs)
    bs = _vectors(B, 70)
    xs = [torch.zeros_like(b) for b in bs]
    B.vcycle(xs, bs)
    for (k, n), b, x in zip(probs, bs, xs):
        H = multigrid.Hierarchy(n, k)
        assert rel_l2(to_cpu(x), H.precondition(to_cpu(b))) < 1e-12, (k, n)


@pytest.mark.parametrize("use_graph", [False, True, "device"])
def test_batch_solve_matches_sequential(use_graph):
    from paper_2407_09621_amd import Batch
    announce("batch solve", use_graph)
    B = Batch(MIXED)
    bs = _vectors(B, 80)
    xs, infos = B.solve(bs, rtol=1e-10, use_graph=use_graph)
    xq, iq = B.solve(bs, rtol=1e-10, sequential=True)
    for i, (k, n) in enumerate(MIXED):
        assert infos[i]["rel_res_true"] < 1e-10, (k, n, infos[i])
        assert infos[i]["iterations"] == iq[i]["iterations"], (k, n)
        assert rel_l2(to_cpu(xs[i]), to_cpu(xq[i])) < 1e-12, (k, n)
        h, hq = np.array(infos[i]["history"]), np.array(iq[i]["history"])
        assert len(h) == len(hq)
        np.testing.assert_allclose(h, hq, rtol=1e-9, atol=1e-14)


def test_batch_solve_matches_oracle():
    from paper_2407_09621_amd import Batch
    announce("batch solve oracle")
    probs = [(2, 4), (3, 4), (1, 6)]
    B = Batch(probs)
    bs = _vectors(B, 90)
    xs, infos = B.solve(bs, rtol=1e-10)
    for i, (k, n) in enumerate(probs):
        H = multigrid.Hierarchy(n, k)
        A = H.levels[-1].A
        xo, io = ofg.fgmres(lambda v: A @ v, to_cpu(bs[i]), H.precondition, rtol=1e-10)
        assert abs(infos[i]["iterations"] - io["iterations"]) <= 1
        assert rel_l2(to_cpu(xs[i]), xo) < 1e-8


def test_batch_graph_replays_match_eager():
    """Four solves: the first captures one graph per Krylov step, the next
    ones replay them; GPU work of another kind and host synchronisations
    run between the replays.  Every replayed solve equals the eager solve of
    the same right-hand side."""
    from paper_2407_09621_amd import Batch
    announce("batch graph replays")
    import torch
    probs = [(2, 8), (3, 4), (5, 2), (2, 6)]
    Bg, Be = Batch(probs), Batch(probs)
    for rep in range(4):
        bs = _vectors(Bg, 100 + 10 * rep)
        xg, ig = Bg.solve(bs, rtol=1e-9, restart=8, use_graph=True)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
        xe, ie = Be.solve(bs, rtol=1e-9, restart=8, use_graph=False)
        for i in range(len(probs)):
            assert ig[i]["iterations"] == ie[i]["iterations"], (rep, i)
            assert rel_l2(to_cpu(xg[i]), to_cpu(xe[i])) < 1e-12, (rep, i)
            assert ig[i]["rel_res_true"] < 1e-9


def test_batch_solve_lowprec():
    """FP16 V-cycle with error correction inside the batched FGMRES: FP64
    accuracy and the FP64 batch's iteration counts (+1)."""
    from paper_2407_09621_amd import Batch
    announce("batch solve f16 ec")
    probs = [(3, 8), (2, 12), (5, 4), (7, 2)]
    B64, B16 = Batch(probs), Batch(probs, mg_precision="f16", error_correction=True)
    bs = _vectors(B64, 120)
    x64, i64 = B64.solve(bs, rtol=1e-10)
    x16, i16 = B16.solve(bs, rtol=1e-10)
    for i in range(len(probs)):
        assert i16[i]["rel_res_true"] < 1e-10
        assert i16[i]["iterations"] <= i64[i]["iterations"] + 1
        assert rel_l2(to_cpu(x16[i]), to_cpu(x64[i])) < 1e-8


def test_batch_zero_rhs_and_restart_growth():
    """A zero right-hand side converges at once with x = 0; growing the
    restart length reallocates the Krylov space and drops stale graphs."""
    from paper_2407_09621_amd import Batch
    announce("batch zero rhs")
    import torch
    probs = [(2, 4), (3, 4)]
    B = Batch(probs)
    bs = _vectors(B, 130)
    bs[0].zero_()
    xs = [torch.ones_like(b) for b in bs]
    for restart in (4, 12, 4):
        xs = [torch.ones_like(b) for b in bs]
        xs, infos = B.solve(bs, xs=xs, rtol=1e-10, restart=restart)
        assert infos[0]["iterations"] == 0 and float(xs[0].abs().max()) == 0.0
        assert infos[1]["rel_res_true"] < 1e-10


def test_device_scalar_solves_over_restarts_and_replays():
    """FGMRES with the scalars on the device and whole Krylov steps as
    graphs: restart 2 forces several cycles (so problems stop at different
    steps and cycles), a zero right-hand side rides along, and three solves
    replay the captured steps with other GPU work and host synchronisations
    between them; every solve equals the host-scalar solve of the same
    right-hand side (iterations, iterate, true residual)."""
    from paper_2407_09621_amd import Batch
    announce("batch device scalars")
    import torch
    probs = [(2, 8), (3, 4), (5, 2), (2, 6), (1, 4)]
    Bd, Bh = Batch(probs), Batch(probs)
    for rep in range(3):
        bs = _vectors(Bd, 140 + 10 * rep)
        bs[4].zero_()
        xd, idv = Bd.solve(bs, rtol=1e-9, restart=2, use_graph="device")
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
        xh, ih = Bh.solve(bs, rtol=1e-9, restart=2, use_graph=False)
        for i in range(len(probs)):
            assert idv[i]["iterations"] == ih[i]["iterations"], (rep, i, idv[i], ih[i])
            assert rel_l2(to_cpu(xd[i]), to_cpu(xh[i])) < 1e-10, (rep, i)
            assert idv[i]["rel_res_true"] < 1e-9 or i == 4
            np.testing.assert_allclose(idv[i]["history"], ih[i]["history"], rtol=1e-6, atol=1e-14)
        assert float(xd[4].abs().max()) == 0.0 and idv[4]["iterations"] == 0


def test_device_scalar_solve_lowprec_and_limits():
    """FP16-EC V-cycle inside the device-scalar FGMRES; an iteration budget
    stops every problem at the same count with SIPG_ERR_NOT_CONVERGED
    reported as a status, and restart above 32 is refused."""
    from paper_2407_09621_amd import Batch
    from paper_2407_09621_amd.sipg import SipgError
    announce("batch device scalars f16")
    probs = [(3, 8), (2, 12), (5, 4)]
    B16 = Batch(probs, mg_precision="f16", error_correction=True)
    bs = _vectors(B16, 160)
    xd, idv = B16.solve(bs, rtol=1e-10, use_graph="device", restart=8)
    xh, ih = B16.solve(bs, rtol=1e-10, use_graph=False, restart=8)
    for i in range(len(probs)):
        assert idv[i]["rel_res_true"] < 1e-10
        assert idv[i]["iterations"] == ih[i]["iterations"]
    xd, idv = B16.solve(bs, rtol=1e-14, use_graph="device", restart=8, max_iters=2)
    assert all(d["iterations"] == 2 and d["status"] == "SIPG_ERR_NOT_CONVERGED" for d in idv)
    with pytest.raises(SipgError):
        B16.solve(bs, restart=40, use_graph="device")


@pytest.mark.parametrize("k,n", [(5, 16), (7, 8)])
def test_autotune_keeps_apply(k, n):
    """The cell order the tuner picks changes which wave or workgroup tile
    handles a cell, never the cell's arithmetic: results stay bit-identical
    (degree 5: workgroup tiles; degree 7: matrix cores)."""
    from paper_2407_09621_amd import Problem
    announce("autotune apply", k, n)
    P = Problem(k, n, n_levels=1)
    u = to_gpu(inputs.uniform_vector(P.n_dofs(), 6))
    v0 = to_cpu(P.apply(u))
    assert P.autotune() in (1, 2, 4, 8)
    assert np.array_equal(to_cpu(P.apply(u)), v0)


def test_autotune_keeps_results():
    from paper_2407_09621_amd import Batch, Problem
    announce("autotune")
    P = Problem(3, 16, n_levels=1)
    u = to_gpu(inputs.uniform_vector(P.n_dofs(), 5))
    v0 = to_cpu(P.apply(u))
    best = P.autotune()
    assert best in (1, 2, 4, 8)
    assert np.array_equal(to_cpu(P.apply(u)), v0)
    B = Batch([(3, 16), (2, 16), (3, 16)])
    bs = _vectors(B, 140)
    x0, i0 = B.solve(bs, rtol=1e-10)
    B.autotune()
    x1, i1 = B.solve(bs, rtol=1e-10)
    for i in range(3):
        assert i0[i]["iterations"] == i1[i]["iterations"]
        assert rel_l2(to_cpu(x0[i]), to_cpu(x1[i])) < 1e-12
