"""Benchmark of the FP64 SIPG operator apply on one MI355X.

Workload (the paper's operator-apply benchmark, Sec. 4, at the apply
configuration of this project): the SIPG Laplacian on uniform Cartesian
meshes of the unit cube, degree 3 on 64^3 cells (16.8 MDoF), degree 5 on
40^3 (13.8 MDoF) and degree 7 on 32^3 (16.8 MDoF), input vectors seeded
U[-1, 1] FP64.  One step = one apply at each of the three degrees.  Inputs
are resident in HBM before timing; each degree rotates over 4 (u, v) pairs
(>= 1 GB) so the 256 MB last-level cache cannot hold the working set.

Prints one JSON line: value = total DoFs applied / second (GDoF/s) over the
timed steps, the roofline of the dominant kernel (HIP-event timing of the
kernel on its own stream; HBM traffic from the committed counter profile of
the same kernel source), the oracle's CPU rate on a bounded sample (one core
and all host cores), and, outside the timed region: the FP64 apply on the
vector units beside the matrix cores, the reduced-precision applies, the
FP64 / mixed-precision FGMRES + multigrid solves of degrees 3, 5, 7 on 16^3,
32^3 and 64^3 cells against a tight FP64 reference, single V-cycle times
against their byte model, flexible vs plain GMRES and multiplicative vs
additive smoothing, the batched uneven solves and the learned correction
stage.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = [(3, 64), (5, 40), (7, 32)]
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP16_PEAK_TFLOPS = 2500.0     # dense FP16 matrix-core peak
BYTES_PER_DOF = 16.0          # read u, write v (FP64)
# the kernel each benchmark degree runs (FP64 apply)
APPLY_KERNEL = {"k3_n64": "apply_mfma4_kernel", "k5_n40": "apply_wave_kernel",
                "k7_n32": "apply_mfma8eo_kernel"}
ROTATE = 4
PROFILE = os.path.join(ROOT, "profiles", "apply_f64_k3n64_k5n40_k7n32.md")
KERNEL_SOURCE = {"apply_mfma4_kernel": "sipg_mfma.hip", "apply_mfma8eo_kernel": "sipg_mfma.hip",
                 "apply_wave_kernel": "sipg_valu.hip"}


def source_sha16(kernel):
    """sha256 prefix of the kernel's definition in its source file (from the
    template line before `void <kernel>(` to the closing brace at column 0),
    so that edits elsewhere in the file keep a profile valid."""
    import hashlib
    path = os.path.join(ROOT, "paper_2407_09621_amd", "csrc", KERNEL_SOURCE[kernel])
    text = open(path).read()
    at = text.find("void " + kernel + "(")
    if at < 0:
        return None
    start = text.rfind("\ntemplate", 0, at) + 1
    end = text.find("\n}\n", at)
    return hashlib.sha256(text[start:end + 3].encode()).hexdigest()[:16]


def profiled_traffic(kernel, key):
    """HBM bytes per launch of `kernel` (FETCH + WRITE, calibrated) from the
    traffic block of the committed apply profile, or None when the profile
    lacks it or was taken from a different source of that kernel."""
    try:
        text = open(PROFILE).read()
        block = text.split("```traffic-json", 1)[1].split("```", 1)[0]
        rows = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    row = rows.get(key)
    if not row or row.get("kernel") != kernel or row.get("source_sha16") != source_sha16(kernel):
        return None
    return row["fetch_bytes"] + row["write_bytes"]



def flops_per_dof(k):
    """Model count: 7 sum-factorized N x N products per cell (14 N flop/DoF)
    plus face traces and expansions (48 flop/DoF)."""
    return 14 * (k + 1) + 48


def _oracle_import(_=None):
    from oracle import sipg  # noqa: F401
    from paper_2407_09621_amd import inputs  # noqa: F401


def _oracle_apply_round(_=None):
    """One oracle apply at each benchmark degree; returns (DoFs, seconds)."""
    from oracle import sipg as osipg
    from paper_2407_09621_amd import inputs
    total, t = 0, 0.0
    for k, n in CONFIGS:
        u = inputs.uniform_vector(n ** 3 * (k + 1) ** 3, seed=2 + k)
        t0 = time.perf_counter()
        osipg.kron_apply(u, n, k)
        t += time.perf_counter() - t0
        total += u.size
    return total, t


def measured_copy_rate(stream, nbytes=1 << 30, reps=20):
    """Device copy of nbytes (read + write) between two buffers, HIP events
    on the stream: the achievable HBM rate, GB/s of bytes moved."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    b2 = torch.empty_like(a)
    with torch.cuda.stream(stream):
        b2.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b2.copy_(a)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b2
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def _oracle_solve_sample():
    """The oracle's FGMRES(30) + V(2,2) solve of the sine problem on the small
    configuration (k=2, 8^3 cells), rtol 1e-10, one core: hierarchy setup
    (assembly, patch factors, coarse factor) and solve time."""
    from oracle import fgmres, multigrid, rhs
    n, k = 8, 2
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(n, k)
    A = H.levels[-1].A
    prob = rhs.single_sine()
    b = rhs.rhs(prob, n, k)
    t1 = time.perf_counter()
    x, info = fgmres.fgmres(lambda v: A @ v, b, H.precondition, rtol=1e-10)
    t2 = time.perf_counter()
    return {"setup_seconds": round(t1 - t0, 3), "solve_seconds": round(t2 - t1, 3),
            "iterations": info["iterations"], "l2_error": rhs.l2_error(prob, x, n, k),
            "cores": 1, "sample": "k=2, 8^3 cells (13,824 DoFs), sine problem, rtol 1e-10"}


def _oracle_csr_sample(reps=100):
    """The oracle's assembled CSR matrix (3D/2D quadrature) on the small
    configuration (k=2, 8^3 cells, 13,824 DoFs): assembly time and 100
    sparse products on one core (larger meshes need too much host memory
    for the assembled matrix)."""
    from oracle import sipg
    from paper_2407_09621_amd import inputs
    t0 = time.perf_counter()
    A = sipg.assemble(8, 2)
    ta = time.perf_counter() - t0
    u = inputs.uniform_vector(A.shape[0], 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        A @ u
    dt = time.perf_counter() - t0
    return {"value": A.shape[0] * reps / dt / 1e9, "unit": "GDoF/s", "cores": 1,
            "sample": f"k=2, 8^3 cells: assembly {ta:.2f} s, {reps} products in {dt:.3f} s, "
                      f"{A.nnz} nonzeros"}


def _oracle_mapped_sample():
    """The oracle's apply on trilinear cells (quadrature blocks cell by cell,
    one core) on a sample of cells of the benchmark meshes with the smooth
    deformation: 128 cells at k=3 (64^3) and 16 at k=7 (32^3)."""
    import numpy as np
    from oracle import mapped
    from paper_2407_09621_amd import inputs
    out = {}
    for k, n, count in ((3, 64, 128), (7, 32, 16)):
        V = inputs.mesh_vertices(n, "smooth", MAPPED_AMPLITUDE, seed=1)
        u = inputs.uniform_vector(n ** 3 * (k + 1) ** 3, seed=60 + k)
        cells = np.random.default_rng(k).integers(0, n ** 3, count)
        mapped.apply_cells_mapped(u, n, k, V, cells[:1])   # reference tables
        t0 = time.perf_counter()
        mapped.apply_cells_mapped(u, n, k, V, cells)
        dt = time.perf_counter() - t0
        out[f"k{k}_n{n}"] = {"value": count * (k + 1) ** 3 / dt / 1e9, "unit": "GDoF/s",
                             "cores": 1, "sample": f"{count} random cells, {dt:.2f} s"}
    return out


def cpu_baseline(max_workers=16):
    """The oracle's Kronecker-sum apply (numpy/scipy, FP64, single-threaded
    per process) at the full benchmark sizes: one apply per degree on one
    core, then one apply per degree in each of W worker processes at once
    (all host cores, at most the box's share of 16).  Runs before the GPU is
    touched; the workers are spawned interpreters that never import torch."""
    import multiprocessing as mp
    dofs1, t1 = _oracle_apply_round()
    W = max(1, min(max_workers, os.cpu_count() or 1))
    env_keep = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                "MKL_NUM_THREADS")}
    for v in env_keep:
        os.environ[v] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(W) as pool:
            pool.map(_oracle_import, range(W))
            t0 = time.perf_counter()
            res = pool.map(_oracle_apply_round, range(W))
            wall = time.perf_counter() - t0
    finally:
        for v, val in env_keep.items():
            if val is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = val
    dofs_all = sum(r[0] for r in res)
    geo = _oracle_mapped_sample()
    csr = _oracle_csr_sample()
    solve = _oracle_solve_sample()
    return {"value": dofs_all / wall / 1e9, "unit": "GDoF/s", "cores": W, "kind": "oracle",
            "general_geometry": geo, "csr_spmv_small": csr, "solve_small": solve,
            "sample": f"{W} worker processes at once, each one FP64 apply at k=3 (64^3), "
                      f"k=5 (40^3) and k=7 (32^3) by the oracle's Kronecker-sum path "
                      f"(scipy.sparse, one thread each): {3 * W} applies, "
                      f"{dofs_all / 1e6:.0f} MDoF in {wall:.1f} s wall",
            "single_core": {"value": dofs1 / t1 / 1e9, "unit": "GDoF/s", "cores": 1,
                            "sample": f"one apply per degree, {dofs1 / 1e6:.1f} MDoF in "
                                      f"{t1:.1f} s"}}


SOLVE_CONFIGS = [(k, n) for k in (3, 5, 7) for n in (16, 32, 64)]
SOLVE_CONFIGS_QUICK = [(3, 64), (5, 32), (7, 32)]
SOLVE_VARIANTS = [("f64", 0), ("f32", 0), ("f16", 0), ("f16", 1), ("bf16", 0), ("bf16", 1),
                  ("bf16", 2)]
# the discretization error lies below this for k = 5, 7 on these meshes (the
# round-off floor of the L2 error, ~1e-12): there the 1% test of the L2 error
# is not informative and the algebraic error ||x - x_ref|| / ||x_ref|| is
# the measure
L2_FLOOR = 1e-11


def progress(*what):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench]", *what, file=sys.stderr, flush=True)


def _timed_solve(P, b, rtol, torch):
    """Warm-up solve (allocates the Krylov space), then the timed solve."""
    x, info = P.fgmres(b, rtol=rtol, max_iters=200, raise_on_nonconvergence=False)
    x.zero_()
    torch.cuda.synchronize()
    return P.fgmres(b, x=x, rtol=rtol, max_iters=200, raise_on_nonconvergence=False)


def run_solves(configs):
    """FP64 FGMRES(30) + V(2,2) solves of the sine problem (Sec. 7.2) with the
    V-cycle in FP64, FP32, FP16, BF16 (with and without error correction),
    outside the timed apply region.  Per configuration a reference FP64 solve
    to rtol 1e-14 gives the reference L2 error and solution x_ref.  Per
    variant: time to rtol 1e-10 (after a warm-up solve), iterations, true
    residual, L2 error, algebraic error ||x - x_ref|| / ||x_ref||, the speed
    multiple over the FP64 solve, and whether the L2 error is within 1% of
    the reference (where the discretization error is above the floor); a
    variant that misses 1% at rtol 1e-10 is solved again at 1e-12 and the
    time of that solve is reported as the time to reach it."""
    import torch
    from paper_2407_09621_amd import Problem, SipgError, inputs
    out = {}
    amps, pqr = inputs.single_sine_modes()
    for k, n in configs:
        row = {}
        P = Problem(k, n)
        b = P.rhs_sines(amps, pqr)
        xr, ir = P.fgmres(b, rtol=1e-14, max_iters=60, raise_on_nonconvergence=False)
        e_ref = P.l2_error_sines(amps, pqr, xr)
        nref = float(torch.linalg.vector_norm(xr))
        P.close()
        at_floor = e_ref < L2_FLOOR
        for prec, ec in SOLVE_VARIANTS:
            name = prec + ("" if ec == 0 else ("_ec" if ec == 1 else "_ecm"))
            try:
                P = Problem(k, n, mg_precision=prec, error_correction=ec)
            except SipgError as e:
                row[name] = {"status": "SIPG_ERR_UNSUPPORTED", "reason": str(e)}
                continue
            x, info = _timed_solve(P, b, 1e-10, torch)
            err = P.l2_error_sines(amps, pqr, x)
            r = {"seconds": round(info["seconds"], 5), "iterations": info["iterations"],
                 "rel_res_true": info["rel_res_true"], "l2_error": err,
                 "algebraic_error": float(torch.linalg.vector_norm(x - xr)) / nref,
                 "status": info["status"]}
            if not at_floor:
                r["l2_within_1pct"] = abs(err - e_ref) <= 0.01 * e_ref
                if not r["l2_within_1pct"]:
                    x2, i2 = _timed_solve(P, b, 1e-12, torch)
                    e2 = P.l2_error_sines(amps, pqr, x2)
                    r["tighter"] = {"rtol": 1e-12, "seconds": round(i2["seconds"], 5),
                                    "iterations": i2["iterations"], "l2_error": e2,
                                    "l2_within_1pct": abs(e2 - e_ref) <= 0.01 * e_ref}
                    del x2
            row[name] = r
            P.close()
            del x
        base = row["f64"]
        for v in row.values():
            if "seconds" in v:
                v["speedup_vs_f64"] = round(base["seconds"] / v["seconds"], 3)
        progress(f"solves k={k} n={n} done")
        out[f"k{k}_n{n}"] = {"n_dofs": n ** 3 * (k + 1) ** 3,
                             "reference": {"rtol": 1e-14, "iterations": ir["iterations"],
                                           "rel_res_true": ir["rel_res_true"],
                                           "l2_error": e_ref, "at_l2_floor": at_floor},
                             **row}
        del b, xr
        torch.cuda.empty_cache()
    return out


# V(2,2) bytes per fine DoF (8 colours x (residual: read x, b, write r; patch
# solve: read r, x, write x) per sweep, 4 sweeps, transfers, x 8/7 for the
# coarser levels), per vector element size
VCYCLE_BYTES_PER_DOF = {8: 940.0, 4: 470.0}


def run_vcycles(configs=((3, 64), (5, 32), (7, 32)), reps=5):
    """One V(2,2) from zero (HIP events, mean of `reps`) in FP64, FP32 and
    FP16-EC against the model's bytes per fine DoF (HBM roofline); FP64 and
    FP32 also with the fused colour step (one launch per smoother colour)
    instead of a residual launch and the patch solves."""
    import torch
    from paper_2407_09621_amd import Problem, inputs
    out = {}
    for k, n in configs:
        for prec, ec, es, sm in (("f64", 0, 8, "multiplicative"),
                                 ("f64", 0, 8, "multiplicative_fused"),
                                 ("f32", 0, 4, "multiplicative"),
                                 ("f32", 0, 4, "multiplicative_fused"),
                                 ("f16", 1, 4, "multiplicative")):
            P = Problem(k, n, mg_precision=prec, error_correction=ec, smoother=sm)
            b = torch.from_numpy(inputs.uniform_vector(P.n_dofs(), 5)).cuda()
            x = torch.zeros_like(b)
            P.vcycle(x, b)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                x.zero_()
                P.vcycle(x, b)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            model = VCYCLE_BYTES_PER_DOF[es] * P.n_dofs()
            out[f"k{k}_n{n}_{prec}{'_ec' if ec else ''}{'_fused' if 'fused' in sm else ''}"] = {
                "ms": round(ms, 4), "model_bytes": model,
                "model_gb_s": round(model / ms / 1e6, 1),
                "hbm_frac": round(model / ms / 1e6 / HBM_PEAK_GBS, 4)}
            P.close()
            del b, x
    torch.cuda.empty_cache()
    progress("v-cycles done")
    return out


def run_small_solve():
    """The small configuration (k=2, 8^3 cells, 13,824 DoFs): FP64 FGMRES(30)
    + V(2,2) of the sine problem to rtol 1e-10 on the GPU, beside the
    oracle's solve of the same problem in the CPU baseline."""
    from paper_2407_09621_amd import Problem, inputs
    P = Problem(2, 8)
    amps, pqr = inputs.single_sine_modes()
    b = P.rhs_sines(amps, pqr)
    P.fgmres(b, rtol=1e-10)
    x, info = P.fgmres(b, rtol=1e-10)
    out = {"workload": "k=2, 8^3 cells, sine problem, rtol 1e-10",
           "seconds": round(info["seconds"], 5), "iterations": info["iterations"],
           "rel_res_true": info["rel_res_true"], "l2_error": P.l2_error_sines(amps, pqr, x)}
    P.close()
    return out


def run_comparisons(k=3, n=32):
    """The paper's robustness comparisons (Sec. 7.2): flexible vs
    non-flexible GMRES with the multiplicative smoother, and the
    multiplicative vs additive vertex-patch smoother (FP64 V-cycles), on the
    sine problem to rtol 1e-10."""
    import torch
    from paper_2407_09621_amd import Problem, inputs
    amps, pqr = inputs.single_sine_modes()
    out = {}
    for name, kw, var in (("fgmres_multiplicative", {}, "fgmres"),
                          ("gmres_multiplicative", {}, "gmres"),
                          ("fgmres_additive", {"smoother": "additive"}, "fgmres"),
                          ("gmres_additive", {"smoother": "additive"}, "gmres")):
        P = Problem(k, n, **kw)
        b = P.rhs_sines(amps, pqr)
        P.fgmres(b, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False, variant=var)
        x, info = P.fgmres(b, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False,
                           variant=var)
        out[name] = {"iterations": info["iterations"], "seconds": round(info["seconds"], 5),
                     "rel_res_true": info["rel_res_true"], "status": info["status"],
                     "l2_error": P.l2_error_sines(amps, pqr, x)}
        P.close()
        del x, b
    torch.cuda.empty_cache()
    progress("krylov / smoother comparison done")
    return {"workload": f"k={k}, {n}^3 cells, sine solution", **out}


def patchwise_flops_per_dof(k):
    """Products of the patch-wise evaluation as implemented: per patch three
    window stiffness contractions (2 (2N)^4 flop each) and four block-diagonal
    window mass contractions (16 N^4 flop each), about n^3 patches of N^3
    DoFs per cell: 160 N flop/DoF (the paper's count with full 2N x 2N
    masses is 7 x 2 (2N)^4 / (N^3) = 224 N, Table flop_byte)."""
    return 160 * (k + 1)


def _event_ms(fn, reps, stream):
    import torch
    fn(0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        fn(i)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


# cells per direction giving ~16 MDoF for each N = k + 1
SWEEP_N = {1: 128, 2: 85, 3: 64, 4: 51, 5: 42, 6: 36, 7: 32}


def run_patchwise(stream, reps=10):
    """The paper's patch-wise evaluation (Sec. 2.1, Fig. patch_int; vertex
    patches of 2x2x2 cells, 2N x 2N window matrices) beside the cell-wise
    apply, over the matrix dimensions of Fig. all_perf: cell-wise N = k+1 =
    2..8 and patch-wise G = 2(k+1) = 4..16 (even), each at ~16 MDoF (FP64,
    HIP events, 2 rotating vector pairs)."""
    import torch
    from paper_2407_09621_amd import Problem, inputs
    out = {}
    for k, n in SWEEP_N.items():
        P = Problem(k, n, n_levels=1)
        nd = P.n_dofs()
        us = [torch.from_numpy(inputs.uniform_vector(nd, seed=40 + k + i)).cuda() for i in range(2)]
        vs = [torch.empty_like(us[0]) for _ in range(2)]
        mc = _event_ms(lambda i: P.apply(us[i % 2], vs[i % 2], stream=stream), reps, stream)
        mp = _event_ms(lambda i: P.apply_patchwise(us[i % 2], vs[i % 2], stream=stream), reps,
                       stream)
        gc, gp = nd / mc / 1e6, nd / mp / 1e6
        out[f"k{k}_n{n}"] = {
            "n_dofs": nd, "cell_N": k + 1, "patch_G": 2 * (k + 1),
            "cellwise_ms": round(mc, 4), "cellwise_gdof_s": round(gc, 2),
            "cellwise_tflops_model": round(gc * flops_per_dof(k) / 1e3, 2),
            "patchwise_ms": round(mp, 4), "patchwise_gdof_s": round(gp, 2),
            "patchwise_tflops_model": round(gp * patchwise_flops_per_dof(k) / 1e3, 2),
            "patchwise_frac_fp64_peak": round(gp * patchwise_flops_per_dof(k) / 1e3
                                              / FP64_PEAK_TFLOPS, 4),
            "cellwise_over_patchwise": round(mp / mc, 2)}
        P.close()
        del us, vs
    torch.cuda.empty_cache()
    progress("patch-wise sweep done")
    return out


def mapped_flops_per_dof(k):
    """Model count of the trilinear-cell apply as implemented (FP64 vector
    units): 16 sum-factorized N x N line products per cell (32 N flop/DoF),
    ~206 flop per quadrature point for the Jacobian, its cofactors and the
    metric product, and per cell 6 N^2 face points that each take
    46 N flop of face-trace products and ~400 flop of two Jacobians, normals
    and the flux terms, plus the expansion into the cell
    (= 32 N + 500 + 2400 / N per DoF)."""
    N = k + 1
    return 32 * N + 500 + 2400 / N


MAPPED_AMPLITUDE = 0.08


def run_mapped(stream, reps=10):
    """General geometry (trilinear hexahedra, Sec. 2.1 mapped integrals):
    the apply at the benchmark sizes on the unit cube moved by a smooth
    interior deformation (amplitude 0.08, seeded), timed with HIP events
    beside the Cartesian apply on the same problem; then FGMRES + V(2,2)
    solves (the Cartesian patch smoother and coarse solve as an approximate
    inverse) on mapped and Cartesian meshes with the same seeded random
    right-hand side, to rtol 1e-10."""
    import torch
    from paper_2407_09621_amd import Problem, inputs
    out = {"mesh": f"unit cube, smooth deformation amplitude {MAPPED_AMPLITUDE}, seed 1"}
    for k, n in ((3, 64), (5, 40), (7, 32)):
        P = Problem(k, n, n_levels=1)
        nd = P.n_dofs()
        us = [torch.from_numpy(inputs.uniform_vector(nd, seed=60 + k + i)).cuda() for i in range(2)]
        vs = [torch.empty_like(us[0]) for _ in range(2)]
        mc = _event_ms(lambda i: P.apply(us[i % 2], vs[i % 2], stream=stream), reps, stream)
        t0 = time.perf_counter()
        P.set_geometry(inputs.mesh_vertices(n, "smooth", MAPPED_AMPLITUDE, seed=1))
        setup = time.perf_counter() - t0
        mm = _event_ms(lambda i: P.apply(us[i % 2], vs[i % 2], stream=stream), reps, stream)
        g = nd / mm / 1e6
        tf = g * mapped_flops_per_dof(k) / 1e3
        bpd = BYTES_PER_DOF + 72.0 / (k + 1) ** 3
        out[f"k{k}_n{n}"] = {
            "n_dofs": nd, "mapped_ms": round(mm, 4), "mapped_gdof_s": round(g, 2),
            "cartesian_ms": round(mc, 4), "mapped_over_cartesian_time": round(mm / mc, 2),
            "flops_per_dof_model": round(mapped_flops_per_dof(k), 1),
            "tflops_model": round(tf, 2), "frac_fp64_vector_peak": round(tf / FP64_PEAK_TFLOPS, 4),
            "hbm_gb_s_algorithmic": round(g * bpd, 1),
            "geometry_setup_s": round(setup, 3)}
        P.close()
        del us, vs
        torch.cuda.empty_cache()
    solves = {}
    for k, n in ((3, 32), (7, 16)):
        for geo in ("cartesian", "mapped", "jitter0.1"):
            P = Problem(k, n)
            if geo == "mapped":
                P.set_geometry(inputs.mesh_vertices(n, "smooth", MAPPED_AMPLITUDE, seed=1))
            elif geo == "jitter0.1":   # interior vertices moved by up to 0.1 h
                P.set_geometry(inputs.mesh_vertices(n, "jitter", 0.1, seed=8))
            b = torch.from_numpy(inputs.uniform_vector(P.n_dofs(), seed=77)).cuda()
            P.fgmres(b, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False)
            x, info = P.fgmres(b, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False)
            solves[f"k{k}_n{n}_{geo}"] = {"iterations": info["iterations"],
                                          "seconds": round(info["seconds"], 5),
                                          "rel_res_true": info["rel_res_true"],
                                          "status": info["status"]}
            P.close()
            del x, b
    out["solves"] = solves
    torch.cuda.empty_cache()
    progress("general-geometry apply and solves done")
    return out


BATCH_SEED, BATCH_COUNT, BATCH_RESTART = 4, 64, 6
SMALL_EDGES = (4, 6, 8, 12)


def run_batch(count=BATCH_COUNT, seed=BATCH_SEED, restart=BATCH_RESTART,
              edges=(16, 24, 32, 48, 64)):
    """Batched uneven solves: `count` seeded problems (mesh edge in
    {16,24,32,48,64}, k in 2..7), right-hand sides from 4 seeded sine modes,
    FGMRES(restart) + FP64 V(2,2) to rtol 1e-10.  Times one batched solve
    with captured V-cycle graphs (after a warm-up solve that captures them),
    one batched solve without graphs, one with the FGMRES scalars on the
    device and every whole Krylov step a captured graph (after its own
    warm-up), and the one-problem-at-a-time loop on the same handles.  Aggregate rate = sum over problems of DoFs x
    iterations / wall time.  The Krylov space holds restart + 1 and restart
    vectors per problem, sized so the whole batch fits in HBM (the sine
    right-hand sides converge in <= 3 iterations, so no restart occurs).
    The same measurement on small meshes (edges 4..12) shows the launch-bound
    regime that batching and graph capture target."""
    import torch
    from paper_2407_09621_amd import Batch, inputs
    pairs = [(k, n) for n, k in inputs.batch_problems(seed, count, edges=edges)]
    B = Batch(pairs)
    B.autotune()
    modes = [inputs.sine_modes(1000 * seed + i) for i in range(count)]
    bs = [B.rhs_sines(i, *modes[i]) for i in range(count)]
    torch.cuda.synchronize()
    res = {}
    for name, kw in [("warmup", dict(use_graph=True)), ("graph", dict(use_graph=True)),
                     ("eager", dict(use_graph=False)),
                     ("warmup_device", dict(use_graph="device")),
                     ("device", dict(use_graph="device")), ("sequential", dict(sequential=True))]:
        xs = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, infos = B.solve(bs, xs=xs, rtol=1e-10, restart=restart, max_iters=100, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = [i["iterations"] for i in infos]
        work = sum(m * it for m, it in zip(B.sizes, its))
        res[name] = {"seconds": round(dt, 4), "gdof_s": round(work / dt / 1e9, 3),
                     "iterations_total": sum(its), "iterations_max": max(its),
                     "max_rel_res_true": max(i["rel_res_true"] for i in infos),
                     "converged": all(i["status"] == "SIPG_OK" for i in infos)}
        if name in ("graph", "device", "sequential"):
            res[name]["l2_errors"] = [B.l2_error_sines(i, *modes[i], xs[i]) for i in range(count)]
        del xs
        torch.cuda.empty_cache()
    eg, es = res["graph"].pop("l2_errors"), res["sequential"].pop("l2_errors")
    ed = res["device"].pop("l2_errors")
    out = {"problems": count, "seed": seed, "restart": restart,
           "total_dofs": int(sum(B.sizes)),
           "degrees": sorted({k for k, _ in pairs}), "edges": sorted({n for _, n in pairs}),
           "l2_max_rel_diff_vs_sequential": max(abs(a - b) / b for a, b in zip(eg, es)),
           "speedup_graph_vs_sequential": round(res["sequential"]["seconds"] / res["graph"]["seconds"], 3),
           "speedup_graph_vs_eager": round(res["eager"]["seconds"] / res["graph"]["seconds"], 3),
           "l2_max_rel_diff_device_vs_sequential": max(abs(a - b) / b for a, b in zip(ed, es)),
           "speedup_device_vs_sequential": round(res["sequential"]["seconds"] / res["device"]["seconds"], 3),
           "speedup_device_vs_graph": round(res["graph"]["seconds"] / res["device"]["seconds"], 3)}
    out.update({k: v for k, v in res.items() if not k.startswith("warmup")})
    progress(f"batch of {count} (edges {edges}) done")
    B.close()
    del bs
    torch.cuda.empty_cache()
    return out


CNN_CHAINS = 5000   # x 4 pairs = the configured 20,000 solver-made pairs
CNN_CHUNK = 250     # right-hand sides per training call


def run_learned(chains=CNN_CHAINS, loss="residual"):
    """Learned correction stage at k = 3 on 32^3 cells (128^3 grid): train
    on the GPU with 4 solver-made pairs per right-hand side (one Adam step
    per pair; loss "residual": what the correction leaves of the post-V-cycle
    residual, on the whole grid; "mse": the pointwise error on 8 random 32^3
    crops), measure on 3 held-out pairs the fraction of the residual the
    stage leaves (sqrt of the residual loss, with the stage's own step
    length) before and after training, then solve held-out right-hand sides (4 sine modes, seeds
    100000..100003) to rtol 1e-10 with and without the stage.  Also times
    the network forward on the full grid (FP16 matrix cores;
    2 x 32 x 32 x 27 x 2 flop per point in each 32 -> 32 layer)."""
    import numpy as np
    import torch
    from paper_2407_09621_amd import Network, Problem, inputs
    k, n = 3, 32
    P = Problem(k, n)
    net = Network(seed=1)
    # held-out pairs from a right-hand side outside the training draws
    b0 = P.rhs_sines(*inputs.sine_modes(300))
    x0 = torch.zeros_like(b0)
    P.vcycle(x0, b0)
    rho, _, _ = Network.make_pairs(P, x0, 3)
    N = k + 1

    def to_cells(g):  # grid (gx + G (gy + G gz)) -> cell-blocked vector
        a = g.double().reshape(n, N, n, N, n, N).permute(0, 2, 4, 1, 3, 5).contiguous()
        return a.reshape(-1)

    def held_out(nw):
        vals = [float(nw.gradient_residual(P, to_cells(rho[j]))[1].item()) for j in range(3)]
        return float(np.sqrt(np.mean(vals)))

    # in chunks of CNN_CHUNK right-hand sides (the network keeps its Adam
    # state and output scale between calls), one progress line per chunk
    tr = None
    for c0 in range(0, chains, CNN_CHUNK):
        part = net.train(P, n_chains=min(CNN_CHUNK, chains - c0), chain_length=4,
                         crops_per_pair=8, crop=32, lr=1e-3, seed=2 + c0, loss=loss)
        if tr is None:
            tr = part
        else:
            tr.update(steps=tr["steps"] + part["steps"], loss_last=part["loss_last"],
                      sigma=part["sigma"], seconds=tr["seconds"] + part["seconds"],
                      seconds_pairs=tr["seconds_pairs"] + part["seconds_pairs"])
        progress(f"learned stage: {tr['steps']} pairs ({loss} loss), {tr['seconds']:.0f} s")
    untrained = Network(seed=1)
    untrained.set_params(untrained.get_params()[0], tr["sigma"])
    factor_before, factor_after = held_out(untrained), held_out(net)
    P.attach(net)
    rows = []
    for seed in range(100000, 100004):
        amps, pqr = inputs.sine_modes(seed)
        b = P.rhs_sines(amps, pqr)
        P.fgmres(b, rtol=1e-10)                      # warm-up (Krylov space)
        res = {}
        for name, ul in (("plain", False), ("learned", True)):
            x, info = P.fgmres(b, rtol=1e-10, use_learned=ul)
            res[name] = {"iterations": info["iterations"], "seconds": round(info["seconds"], 5),
                         "rel_res_true": info["rel_res_true"], "fell_back": info["fell_back"],
                         "l2_error": P.l2_error_sines(amps, pqr, x)}
        rows.append({"seed": seed, **res})
    G = n * (k + 1)
    g = torch.rand((1, G, G, G), device="cuda", dtype=torch.float32) * 2 - 1
    net.forward(g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        net.forward(g)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 20
    mid_flop = 2 * 32 * 32 * 27 * G ** 3
    fwd_flop = 2 * mid_flop + 2 * 2 * 27 * 32 * G ** 3
    tp = sum(r["plain"]["seconds"] for r in rows)
    tl = sum(r["learned"]["seconds"] for r in rows)
    return {"workload": "k=3, 32^3 cells (128^3 grid), 2,097,152 DoFs",
            "training": {"pairs": tr["steps"], "loss": loss, **tr},
            "held_out_residual_factor": {"untrained": round(factor_before, 4),
                                         "trained": round(factor_after, 4)},
            "solves": rows,
            "iterations_plain": [r["plain"]["iterations"] for r in rows],
            "iterations_learned": [r["learned"]["iterations"] for r in rows],
            "speedup_learned_vs_plain": round(tp / tl, 3),
            "forward_ms": round(ms, 4), "forward_tflops": round(fwd_flop / ms / 1e9, 1),
            "forward_frac_fp16_peak": round(fwd_flop / ms / 1e9 / FP16_PEAK_TFLOPS, 4)}


def lp_apply_rates(probs, stream, reps):
    """Reduced-precision applies (FP32 storage, 8 B/DoF) at the apply sizes,
    rotating over 2 ROTATE (u, v) pairs (>= 1 GB, like the FP64 leg)."""
    import torch
    out = {}
    R = 2 * ROTATE
    for k, n, P, nd, us, vs in probs:
        u32 = [us[i % ROTATE].float().mul_(1.0 + 0.001 * i) for i in range(R)]
        v32 = [torch.empty_like(u32[0]) for _ in range(R)]
        for prec, ec in [("f32", 0), ("f16", 0), ("f16", 1), ("bf16", 0), ("bf16", 1)]:
            P.apply_lp(u32[0], v32[0], precision=prec, ec=ec, stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(reps):
                P.apply_lp(u32[i % R], v32[i % R], precision=prec, ec=ec, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            g = nd / (ms * 1e-3) / 1e9
            out[f"k{k}_n{n}_{prec}{'_ec' if ec else ''}"] = {
                "ms_per_apply": round(ms, 5), "gdof_s": round(g, 2),
                "hbm_frac": round(g * 8.0 / HBM_PEAK_GBS, 4)}
        del u32, v32
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve measurements")
    ap.add_argument("--quick-solves", action="store_true",
                    help="solve only k=3 on 64^3, k=5 and k=7 on 32^3 (default: all nine "
                         "degree 3/5/7 x 16^3/32^3/64^3 configurations)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve measurement")
    ap.add_argument("--no-patchwise", action="store_true",
                    help="skip the patch-wise evaluation and matrix-size sweep")
    ap.add_argument("--batch-count", type=int, default=BATCH_COUNT,
                    help="problems in the batched-solve measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-stage measurement")
    ap.add_argument("--no-mapped", action="store_true",
                    help="skip the general-geometry (trilinear cells) measurement")
    ap.add_argument("--cnn-loss", choices=["residual", "mse"], default="residual",
                    help="training loss of the learned stage")
    ap.add_argument("--cnn-chains", type=int, default=CNN_CHAINS,
                    help="right-hand sides for the learned stage's training (4 pairs each)")
    ap.add_argument("--mode", choices=["bench", "profile"], default="bench",
                    help="profile: a few applies per degree (matrix and vector units, "
                         "patch-wise, FP16/BF16-EC), three k=3 solves, V-cycles of k=5 and 7, "
                         "two short training "
                         "runs, network forwards and a plain copy of a known size (for "
                         "rocprofv3 kernel traces and counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # the oracle's CPU rate first, before anything initialises the GPU (its
    # worker processes are spawned)
    cpu = None if (args.no_cpu or args.mode == "profile") else cpu_baseline()

    import torch
    from paper_2407_09621_amd import Problem, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    probs = []
    for k, n in CONFIGS:
        P = Problem(k, n, n_levels=1)
        nd = P.n_dofs()
        base = torch.from_numpy(inputs.uniform_vector(nd, seed=2 + k)).to(dev)
        us = [base.clone() for _ in range(ROTATE)]
        for i in range(1, ROTATE):
            us[i].mul_(1.0 - 0.01 * i)
        vs = [torch.empty_like(base) for _ in range(ROTATE)]
        probs.append((k, n, P, nd, us, vs))
    torch.cuda.synchronize()

    if args.mode == "profile":
        for k, n, P, nd, us, vs in probs:
            for i in range(5):
                P.apply(us[i % ROTATE], vs[i % ROTATE], stream=stream)
            torch.cuda.synchronize()
            print(f"profiled apply k={k} n={n}: 5 launches, {nd} DoFs", flush=True)
            if k in (3, 7):
                for i in range(5):
                    P.apply(us[i % ROTATE], vs[i % ROTATE], stream=stream, units="vector")
                torch.cuda.synchronize()
                print(f"profiled vector-unit apply k={k} n={n}: 5 launches", flush=True)
            for i in range(3):
                P.apply_patchwise(us[i % ROTATE], vs[i % ROTATE], stream=stream)
            torch.cuda.synchronize()
            print(f"profiled patch-wise apply k={k} n={n}: 3 launches", flush=True)
            u32 = us[0].float()
            v32 = torch.empty_like(u32)
            for prec, ec in [("f16", 1), ("bf16", 1)]:
                for i in range(3):
                    P.apply_lp(u32, v32, precision=prec, ec=ec, stream=stream)
            torch.cuda.synchronize()
            del u32, v32
            print(f"profiled low-precision apply k={k} n={n}: 3 launches each", flush=True)
        for prec, ec, sm in (("f64", 0, "multiplicative"), ("f64", 0, "multiplicative_fused"),
                             ("f16", 1, "multiplicative")):
            Ps = Problem(3, 32, mg_precision=prec, error_correction=bool(ec), smoother=sm)
            amps, pqr = inputs.single_sine_modes()
            x, info = Ps.fgmres(Ps.rhs_sines(amps, pqr), rtol=1e-10)
            print(f"profiled solve k=3 n=32 {prec}{'_ec' if ec else ''} {sm}: "
                  f"{info['iterations']} iterations", flush=True)
            Ps.close()
        for kv in (5, 7):  # V(2,2) cycles of the vector-unit patch solves
            for prec in ("f64", "f32"):
                Pv = Problem(kv, 32, mg_precision=prec)
                bv = torch.from_numpy(inputs.uniform_vector(Pv.n_dofs(), 5)).to(dev)
                xv = torch.zeros_like(bv)
                for _ in range(2):
                    xv.zero_()
                    Pv.vcycle(xv, bv)
                torch.cuda.synchronize()
                print(f"profiled V-cycles k={kv} n=32 {prec}: 2", flush=True)
                Pv.close()
                del bv, xv
        for kv, nv in ((3, 64), (7, 32)):  # applies on trilinear cells
            Pm = Problem(kv, nv, n_levels=1)
            Pm.set_geometry(inputs.mesh_vertices(nv, "smooth", MAPPED_AMPLITUDE, seed=1))
            um = torch.from_numpy(inputs.uniform_vector(Pm.n_dofs(), 6)).to(dev)
            vm = torch.empty_like(um)
            for _ in range(3):
                Pm.apply(um, vm, stream=stream)
            torch.cuda.synchronize()
            print(f"profiled general-geometry apply k={kv} n={nv}: 3 launches", flush=True)
            Pm.close()
            del um, vm
        from paper_2407_09621_amd import Network
        Pt = Problem(3, 32)
        for loss in ("residual", "mse"):
            tr = Network(seed=1).train(Pt, n_chains=5, chain_length=4, crops_per_pair=8, crop=32,
                                       lr=1e-3, seed=2, loss=loss)
            print(f"profiled training k=3 n=32 ({loss} loss): {tr['steps']} pairs", flush=True)
        Pt.close()
        net = Network(seed=1)
        net.set_params(net.get_params()[0], 1.0)
        g = torch.rand((1, 128, 128, 128), device=dev, dtype=torch.float32)
        for _ in range(3):
            net.forward(g)
        torch.cuda.synchronize()
        print("profiled network forward: 3 x 128^3 grid", flush=True)
        del net, g
        # calibration: a plain device copy of exactly 2^27 bytes (read) + 2^27 (write)
        a = torch.empty(1 << 24, dtype=torch.float64, device=dev).uniform_()
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print("profiled copy: 5 launches of 134217728 bytes", flush=True)
        return

    # warm-up
    for _ in range(args.warmup):
        for k, n, P, nd, us, vs in probs:
            P.apply(us[0], vs[0], stream=stream)
    torch.cuda.synchronize()

    # per-degree kernel timing with events on the launch stream
    per_k = {}
    for k, n, P, nd, us, vs in probs:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 1)
        e0.record(stream)
        for i in range(reps):
            P.apply(us[i % ROTATE], vs[i % ROTATE], stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gdofs = nd / (ms * 1e-3) / 1e9
        per_k[f"k{k}_n{n}"] = {
            "ms_per_apply": round(ms, 5), "gdof_s": round(gdofs, 2),
            "hbm_gb_s": round(gdofs * BYTES_PER_DOF, 1),
            "hbm_frac": round(gdofs * BYTES_PER_DOF / HBM_PEAK_GBS, 4),
            "fp64_tflops_model": round(gdofs * flops_per_dof(k) / 1e3, 2),
            "fp64_frac_model": round(gdofs * flops_per_dof(k) / 1e3 / FP64_PEAK_TFLOPS, 4),
            "n_dofs": nd, "kernel": APPLY_KERNEL[f"k{k}_n{n}"]}

    # unrotated: the same (u, v) pair every launch (the L2/MALL may keep part
    # of the working set), and the measured HBM copy rate as a second peak
    for k, n, P, nd, us, vs in probs:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 1)
        P.apply(us[0], vs[0], stream=stream)
        e0.record(stream)
        for i in range(reps):
            P.apply(us[0], vs[0], stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        per_k[f"k{k}_n{n}"]["unrotated_gdof_s"] = round(nd / (ms * 1e-3) / 1e9, 2)
    copy_gb_s = measured_copy_rate(stream)
    for key in per_k:
        per_k[key]["hbm_frac_of_copy"] = round(per_k[key]["hbm_gb_s"] / copy_gb_s, 4)

    # the same apply on the FP64 vector units (the paper's CUDA-core
    # comparison, App. A) where the default runs on the matrix cores
    units = {}
    for k, n, P, nd, us, vs in probs:
        if k not in (3, 7):
            continue
        P.apply(us[0], vs[0], stream=stream, units="vector")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 1)
        e0.record(stream)
        for i in range(reps):
            P.apply(us[i % ROTATE], vs[i % ROTATE], stream=stream, units="vector")
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        mat = per_k[f"k{k}_n{n}"]
        units[f"k{k}_n{n}"] = {"vector_ms": round(ms, 5),
                               "vector_gdof_s": round(nd / (ms * 1e-3) / 1e9, 2),
                               "matrix_ms": mat["ms_per_apply"], "matrix_gdof_s": mat["gdof_s"],
                               "matrix_over_vector": round(ms / mat["ms_per_apply"], 3)}

    # the timed region: K steps, each one apply per degree
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for k, n, P, nd, us, vs in probs:
            P.apply(us[s % ROTATE], vs[s % ROTATE], stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_dofs = sum(p[3] for p in probs) * args.steps
    seconds = t1 - t0
    value = total_dofs / seconds / 1e9

    # dominant kernel = the degree with the largest share of the step
    dom = max(per_k.items(), key=lambda kv: kv[1]["ms_per_apply"])
    dk = dom[1]
    roofline = {"bound": "hbm", "achieved": dk["hbm_gb_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dk["hbm_gb_s"] / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(APPLY_KERNEL[dom[0]], dom[0]),
                "kernel": APPLY_KERNEL[dom[0]] + f" ({dom[0]})",
                "bytes_per_launch": int(dk["n_dofs"] * BYTES_PER_DOF)}

    progress(f"timed applies done: {value:.1f} GDoF/s")
    lp_rates = lp_apply_rates(probs, stream, max(10, args.steps // 4))
    patchwise = None if args.no_patchwise else run_patchwise(stream)
    for k, n, P, nd, us, vs in probs:
        P.close()
    del probs
    torch.cuda.empty_cache()

    solves = None if args.no_solve else run_solves(SOLVE_CONFIGS_QUICK if args.quick_solves
                                                   else SOLVE_CONFIGS)
    vcycles = None if args.no_solve else run_vcycles()
    comparisons = None if args.no_solve else run_comparisons()
    small_solve = None if args.no_solve else run_small_solve()
    batch = None
    if not args.no_batch:
        batch = {"large": run_batch(count=args.batch_count),
                 "small": run_batch(count=args.batch_count, edges=SMALL_EDGES)}
    learned = None if args.no_learned else run_learned(args.cnn_chains, args.cnn_loss)
    mapped = None if args.no_mapped else run_mapped(stream)

    line = {
        "metric": "SIPG apply GDoF/s (FP64/FP16 MFMA); FGMRES-MG solve time at equal L2 error",
        "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(seconds / max(args.steps, 1) * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 SIPG operator apply, unit cube, uniform Cartesian: "
                               "k=3 on 64^3 cells, k=5 on 40^3, k=7 on 32^3; u ~ U[-1,1] seeded; "
                               "one step = one apply per degree",
                   "parallelism": "single GPU"},
        "per_k": per_k, "roofline": roofline, "measured_copy_gb_s": round(copy_gb_s, 1),
        "cpu_baseline": cpu, "apply_units": units,
        "lowprec_apply": lp_rates, "patchwise_sweep": patchwise, "solves": solves,
        "vcycles": vcycles,
        "krylov_smoother_comparison": comparisons, "small_solve": small_solve,
        "batch": batch, "learned": learned,
        "general_geometry": mapped,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
