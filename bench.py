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
kernel on its own stream), the oracle's CPU rate on a bounded sample, and,
outside the timed region, the FP64 / mixed-precision FGMRES + multigrid
solve times, the batched uneven solves and the learned correction stage.
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
# HBM bytes per launch of the apply kernel as profiled (FETCH_SIZE x 2 +
# WRITE_SIZE x 1, profiles/apply_f64_k3n64_k5n40_k7n32.md); set an entry
# to None when the kernel changes until it is profiled again.
PROFILED_TRAFFIC = {"k3_n64": 314.1e6, "k5_n40": 274.1e6, "k7_n32": 327.3e6}
# the kernel each benchmark degree runs (FP64 apply)
APPLY_KERNEL = {"k3_n64": "apply_mfma4_kernel", "k5_n40": "apply_wave_kernel",
                "k7_n32": "apply_mfma8_kernel"}
ROTATE = 4


def flops_per_dof(k):
    """Model count: 7 sum-factorized N x N products per cell (14 N flop/DoF)
    plus face traces and expansions (48 flop/DoF)."""
    return 14 * (k + 1) + 48


def cpu_baseline():
    """The oracle's Kronecker-sum apply (numpy/scipy, FP64) on one apply of
    each degree at the full sizes."""
    import numpy as np
    from oracle import sipg as osipg
    from paper_2407_09621_amd import inputs
    total = 0
    t = 0.0
    for k, n in CONFIGS:
        u = inputs.uniform_vector(n ** 3 * (k + 1) ** 3, seed=2 + k)
        t0 = time.perf_counter()
        osipg.kron_apply(u, n, k)
        t += time.perf_counter() - t0
        total += u.size
    return {"value": total / t / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": "one FP64 apply at each of k=3 (64^3), k=5 (40^3), k=7 (32^3) "
                      "by the oracle's Kronecker-sum path (scipy.sparse, single-threaded); "
                      f"{t:.1f} s"}


SOLVE_CONFIGS = [(3, 64), (5, 32), (7, 32)]
SOLVE_CONFIGS_ALL = [(k, n) for k in (3, 5, 7) for n in (16, 32, 64)]
SOLVE_VARIANTS = [("f64", 0), ("f32", 0), ("f16", 0), ("f16", 1), ("bf16", 0), ("bf16", 1)]


def run_solves(configs):
    """FP64 FGMRES(30) + V(2,2) solves of the sine problem with the V-cycle in
    FP64, FP32, FP16 and BF16 (the latter two with and without error
    correction), outside the timed apply region: time to rtol 1e-10
    (after one warm-up solve that allocates the Krylov space), iterations,
    true residual, L2 error and the speed multiple over the FP64 solve."""
    import torch
    from paper_2407_09621_amd import Problem, inputs
    out = {}
    amps, pqr = inputs.single_sine_modes()
    for k, n in configs:
        row = {}
        for prec, ec in SOLVE_VARIANTS:
            P = Problem(k, n, mg_precision=prec, error_correction=bool(ec))
            b = P.rhs_sines(amps, pqr)
            x, info = P.fgmres(b, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False)
            x.zero_()
            torch.cuda.synchronize()
            x, info = P.fgmres(b, x=x, rtol=1e-10, max_iters=200, raise_on_nonconvergence=False)
            err = P.l2_error_sines(amps, pqr, x)
            row[prec + ("_ec" if ec else "")] = {
                "seconds": round(info["seconds"], 5), "iterations": info["iterations"],
                "rel_res_true": info["rel_res_true"], "l2_error": err, "status": info["status"]}
            P.close()
            del x, b
        base = row["f64"]
        for v in row.values():
            v["speedup_vs_f64"] = round(base["seconds"] / v["seconds"], 3)
            v["l2_within_1pct_of_f64"] = abs(v["l2_error"] - base["l2_error"]) <= 0.01 * base["l2_error"]
        out[f"k{k}_n{n}"] = row
        torch.cuda.empty_cache()
    return out


BATCH_SEED, BATCH_COUNT, BATCH_RESTART = 4, 64, 6
SMALL_EDGES = (4, 6, 8, 12)


def run_batch(count=BATCH_COUNT, seed=BATCH_SEED, restart=BATCH_RESTART,
              edges=(16, 24, 32, 48, 64)):
    """Batched uneven solves: `count` seeded problems (mesh edge in
    {16,24,32,48,64}, k in 2..7), right-hand sides from 4 seeded sine modes,
    FGMRES(restart) + FP64 V(2,2) to rtol 1e-10.  Times one batched solve
    with captured V-cycle graphs (after a warm-up solve that captures them),
    one batched solve without graphs, and the one-problem-at-a-time loop on
    the same handles.  Aggregate rate = sum over problems of DoFs x
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
                     ("eager", dict(use_graph=False)), ("sequential", dict(sequential=True))]:
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
        if name in ("graph", "sequential"):
            res[name]["l2_errors"] = [B.l2_error_sines(i, *modes[i], xs[i]) for i in range(count)]
        del xs
        torch.cuda.empty_cache()
    eg, es = res["graph"].pop("l2_errors"), res["sequential"].pop("l2_errors")
    out = {"problems": count, "seed": seed, "restart": restart,
           "total_dofs": int(sum(B.sizes)),
           "degrees": sorted({k for k, _ in pairs}), "edges": sorted({n for _, n in pairs}),
           "l2_max_rel_diff_vs_sequential": max(abs(a - b) / b for a, b in zip(eg, es)),
           "speedup_graph_vs_sequential": round(res["sequential"]["seconds"] / res["graph"]["seconds"], 3),
           "speedup_graph_vs_eager": round(res["eager"]["seconds"] / res["graph"]["seconds"], 3)}
    out.update({k: v for k, v in res.items() if k != "warmup"})
    B.close()
    del bs
    torch.cuda.empty_cache()
    return out


CNN_CHAINS = 500


def run_learned(chains=CNN_CHAINS):
    """Learned correction stage at k = 3 on 32^3 cells (128^3 grid): train
    on the GPU with 4 solver-made pairs per right-hand side (one Adam step on
    8 random 32^3 crops per pair), then solve held-out right-hand sides
    (4 sine modes, seeds 100000..100003) to rtol 1e-10 with and without the
    stage.  Also times the network forward on the full grid (FP16 matrix
    cores; 2 x 32 x 32 x 27 x 2 flop per point in each 32 -> 32 layer)."""
    import torch
    from paper_2407_09621_amd import Network, Problem, inputs
    k, n = 3, 32
    P = Problem(k, n)
    net = Network(seed=1)
    tr = net.train(P, n_chains=chains, chain_length=4, crops_per_pair=8, crop=32, lr=1e-3, seed=2)
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
            "training": {"pairs": tr["steps"], "crops_per_step": 8, "crop": 32, **tr},
            "solves": rows,
            "iterations_plain": [r["plain"]["iterations"] for r in rows],
            "iterations_learned": [r["learned"]["iterations"] for r in rows],
            "speedup_learned_vs_plain": round(tp / tl, 3),
            "forward_ms": round(ms, 4), "forward_tflops": round(fwd_flop / ms / 1e9, 1),
            "forward_frac_fp16_peak": round(fwd_flop / ms / 1e9 / FP16_PEAK_TFLOPS, 4)}


def lp_apply_rates(probs, stream, reps):
    """Reduced-precision applies (FP32 storage, 8 B/DoF) at the apply sizes."""
    import torch
    out = {}
    for k, n, P, nd, us, vs in probs:
        u32 = [u.float() for u in us[:2]]
        v32 = [torch.empty_like(u32[0]) for _ in range(2)]
        for prec, ec in [("f32", 0), ("f16", 0), ("f16", 1), ("bf16", 0), ("bf16", 1)]:
            P.apply_lp(u32[0], v32[0], precision=prec, ec=ec, stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(reps):
                P.apply_lp(u32[i % 2], v32[i % 2], precision=prec, ec=ec, stream=stream)
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
    ap.add_argument("--all-solves", action="store_true",
                    help="solve every degree 3/5/7 x 16^3/32^3/64^3 configuration")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve measurement")
    ap.add_argument("--batch-count", type=int, default=BATCH_COUNT,
                    help="problems in the batched-solve measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-stage measurement")
    ap.add_argument("--cnn-chains", type=int, default=CNN_CHAINS,
                    help="right-hand sides for the learned stage's training (4 pairs each)")
    ap.add_argument("--mode", choices=["bench", "profile"], default="bench",
                    help="profile: a few applies per degree and a plain copy of a known size "
                         "(for rocprofv3 kernel traces and HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

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
            u32 = us[0].float()
            v32 = torch.empty_like(u32)
            for prec, ec in [("f16", 1), ("bf16", 1)]:
                for i in range(3):
                    P.apply_lp(u32, v32, precision=prec, ec=ec, stream=stream)
            torch.cuda.synchronize()
            del u32, v32
            print(f"profiled low-precision apply k={k} n={n}: 3 launches each", flush=True)
        for prec, ec in (("f64", 0), ("f16", 1)):
            Ps = Problem(3, 32, mg_precision=prec, error_correction=bool(ec))
            amps, pqr = inputs.single_sine_modes()
            x, info = Ps.fgmres(Ps.rhs_sines(amps, pqr), rtol=1e-10)
            print(f"profiled solve k=3 n=32 {prec}{'_ec' if ec else ''}: "
                  f"{info['iterations']} iterations", flush=True)
            Ps.close()
        from paper_2407_09621_amd import Network
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
            "n_dofs": nd}

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
                "traffic": PROFILED_TRAFFIC.get(dom[0]),
                "kernel": APPLY_KERNEL[dom[0]] + f" ({dom[0]})",
                "bytes_per_launch": int(dk["n_dofs"] * BYTES_PER_DOF)}

    lp_rates = lp_apply_rates(probs, stream, max(10, args.steps // 4))
    for k, n, P, nd, us, vs in probs:
        P.close()
    del probs
    torch.cuda.empty_cache()

    solves = None if args.no_solve else run_solves(SOLVE_CONFIGS_ALL if args.all_solves
                                                   else SOLVE_CONFIGS)
    batch = None
    if not args.no_batch:
        batch = {"large": run_batch(count=args.batch_count),
                 "small": run_batch(count=args.batch_count, edges=SMALL_EDGES)}
    learned = None if args.no_learned else run_learned(args.cnn_chains)
    cpu = None if args.no_cpu else cpu_baseline()

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
        "per_k": per_k, "roofline": roofline, "cpu_baseline": cpu,
        "lowprec_apply": lp_rates, "solves": solves, "batch": batch, "learned": learned,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
