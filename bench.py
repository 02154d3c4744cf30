#!/usr/bin/env python3
"""Benchmark: H-LU factor seconds and H-LU preconditioned GMRES solves/sec to
a relative residual of 1e-8, FP32 H-LU vs FP64 H-LU, on one MI355X.

Workload (default): the Kuhn-split unit cube with 32^3 cubes (N = 220,256
interior-edge unknowns), A = K - kappa^2 M with kappa = 8, eta = 2, leaf 64,
truncation eps = 1e-3, right-hand sides b = A x* with x* uniform in [-1, 1]
(8 columns per seed, seeds 0..2), FP64 GMRES(50) to 1e-8.  Inputs are
synthetic and seeded; everything is resident in HBM before timing.

A step is one GMRES(50) solve of the workload's right-hand sides (8 columns
for each of the seeds 0, 1, 2: 24 columns, iterated together) with the
cached FP32 H-LU preconditioner (SpMV, H-solves, orthogonalisation, true
residual).  value = right-hand sides solved per second.  The FP32 and FP64
factorisations are timed separately (HIP events) and reported beside it,
with the same steps for the FP64 H-LU and for FP32 factors computed with
FP64 task arithmetic, and one solve of the same columns at kappa = 16.

Prints ONE JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=32)
    p.add_argument("--kappa", type=float, default=8.0)
    p.add_argument("--eps", type=float, default=1e-3)
    p.add_argument("--leaf", type=int, default=64)
    p.add_argument("--nrhs", type=int, default=8)
    p.add_argument("--restart", type=int, default=50)
    p.add_argument("--tol", type=float, default=1e-8)
    p.add_argument("--no-fp64", action="store_true",
                   help="skip the FP64 and FP32-storage/FP64-arithmetic H-LU comparisons")
    p.add_argument("--kappa2", type=float, default=16.0,
                   help="second wavenumber of the workload (near a cavity resonance at 32^3): one GMRES "
                        "call per precision, reported beside the timed steps (0: skip)")
    p.add_argument("--kappa2-max-iters", type=int, default=300)
    p.add_argument("--copy-probe-gib", type=float, default=0.0,
                   help="first run one plain device-to-device copy of this many GiB, whose HBM counter "
                        "readings calibrate those of the solve kernel under rocprofv3 --pmc")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--inverse", action="store_true",
                   help="H-matrix inverse by the Schulz iteration instead (--n, --kappa, --leaf, --inv-eps): "
                        "build B_H, then GMRES(50) with B_H and with the H-LU at the same eps on the same rhs")
    p.add_argument("--inv-eps", type=float, default=1e-2)
    p.add_argument("--inv-max-steps", type=int, default=40)
    p.add_argument("--factor-only", action="store_true",
                   help="only the FP32 factorisation of the workload, twice (the second timed), for counter "
                        "runs of the factor kernels")
    p.add_argument("--fit-margin", type=int, default=4,
                   help="after the timed runs, refit the rank capacities to the measured ranks plus this "
                        "margin (hlu_fit_ranks) and factor and solve once more in FP32 (-1: skip)")
    p.add_argument("--cpu-level", type=int, default=4,
                   help="cluster-tree level of the principal block the oracle sample factors")
    p.add_argument("--batch", action="store_true",
                   help="batched workload instead: 64 problems (8^3..24^3, kappa in [1, 10]) factored and "
                        "solved as one batch, against the same problems run one by one")
    p.add_argument("--table1", action="store_true",
                   help="Example 1 protocol of the paper instead (Table 1): GMRES iteration counts per refinement "
                        "level and kappa, beside the paper's")
    p.add_argument("--table1-levels", type=str, default="2,3,4,5",
                   help="refinement levels k (n = 2^(k-1) cubes per side)")
    p.add_argument("--table1-max-iters", type=int, default=500)
    p.add_argument("--batch-count", type=int, default=64)
    p.add_argument("--batch-leaves", type=str, default="32,48,64,96,128",
                   help="leaf sizes the autotuner measures per mesh size (one value: fixed leaf)")
    p.add_argument("--serve", action="store_true",
                   help="serving workload instead: Poisson arrivals of solve requests answered by hlu_server")
    p.add_argument("--serve-rate", type=float, default=20.0, help="arrivals per second")
    p.add_argument("--serve-count", type=int, default=400)
    p.add_argument("--serve-sizes", type=str, default="8,12,16,20,24")
    p.add_argument("--serve-workers", type=int, default=4)
    p.add_argument("--serve-budget-gb", type=float, default=200.0)
    p.add_argument("--serve-refine-iters", type=int, default=100,
                   help="first-try GMRES iterations before a cached factor is refined (0: never refine)")
    p.add_argument("--serve-warm", action="store_true",
                   help="factor every (n, kappa) of the request list before the timed arrivals (steady state)")
    p.add_argument("--serve-rates", type=str, default="",
                   help="comma list of arrival rates: one run per rate on one server (cache kept between "
                        "rates), a JSON line per rate and a summary line (replaces --serve-rate)")
    p.add_argument("--serve-window", type=float, default=10.0,
                   help="seconds of arrivals per rate of --serve-rates (at most --serve-count requests)")
    p.add_argument("--serve-kappas", type=str, default="",
                   help="comma list of the wavenumbers requests draw from (default 1..16)")
    p.add_argument("--serve-max-rank", type=int, default=32, help="rank capacity of the served H-LUs")
    p.add_argument("--batch-max-rank", type=int, default=32,
                   help="rank capacity per low-rank block in the batched workload")
    return p.parse_args()


# HBM traffic of one chain-solve launch (24 columns, 32^3, FP32 factors)
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, each scaled by the reading
# of a plain copy kernel of known size (FETCH 2.0, WRITE 1.0), the mean over
# the 9 launches of the timed step; valid only for the sources it was
# measured on (SHA-256 of SOLVE_SOURCES), and reported as null otherwise.
SOLVE_TRAFFIC = {"sha256": "962285794c6adf35fc3fe5c8cd60ea0b37d255d57eae3348c53c297d0b2338cf", "columns": 24,
                 "bytes_per_launch": 17764875897, "fetch_bytes": 9583219040, "write_bytes": 8181656856}
SOLVE_SOURCES = ("paper_2211_11303_amd/csrc/kernels_chain.hip", "paper_2211_11303_amd/csrc/chain_sched.cpp",
                 "paper_2211_11303_amd/csrc/chain_sched.h")


def solve_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in SOLVE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def event_time(fn, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = fn()
    e1.record(stream)
    e1.synchronize()
    return out, e0.elapsed_time(e1) / 1e3


def oracle_errors(args, x, X):
    """Per-solve ||x - x_oracle|| / ||x_oracle|| against the oracle's
    solutions of the same right-hand sides (stored by
    tests/golden/make_oracle_cfg2.py, oracle only), when the workload is the
    one they were computed for; else None."""
    import numpy as np
    tag = os.path.join(ROOT, "tests", "golden", f"oracle_cfg2_k{int(args.kappa)}")
    if not (args.n == 32 and args.leaf == 64 and args.eps == 1e-3 and args.restart == 50 and args.tol == 1e-8
            and args.nrhs == 8 and float(args.kappa) == int(args.kappa) and os.path.exists(tag + "_x.npz")):
        return None
    z = np.load(tag + "_x.npz")
    with open(tag + ".json") as f:
        g = json.load(f)
    xs = x.cpu().numpy()
    Xs = X.cpu().numpy()
    out = []
    for k in range(len(z["seeds"])):
        row = int(z["seeds"][k]) * args.nrhs + int(z["cols"][k])   # step block: seeds 0..2 x nrhs columns
        xo = Xs[row] + z["scale"][k] * z["q"][k].astype(np.float64)
        out.append(float(np.linalg.norm(xs[row] - xo) / np.linalg.norm(xo)))
    return {"per_solve": out, "max": max(out), "oracle_err_vs_xstar_max": max(r["err"] for r in g["solves"]),
            "oracle_iters": sorted({r["iters"] for r in g["solves"]}), "oracle_factor_error": g["factor_error"]}


def oracle_full_size(args):
    """The oracle's own timings on the whole workload, as stored with its
    results by tests/golden/make_oracle_cfg2.py (one core, one BLAS thread,
    run once on the build host, not on the GPU host): factor seconds and
    GMRES seconds per right-hand side."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_cfg2_k{int(args.kappa)}.json")
    if not (args.n == 32 and args.leaf == 64 and args.eps == 1e-3 and os.path.exists(path)):
        return None
    with open(path) as f:
        g = json.load(f)
    per = [r["seconds"] for r in g["solves"]]
    return {"factor_s": g["oracle_factor_s"], "solve_s_mean": sum(per) / len(per),
            "solves_per_s": len(per) / sum(per), "threads": g["oracle_threads"], "right_hand_sides": len(per),
            "where": "build host (not the GPU host), stored with the oracle results"}


def per_sweep_rates(A, H, B, args):
    """Solves/s with 1 and 8 right-hand sides per GMRES call (one call each,
    columns 0 and 0..7 of the workload), and the persistent H-solve launch
    time at 1, 8 and all columns (HIP events on the launch stream)."""
    import torch
    from paper_2211_11303_amd import hlu
    out = {}
    for c in (1, 8):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = hlu.gmres_solve(A, B[:c].contiguous(), H, restart=args.restart, tol=args.tol, max_iters=1000,
                                   raise_on_fail=False)
        torch.cuda.synchronize()
        out[f"solves_per_s_{c}rhs"] = c / (time.perf_counter() - t0)
        out[f"iters_{c}rhs"] = max(i["iters"] for i in infos)
    for c in (1, 8, B.shape[0]):
        v = B[:c].contiguous()
        H.hlu_solve(v)
        H.hlu_set_timing(True)
        s0 = H.hlu_get_stats()
        for _ in range(3):
            H.hlu_solve(v)
        torch.cuda.synchronize()
        s1 = H.hlu_get_stats()
        H.hlu_set_timing(False)
        out[f"hsolve_launch_ms_{c}rhs"] = (s1["solve_kernel_ms"] - s0["solve_kernel_ms"]) / max(
            1, s1["solve_launches"] - s0["solve_launches"])
    return out


def cpu_baseline(n, kappa, leaf, eps, restart, tol, level, N_full, iters_full, nrhs=24):
    """The oracle (FP64, plain Python/NumPy, one BLAS thread) on a bounded
    sample of the same workload: the principal diagonal block of A on one
    cluster of the cluster tree at `level`, factored, then solved for nrhs
    right-hand sides one at a time.  The solve time per GMRES iteration per
    unknown of the sample is scaled to the full problem (N_full unknowns,
    iters_full iterations per right-hand side, the FP64 count measured on
    the device) to give the oracle's solves/s on the workload."""
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    import numpy as np
    from oracle.assemble import Discretisation
    from oracle.cluster import Structure
    from oracle.hmatrix import HLU
    from oracle.krylov import gmres
    from paper_2211_11303_amd.inputs import exact_solution_cols

    d = Discretisation(n, kappa)
    mid = d.mesh.midpoints2()
    full = Structure(mid, leaf, 2.0)
    c = next(c for c in full.clusters if c.level == level)
    idx = np.sort(full.perm[c.begin:c.end])
    A = d.A[idx][:, idx].tocsr()
    s = Structure(mid[idx], leaf, 2.0)
    t0 = time.perf_counter()
    h = HLU(s, A, eps).factor()
    t_factor = time.perf_counter() - t0
    X = exact_solution_cols(len(idx), nrhs, seed=0)
    t1 = time.perf_counter()
    iters = 0
    for x in X:
        _, info = gmres(A, A @ x, h.solve, restart=restart, tol=tol, max_iters=500)
        iters += info["iters"]
    t_solve = time.perf_counter() - t1
    per_iter_unknown = t_solve / (iters * len(idx))
    return {
        "value": 1.0 / (per_iter_unknown * N_full * iters_full), "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"principal block of the {n}^3 matrix on one level-{level} cluster "
                   f"({len(idx)} of {d.N} unknowns, kappa {kappa:g}, leaf {leaf}, eps {eps:g}): "
                   f"oracle H-LU factor {t_factor:.1f} s, then GMRES({restart}) to {tol:g} on {nrhs} "
                   f"right-hand sides one at a time ({iters} iterations, {t_solve:.2f} s), 1 BLAS thread; "
                   f"value = that solve time per iteration per unknown scaled to {N_full} unknowns and "
                   f"{iters_full} iterations per right-hand side"),
        "factor_s": t_factor, "solve_s": t_solve, "unknowns": int(len(idx)), "sample_iters": iters,
        "sample_solves_per_s": nrhs / t_solve,
    }


def batch_main(args):
    """Batched workload: problems (n, kappa) from inputs.batch_problems
    (default_rng(7)), FP32 H-LU (eps 1e-3, rank capacity 32), FP64 GMRES(50)
    to 1e-8 with one right-hand side each (x* seed = problem index).  Timed:
    (a) one by one -- hlu_factor + gmres_solve per problem; (b) as one batch
    -- hlu_factor_batch + gmres_solve_batch.  Structures are planned once
    per mesh size before either timed region (host work shared by both)."""
    import numpy as np
    import torch
    from paper_2211_11303_amd import hlu, inputs

    torch.cuda.set_device(0)
    eps, mr, prec = 1e-3, args.batch_max_rank, "fp32"
    probs = inputs.batch_problems(args.batch_count, seed=7)
    # leaf size per mesh size, measured (factor + one GMRES solve at the
    # middle of the kappa range) before either timed region
    cands = tuple(int(v) for v in args.batch_leaves.split(","))
    leaf_by_n, tune_times = {}, {}
    t = time.perf_counter()
    for n in sorted({n for n, _ in probs}):
        if len(cands) == 1:
            leaf_by_n[n] = cands[0]
            continue
        best, secs = hlu.hlu_autotune_leaf(n, 5.5, leaves=cands, eps=eps, max_rank=mr, prec=prec,
                                           restart=args.restart, tol=args.tol)
        leaf_by_n[n], tune_times[n] = best, secs
        log(f"autotune {n}^3: leaf {best} (" + ", ".join(f"{l}: {s:.3f}s" for l, s in zip(cands, secs)) + ")")
    autotune_s = time.perf_counter() - t
    t = time.perf_counter()
    data = [(n, kappa) + tuple(hlu.hlu_kuhn_assemble(n, kappa)) for n, kappa in probs]
    protos = {}
    for n, kappa, rp, ci, va, mid in data:
        if n not in protos:
            log(f"planning {n}^3")
            protos[n] = hlu.HLU(rp, ci, va, mid, 2.0, leaf_by_n[n])
            protos[n].hlu_workspace_bytes(eps, mr, prec)
    mats = [hlu.SpMat(rp, ci, va) for _, _, rp, ci, va, _ in data]
    xs = [torch.tensor(inputs.exact_solution_cols(A.n, 1, seed=p), device="cuda") for p, A in enumerate(mats)]
    bs = [A.hlu_spmv(x) for A, x in zip(mats, xs)]
    # device copies of the plans (first factorisation of each structure)
    for n, H in protos.items():
        H.hlu_factor(eps, mr, prec, allow_overflow=True)
        H.work = None
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t

    def handles():
        return [hlu.HLU(rp, ci, va, share=protos[n]) for n, _, rp, ci, va, _ in data]

    log("one by one")
    seq = handles()
    iters_seq, relres_seq = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, H in enumerate(seq):
        H.hlu_factor(eps, mr, prec, allow_overflow=True)
        x, info = hlu.gmres_solve(mats[p], bs[p], H, restart=args.restart, tol=args.tol, max_iters=1000,
                                  raise_on_fail=False)
        iters_seq.append(info[0]["iters"])
        relres_seq.append(info[0]["relres"])
        seq[p] = None   # frees the workspace and solve buffers
    torch.cuda.synchronize()
    T_seq = time.perf_counter() - t0

    log("batched")
    members = handles()
    t1 = time.perf_counter()
    B = hlu.HLUBatch(members, eps, max_rank=mr, prec=prec, max_rhs=1)
    B.hlu_batch_bind_workspace()
    bstack = B.stack(bs)
    torch.cuda.synchronize()
    batch_setup_s = time.perf_counter() - t1
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    _, tf = event_time(lambda: B.hlu_factor_batch(allow_overflow=True), stream)
    xb, infos = B.gmres_solve_batch(bstack, restart=args.restart, tol=args.tol, max_iters=1000,
                                    raise_on_fail=False)
    torch.cuda.synchronize()
    T_bat = time.perf_counter() - t0
    xparts = B.unstack(xb)
    errs = [((xp - x).norm() / x.norm()).item() for xp, x in zip(xparts, xs)]
    iters_b = [i[0]["iters"] for i in infos]
    caps = max(m.hlu_get_stats()["capped_blocks"] for m in members)
    line = {
        "metric": "batched H-LU + GMRES: problems solved per second (factor + GMRES(50) to 1e-8, 1 rhs each)",
        "value": args.batch_count / T_bat,
        "unit": "problems/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32-hlu+f64-gmres",
        "data": "synthetic",
        "config": {"workload": f"{args.batch_count} Kuhn-cube problems, n in {{8,12,16,20,24}} and kappa in "
                               f"[1,10] from default_rng(7); eta=2, "
                               + (f"leaf autotuned per mesh size from {{{args.batch_leaves}}}" if len(cands) > 1
                                  else f"leaf {cands[0]}")
                               + f", eps={eps:g}, rank capacity {mr}; GMRES({args.restart}) to {args.tol:g}, 1 rhs each",
                   "count": args.batch_count, "N_total": B.n_total, "leaf_by_n": leaf_by_n},
        "autotune_s": autotune_s,
        "autotune_device_s": {n: dict(zip(cands, v)) for n, v in tune_times.items()},
        "one_by_one_problems_per_s": args.batch_count / T_seq,
        "speedup_vs_one_by_one": T_seq / T_bat,
        "batched_s": T_bat,
        "one_by_one_s": T_seq,
        "batched_factor_s": tf,
        "batch_factor_waves": B.factor_waves,
        "sum_member_factor_waves": sum(protos[n].hlu_get_stats()["factor_waves"] for n, *_ in data),
        "iters_batched": [min(iters_b), max(iters_b)],
        "iters_equal_one_by_one": iters_b == iters_seq,
        "relres_max": max(i[0]["relres"] for i in infos),
        "converged": all(i[0]["converged"] for i in infos),
        "err_vs_xstar_max": max(errs),
        "capped_blocks": caps,
        "workspace_gb": B.hlu_batch_workspace_bytes() / 1e9,
        "setup_s": setup_s,
        "batch_setup_s": batch_setup_s,
    }
    print(json.dumps(line), flush=True)


def serve_main(args):
    """Serving workload: requests from inputs.serving_requests (Poisson
    arrivals at --serve-rate, or at each rate of --serve-rates; n from
    --serve-sizes, kappa from --serve-kappas (default 1..16), 1..32
    right-hand sides, x* seed = 1000 + request index), answered by
    hlu_server (FP32 H-LU eps 1e-3, rank capacity --serve-max-rank, FP64
    GMRES(50) to 1e-8, factor cache per (n, kappa), continuous batching,
    refinement of a factor whose columns miss tol within
    --serve-refine-iters iterations).  Latency is measured by the server
    from submission to completion (host wall clock)."""
    import numpy as np
    from paper_2211_11303_amd import hlu, inputs

    sizes = tuple(int(v) for v in args.serve_sizes.split(","))
    kappas = (tuple(float(v) for v in args.serve_kappas.split(",")) if args.serve_kappas
              else tuple(float(k) for k in range(1, 17)))
    rates = [float(v) for v in args.serve_rates.split(",")] if args.serve_rates else [args.serve_rate]
    runs = []
    for i, rate in enumerate(rates):
        count = args.serve_count if not args.serve_rates else max(10, min(args.serve_count,
                                                                          int(round(rate * args.serve_window))))
        runs.append((rate, inputs.serving_requests(count, rate, seed=11 + i, sizes=sizes, kappas=kappas)))
    t = time.perf_counter()
    srv = hlu.Server(workers=args.serve_workers, max_batch_rhs=32, hbm_budget=int(args.serve_budget_gb * (1 << 30)),
                     eta=2.0, leaf=args.leaf, eps=1e-3, max_rank=args.serve_max_rank, prec="fp32",
                     restart=args.restart, max_iters=1000, tol=args.tol, refine_iters=args.serve_refine_iters,
                     max_refines=2, refine_eps_factor=0.1)
    for n in sizes:
        log(f"planning {n}^3")
        srv.hlu_server_prepare(n)
    if args.serve_warm:
        keys = sorted({(r["n"], r["kappa"]) for _, reqs in runs for r in reqs})
        log(f"warming the factor cache: {len(keys)} (n, kappa) pairs")
        for i, (n, k) in enumerate(keys):
            N, _ = hlu.hlu_kuhn_sizes(n)
            srv.hlu_server_wait(srv.hlu_server_submit(n, k, np.zeros((1, N))), raise_on_fail=False)
            if i % 10 == 9:
                log(f"warmed {i + 1}")
    setup_s = time.perf_counter() - t
    mats = {}
    lines = []
    for rate, reqs in runs:
        lines.append(serve_rate(args, srv, rate, reqs, sizes, kappas, mats, setup_s))
        print(json.dumps(lines[-1]), flush=True)
    srv.close()
    if len(lines) > 1:
        table = [{k: l[k] for k in ("rate", "requests", "value", "requests_per_s", "p50_latency_s", "p99_latency_s",
                                    "p50_queue_s", "not_converged", "cache_hit_rate")} for l in lines]
        summary = dict(lines[0])
        summary.update({"metric": "H-LU preconditioned GMRES serving: p50/p99 request latency and solves/s per "
                                  "arrival rate",
                        "value": max(l["value"] for l in lines), "rates": table})
        summary["config"] = dict(lines[0]["config"], rate=None, rates=rates,
                                 workload=lines[0]["config"]["workload"].replace(
                                     f"at {rates[0]:g}/s", "at " + ",".join(f"{r:g}" for r in rates) + "/s"))
        print(json.dumps(summary), flush=True)


def serve_rate(args, srv, rate, reqs, sizes, kappas, mats, setup_s):
    """One timed run of Poisson arrivals `reqs` on the server; its JSON line."""
    import numpy as np
    import scipy.sparse as sp
    from paper_2211_11303_amd import hlu, inputs
    for r in reqs:
        key = (r["n"], r["kappa"])
        if key not in mats:
            rp, ci, va, _ = hlu.hlu_kuhn_assemble(r["n"], r["kappa"])
            mats[key] = sp.csr_matrix((va, ci, rp), shape=(len(rp) - 1, len(rp) - 1))
    rhs = []
    for r in reqs:
        A = mats[(r["n"], r["kappa"])]
        xs = inputs.exact_solution_cols(A.shape[0], r["nrhs"], seed=r["seed"])
        rhs.append((xs, np.ascontiguousarray((A @ xs.T).T)))
    st0 = srv.hlu_server_get_stats()
    log(f"serving {len(reqs)} requests at {rate}/s")
    tickets = []
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        delay = t0 + r["t"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.hlu_server_submit(r["n"], r["kappa"], rhs[i][1]))
        if i % 100 == 99:
            log(f"submitted {i + 1}")
    lat, que, errs, rel, iters, failed, failed_req = [], [], [], [], [], 0, []
    for i, tk in enumerate(tickets):
        x, infos, q, l = srv.hlu_server_wait(tk, raise_on_fail=False)
        lat.append(l)
        que.append(q)
        if not all(f["converged"] for f in infos):
            failed += 1
            failed_req.append({"n": reqs[i]["n"], "kappa": reqs[i]["kappa"], "nrhs": reqs[i]["nrhs"],
                               "iters": max(f["iters"] for f in infos), "relres": max(f["relres"] for f in infos)})
        xs = rhs[i][0]
        errs.append(float(np.max(np.linalg.norm(x - xs, axis=1) / np.linalg.norm(xs, axis=1))))
        rel.append(max(f["relres"] for f in infos))
        iters += [f["iters"] for f in infos]
        if i % 100 == 99:
            log(f"answered {i + 1}")
    T = time.perf_counter() - t0
    st = srv.hlu_server_get_stats()
    nrhs_total = sum(r["nrhs"] for r in reqs)
    lat = np.asarray(lat)
    ktxt = "1..16" if kappas == tuple(float(k) for k in range(1, 17)) else ",".join(f"{k:g}" for k in kappas)
    return {
        "metric": "H-LU preconditioned GMRES serving: p50/p99 request latency and solves/s",
        "value": nrhs_total / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32-hlu+f64-gmres",
        "data": "synthetic",
        "config": {"workload": f"{len(reqs)} Poisson requests at {rate:g}/s (default_rng), n in "
                               f"{list(sizes)}, kappa in {ktxt}, 1..32 rhs; FP32 H-LU eps 1e-3 rank capacity "
                               f"{args.serve_max_rank}, GMRES({args.restart}) to {args.tol:g}, refinement after "
                               f"{args.serve_refine_iters} iterations (eps x 0.1, at most twice); "
                               f"{args.serve_workers} workers, budget {args.serve_budget_gb:g} GB"
                               + ("; cache warmed" if args.serve_warm else ""),
                   "requests": len(reqs), "rate": rate, "sizes": list(sizes), "kappas": list(kappas)},
        "rate": rate,
        "requests": len(reqs),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_s": float(np.percentile(que, 50)),
        "requests_per_s": len(reqs) / T,
        "wall_s": T,
        "rhs_total": nrhs_total,
        "not_converged": failed,
        "not_converged_requests": failed_req[:10],
        "refine_iters": args.serve_refine_iters,
        "relres_max": max(rel),
        "err_vs_xstar_max": max(errs),
        "iters": [min(iters), max(iters)],
        "cache_hit_rate": (st["cache_hits"] - st0["cache_hits"]) / max(1, st["gmres_calls"] - st0["gmres_calls"]),
        "warm_cache": bool(args.serve_warm),
        "server": st,
        "peak_gb": st["peak_bytes"] / 1e9,
        "setup_s": setup_s,
    }


# Table 1 of the paper: GMRES iterations for Example 1 per refinement level k
# (rows) and kappa in {25, 100, 225, 400, 625, 900} (columns); None: ">3000"
PAPER_TABLE1 = {2: [1, 1, 1, 1, 1, 1], 3: [2, 2, 2, 2, 2, 2], 4: [2, 4, 5, 5, 4, 3], 5: [3, 4, 8, 9, 11, None],
                6: [3, 6, 20, 4, 48, 25], 7: [4, 5, 7, 19, 46, 93]}
PAPER_KAPPAS = [25.0, 100.0, 225.0, 400.0, 625.0, 900.0]


def table1_main(args):
    """Example 1 of the paper (Sec. 4, Table 1) with its protocol: the unit
    cube refined k times (here the Kuhn cube with n = 2^(k-1) cubes per side),
    J_S = (0, 0, 1), b_j = <J_S, Phi_j>, the paper's kappa multiplying the
    mass term (A = K - kappa M, so our wavenumber is sqrt(kappa)), GMRES
    restarted after 100 iterations, stopped at relative residual 1e-5.  The
    preconditioner is our FP64 H-LU at --eps and --leaf; the paper's rank r is
    not stated, so the counts are compared in trend, not value."""
    import math
    import torch
    from paper_2211_11303_amd import hlu

    torch.cuda.set_device(0)
    levels = [int(v) for v in args.table1_levels.split(",")]
    rows = []
    overflow = []   # cells whose eps-ranks exceeded the 64-column block capacity
    for k in levels:
        n = 2 ** (k - 1)
        rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, 1.0)
        proto = hlu.HLU(rp, ci, va, mid, 2.0, args.leaf)
        b = torch.tensor(hlu.hlu_kuhn_load(n, (0.0, 0.0, 1.0)), device="cuda").reshape(1, -1)
        its = []
        for kp in PAPER_KAPPAS:
            kappa = math.sqrt(kp)
            rp, ci, va, _ = hlu.hlu_kuhn_assemble(n, kappa)
            A = hlu.SpMat(rp, ci, va)
            H = hlu.HLU(rp, ci, va, share=proto)
            log(f"k={k} (n={n}) kappa={kp:g}: factor")
            H.hlu_factor(args.eps, prec="fp64", allow_overflow=True)
            capped = H.hlu_get_stats()["capped_blocks"]
            x, info = hlu.gmres_solve(A, b, H, restart=100, tol=1e-5, max_iters=args.table1_max_iters,
                                      raise_on_fail=False)
            its.append(info[0]["iters"] if info[0]["converged"] else None)
            if capped:
                overflow.append({"k": k, "kappa": kp, "capped_blocks": int(capped)})
            log(f"k={k} (n={n}, N={A.n}) kappa={kp:g}: iters {info[0]['iters']} converged {info[0]['converged']} "
                f"relres {info[0]['relres']:.2e} capped blocks {capped}")
            del H
        rows.append({"k": k, "n": n, "N": int(len(rp) - 1), "iters": its, "paper": PAPER_TABLE1.get(k)})
    line = {
        "metric": "Example 1 (Table 1 protocol): preconditioned GMRES iterations to 1e-5",
        "unit": "iterations", "n_gpus": 1, "dtype": "f64-hlu+f64-gmres", "data": "synthetic",
        "config": {"workload": f"Kuhn unit cube, n = 2^(k-1), J_S = (0,0,1), paper kappa in {PAPER_KAPPAS} "
                               f"(A = K - kappa M), GMRES(100) to 1e-5, FP64 H-LU eps {args.eps:g}, leaf "
                               f"{args.leaf}, eta 2; None = not converged within {args.table1_max_iters}",
                   "kappas": PAPER_KAPPAS},
        "rows": rows,
        "rank_overflow": overflow,
    }
    print(json.dumps(line), flush=True)


def inverse_main(args, stream):
    """--inverse: the Schulz H-inverse B_H (hlu_inverse, FP64, probe of 8
    standard normal columns) of the workload's matrix to its truncation
    floor or --inv-max-steps, then GMRES(restart) to tol on 8 right-hand
    sides preconditioned by B_H, and the same with the H-LU at the same eps."""
    import torch
    from paper_2211_11303_amd import hlu, inputs
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(args.n, args.kappa)
    A = hlu.SpMat(rp, ci, va)
    N = A.n
    Hi = hlu.HLU(rp, ci, va, mid, eta=2.0, leaf=args.leaf)
    probe = torch.tensor(inputs.probe_block(N, 8), device="cuda")   # (8, N), natural order
    X = torch.tensor(inputs.exact_solution_cols(N, 8, seed=0), device="cuda")
    B = A.hlu_spmv(X)
    log(f"Schulz inverse n={args.n} eps {args.inv_eps:g}")
    info, t_inv = event_time(lambda: Hi.hlu_inverse(probe, args.inv_eps, prec="fp64", tol=1e-12,
                                                     max_iters=args.inv_max_steps), stream)
    sti = Hi.hlu_get_stats()
    out = {}
    for name, H in (("inverse", Hi), ("hlu", None)):
        if H is None:
            H = hlu.HLU(rp, ci, va, mid, eta=2.0, leaf=args.leaf)
            H.hlu_factor(args.inv_eps, prec="fp64", allow_overflow=True)
            _, tf = event_time(lambda: H.hlu_factor(args.inv_eps, prec="fp64", allow_overflow=True), stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, infos = hlu.gmres_solve(A, B, H, restart=args.restart, tol=args.tol, max_iters=1000, raise_on_fail=False)
        torch.cuda.synchronize()
        T = time.perf_counter() - t
        out[name] = {"gmres_iters": sorted({i["iters"] for i in infos}),
                     "converged": all(i["converged"] for i in infos), "solves_per_s": X.shape[0] / T,
                     "err_vs_xstar_max": ((x - X).norm(dim=1) / X.norm(dim=1)).max().item()}
        if name == "hlu":
            out[name]["factor_s"] = tf
    line = {"metric": "Schulz H-inverse B_H: build time and GMRES(50) solves/s with B_H (beside the H-LU)",
            "value": out["inverse"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"kuhn-cube-{args.n}^3 Nedelec (N={N}), kappa={args.kappa:g}, eta=2, "
                                   f"leaf={args.leaf}, eps={args.inv_eps:g}, Schulz to its floor (at most "
                                   f"{args.inv_max_steps} steps), GMRES({args.restart}) to {args.tol:g}, 8 rhs",
                       "n": args.n, "N": N},
            "inverse_s": t_inv, "schulz_steps": info["iters"], "residual0": info["residual0"],
            "residual": info["residual"], "capped_truncations": sti["capped_blocks"],
            "max_rank": sti["max_rank"], "mean_rank": sti["mean_rank"], **out}
    print(json.dumps(line), flush=True)


def factor_only(args, stream):
    """--factor-only: the FP32 factorisation of the workload twice (the first
    uploads the plans); a JSON line with the second one's time and flops."""
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(args.n, args.kappa)
    H = hlu.HLU(rp, ci, va, mid, eta=2.0, leaf=args.leaf)
    H.hlu_factor(args.eps, prec="fp32", allow_overflow=True)
    _, tf = event_time(lambda: H.hlu_factor(args.eps, prec="fp32", allow_overflow=True), stream)
    st = H.hlu_get_stats()
    print(json.dumps({"metric": "H-LU factorisation time (FP32)", "value": tf, "unit": "s", "n_gpus": 1,
                      "higher_is_better": False, "dtype": "f32-hlu", "data": "synthetic",
                      "config": {"workload": f"kuhn-cube-{args.n}^3 Nedelec, kappa={args.kappa:g}, eta=2, "
                                             f"leaf={args.leaf}, eps={args.eps:g}", "n": args.n},
                      "factor_flops": st["factor_flops"],
                      "factor_flops_by_kind": {k: st["factor_flops_" + k] for k in ("getrf", "tri", "gemm",
                                                                                    "trunc")},
                      "max_rank": st["max_rank"], "mean_rank": st["mean_rank"]}), flush=True)


def fitted_capacity(args, H, A, B, r32, stream):
    """Rank capacities fitted to the ranks the last factorisation asked for
    (hlu_fit_ranks, margin --fit-margin), then the FP32 factorisation (timed)
    and one GMRES call on the step's block again: workspace and device bytes
    against the uniform capacity, and whether the solutions are those of the
    uniform-capacity run bit for bit (they are when no capacity is cut)."""
    import torch
    from paper_2211_11303_amd import hlu
    ws_u = H.hlu_workspace_bytes(args.eps, prec="fp32")
    dev_u = H.hlu_device_bytes(args.eps, prec="fp32")
    cap_u = H.hlu_get_stats()["rank_capacity_entries"]
    log("fp32: factorisation with the uniform capacity, for the ranks it asks for")
    H.hlu_factor(args.eps, prec="fp32", allow_overflow=True)
    fit_s, refits = 0.0, 0
    while True:
        log("fitting the rank capacities to the last factorisation")
        t = time.perf_counter()
        ws_f = H.hlu_fit_ranks(args.eps, margin=args.fit_margin, prec="fp32")
        fit_s += time.perf_counter() - t
        torch.cuda.empty_cache()
        H.hlu_factor(args.eps, prec="fp32", allow_overflow=True)
        if H.hlu_get_stats()["capped_blocks"] == 0 or refits == 2:
            break
        refits += 1   # a block asked for more than its fitted capacity: fit again to these ranks
    _, tf = event_time(lambda: H.hlu_factor(args.eps, prec="fp32", allow_overflow=True), stream)
    st = H.hlu_get_stats()
    dev_f = H.hlu_device_bytes(args.eps, prec="fp32")
    torch.cuda.synchronize()
    t = time.perf_counter()
    x, infos = hlu.gmres_solve(A, B, H, restart=args.restart, tol=args.tol, max_iters=1000, raise_on_fail=False)
    torch.cuda.synchronize()
    T = time.perf_counter() - t
    out = {"margin": args.fit_margin, "refits": refits, "refit_plan_s": fit_s, "factor_s": tf,
           "workspace_gb_uniform": ws_u / 1e9, "workspace_gb": ws_f / 1e9,
           "device_gb_uniform": dev_u / 1e9, "device_gb": dev_f / 1e9,
           "rank_capacity_entries_uniform": cap_u, "rank_capacity_entries": st["rank_capacity_entries"],
           "capped_blocks": st["capped_blocks"], "iters": sorted({i["iters"] for i in infos}),
           "solves_per_s": x.shape[0] / T,
           "same_solutions_as_uniform": bool(torch.equal(x, r32["x0"]))}
    log(f"fitted capacities: workspace {ws_u / 1e9:.1f} -> {ws_f / 1e9:.1f} GB, factor {tf:.2f}s, "
        f"same solutions {out['same_solutions_as_uniform']}")
    H.hlu_fit_ranks(args.eps, margin=-1, prec="fp32")
    return out


def second_kappa(args, H1, Xs, stream):
    """The same mesh, structure and x* columns at kappa = args.kappa2 (near
    the cavity eigenvalue 26 pi^2 at kappa = 16): one factorisation (timed
    after a first one) and one GMRES call, capped at --kappa2-max-iters
    iterations, per precision, and for FP32 once more at eps / 10;
    reported, not part of the timed steps."""
    import torch
    from paper_2211_11303_amd import hlu
    rp, ci, va, _ = hlu.hlu_kuhn_assemble(args.n, args.kappa2)
    A2 = hlu.SpMat(rp, ci, va)
    H2 = hlu.HLU(rp, ci, va, share=H1)
    B2 = A2.hlu_spmv(Xs)
    out = {"kappa": args.kappa2, "max_iters": args.kappa2_max_iters}
    runs = [("fp32", args.eps)] if args.no_fp64 else [("fp32", args.eps), ("fp64", args.eps),
                                                      ("fp32", args.eps / 10)]
    for prec, eps in runs:
        key = prec if eps == args.eps else f"{prec}_eps{eps:g}"
        log(f"kappa {args.kappa2:g} {prec} eps {eps:g}: factorisations")
        H2.hlu_factor(eps, prec=prec, allow_overflow=True)
        _, tf = event_time(lambda: H2.hlu_factor(eps, prec=prec, allow_overflow=True), stream)
        log(f"kappa {args.kappa2:g} {prec} eps {eps:g}: factor {tf:.2f}s; GMRES (at most "
            f"{args.kappa2_max_iters} iterations)")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, infos = hlu.gmres_solve(A2, B2, H2, restart=args.restart, tol=args.tol,
                                   max_iters=args.kappa2_max_iters, raise_on_fail=False)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = H2.hlu_get_stats()
        it = [i["iters"] for i in infos]
        log(f"kappa {args.kappa2:g} {prec} eps {eps:g}: iters {min(it)}..{max(it)}, {T:.2f}s")
        out[key] = {"eps": eps, "factor_s": tf, "solves_per_s": Xs.shape[0] / T, "iters": [min(it), max(it)],
                     "converged": all(i["converged"] for i in infos),
                     "relres_max": max(i["relres"] for i in infos),
                     "err_vs_xstar_max": ((x - Xs).norm(dim=1) / Xs.norm(dim=1)).max().item(),
                     "ranks": {"max": st["max_rank"], "mean": st["mean_rank"]}}
    # the single-problem refinement rule (gmres_solve_refined): FP64 at eps,
    # at most 100 first-try iterations, then one refactorisation at eps / 10
    if not args.no_fp64:
        log(f"kappa {args.kappa2:g} fp64 eps {args.eps:g}: GMRES with refinement")
        H2.hlu_factor(args.eps, prec="fp64", allow_overflow=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, infos, refines = hlu.gmres_solve_refined(A2, B2, H2, restart=args.restart, tol=args.tol,
                                                    max_iters=args.kappa2_max_iters, refine_iters=100,
                                                    max_refines=1, eps_factor=0.1, raise_on_fail=False)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        it = [i["iters"] for i in infos]
        log(f"kappa {args.kappa2:g} fp64 refined: {refines} refactorisation(s), iters {min(it)}..{max(it)}, "
            f"{T:.2f}s")
        out["fp64_refined"] = {"eps": args.eps, "refine_iters": 100, "eps_factor": 0.1, "refines": refines,
                               "seconds_incl_refactor": T, "solves_per_s": Xs.shape[0] / T,
                               "iters_last_solve": [min(it), max(it)],
                               "converged": all(i["converged"] for i in infos),
                               "relres_max": max(i["relres"] for i in infos),
                               "err_vs_xstar_max": ((x - Xs).norm(dim=1) / Xs.norm(dim=1)).max().item()}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.batch:
        return batch_main(args)
    if args.table1:
        return table1_main(args)
    if args.serve:
        return serve_main(args)
    import numpy as np
    import torch
    from paper_2211_11303_amd import hlu, inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe_gib > 0:
        nb = int(args.copy_probe_gib * (1 << 30))
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read and {nb} bytes written by one copy kernel")
        del src, dst
    if args.factor_only:
        return factor_only(args, stream)
    if args.inverse:
        return inverse_main(args, stream)
    t = time.perf_counter()
    log(f"assembling n={args.n}")
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(args.n, args.kappa)
    A = hlu.SpMat(rp, ci, va)
    N = A.n
    H = hlu.HLU(rp, ci, va, mid, eta=2.0, leaf=args.leaf)
    log(f"N={N}: planning the factorisation")
    ws32 = H.hlu_workspace_bytes(args.eps, prec="fp32")
    setup_s = time.perf_counter() - t
    log(f"setup {setup_s:.1f}s, workspace {ws32 / 1e9:.1f} GB")
    stats0 = H.hlu_get_stats()

    # right-hand sides for seeds 0..2, resident on the device, one block
    Xb = torch.cat([torch.tensor(inputs.exact_solution_cols(N, args.nrhs, seed=s), device="cuda")
                    for s in range(3)]).contiguous()
    Bb = A.hlu_spmv(Xb)
    X = [Xb]
    B = [Bb]
    nrhs_step = Xb.shape[0]
    torch.cuda.synchronize()

    def factor(prec):
        log(f"{prec}: first factorisation (uploads plans, binds workspace)")
        H.hlu_factor(args.eps, prec=prec, allow_overflow=True)
        log(f"{prec}: timed factorisation")
        _, tf = event_time(lambda: H.hlu_factor(args.eps, prec=prec, allow_overflow=True), stream)
        log(f"{prec}: factor {tf:.2f}s")
        return tf, H.hlu_get_stats()

    def solve_batch(i):
        return hlu.gmres_solve(A, B[0], H, restart=args.restart, tol=args.tol, max_iters=1000,
                               raise_on_fail=False)

    result = {}
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp32-acc64", "fp64"]):
        tf, st = factor(prec)
        for w in range(args.warmup):
            solve_batch(w)
        # every persistent solve launch in the timed region is bracketed by
        # HIP events on its stream (inside the library)
        H.hlu_set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, relres, xs = [], [], []
        for k in range(args.steps):
            x, infos = solve_batch(k)
            log(f"{prec}: step {k} iters {[i['iters'] for i in infos]}")
            iters += [i["iters"] for i in infos]
            relres += [i["relres"] for i in infos]
            xs.append(x)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        errs = [((x - X[0]).norm(dim=1) / X[0].norm(dim=1)).max().item() for x in xs]
        ts = H.hlu_get_stats()
        H.hlu_set_timing(False)
        result[prec] = dict(factor_s=tf, T=T, solves_per_s=args.steps * nrhs_step / T, iters=iters, x0=xs[0],
                            relres_max=max(relres), err_xstar_max=max(errs),
                            solve_launches=ts["solve_launches"], solve_columns=ts["solve_columns"],
                            solve_kernel_s=ts["solve_kernel_ms"] / 1e3,
                            max_rank=st["max_rank"], mean_rank=st["mean_rank"],
                            lowrank_entries=st["lowrank_entries"], capped=st["capped_blocks"],
                            factor_flops=st["factor_flops"],
                            factor_flops_by_kind={k: st["factor_flops_" + k] for k in ("getrf", "tri", "gemm",
                                                                                       "trunc")},
                            err_vs_oracle=oracle_errors(args, x, X[0]),
                            per_sweep=per_sweep_rates(A, H, B[0], args))

    r32 = result["fp32"]
    # algorithmic bytes of one H-solve launch (L then U sweep) on c columns:
    # every stored factor entry read once (4-byte FP32 factors) + the FP64
    # vector block read and written once per sweep: 4 (D + R) + 32 N c
    s_bytes = 4
    D = stats0["dense_entries"]
    R = r32["lowrank_entries"]
    launches = r32["solve_launches"]
    alg_bytes_total = launches * s_bytes * (D + R) + 2 * 2 * 8 * N * r32["solve_columns"]
    alg_bytes = alg_bytes_total / max(1, launches)
    launch_s = r32["solve_kernel_s"] / max(1, launches)
    achieved = alg_bytes / launch_s / 1e9
    cols = r32["solve_columns"] / max(1, launches)
    traffic = (SOLVE_TRAFFIC["bytes_per_launch"]
               if (SOLVE_TRAFFIC["sha256"] == solve_sources_sha256() and cols == SOLVE_TRAFFIC["columns"]
                   and args.n == 32 and args.leaf == 64) else None)
    line = {
        "metric": "H-LU factor s + precond. GMRES solves/sec to 1e-8; FP32-HLU vs FP64-HLU",
        "value": r32["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["T"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-hlu+f64-gmres",
        "data": "synthetic",
        "config": {"workload": f"kuhn-cube-{args.n}^3 Nedelec (N={N}), kappa={args.kappa:g}, eta=2, "
                               f"leaf={args.leaf}, eps={args.eps:g}, GMRES({args.restart}) to {args.tol:g}, "
                               f"{args.nrhs} rhs x seeds 0-2 = {nrhs_step} rhs per step",
                   "n": args.n, "N": N, "nnz": A.nnz, "kappa": args.kappa, "eps": args.eps,
                   "leaf": args.leaf, "nrhs": nrhs_step, "restart": args.restart, "tol": args.tol},
        "factor_s_fp32": r32["factor_s"],
        "iters_fp32": sorted(set(r32["iters"])),
        "relres_max_fp32": r32["relres_max"],
        "err_vs_xstar_max_fp32": r32["err_xstar_max"],
        "setup_s": setup_s,
        "workspace_gb_fp32": ws32 / 1e9,
        "structure": {k: stats0[k] for k in ("num_clusters", "num_leaf_clusters", "num_admissible",
                                              "num_dense", "dense_entries", "factor_waves",
                                              "factor_tasks", "solve_waves")},
        "ranks_fp32": {"max": r32["max_rank"], "mean": r32["mean_rank"], "capped": r32["capped"]},
        "factor_flops_fp32": r32["factor_flops"],
        "factor_gflops_per_s_fp32": r32["factor_flops"] / r32["factor_s"] / 1e9,
        "factor_flops_by_kind_fp32": r32["factor_flops_by_kind"],
        "err_vs_oracle_fp32": r32["err_vs_oracle"],
        "per_sweep_fp32": r32["per_sweep"],
        "roofline": {"bound": "hbm", "kernel": "chain_solve_kernel<float>: one H-solve (L then U sweep) "
                                               "per launch, fp32 factors, fp64 vectors; launches of the "
                                               "timed region",
                     "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes, "launch_s": launch_s,
                     "launches": launches, "columns_per_launch": r32["solve_columns"] / max(1, launches)},
    }
    if "fp64" in result:
        r64 = result["fp64"]
        line.update({"factor_s_fp64": r64["factor_s"], "solves_per_s_fp64": r64["solves_per_s"],
                     "iters_fp64": sorted(set(r64["iters"])), "relres_max_fp64": r64["relres_max"],
                     "err_vs_xstar_max_fp64": r64["err_xstar_max"],
                     "ranks_fp64": {"max": r64["max_rank"], "mean": r64["mean_rank"]},
                     "factor_gflops_per_s_fp64": r64["factor_flops"] / r64["factor_s"] / 1e9,
                     "err_vs_oracle_fp64": r64["err_vs_oracle"], "per_sweep_fp64": r64["per_sweep"],
                     "fp32_over_fp64_solves": r32["solves_per_s"] / r64["solves_per_s"]})
        ra = result["fp32-acc64"]
        line["fp32_storage_fp64_tasks"] = {
            "factor_s": ra["factor_s"], "solves_per_s": ra["solves_per_s"], "iters": sorted(set(ra["iters"])),
            "relres_max": ra["relres_max"], "err_vs_xstar_max": ra["err_xstar_max"],
            "ranks": {"max": ra["max_rank"], "mean": ra["mean_rank"]}}
    if args.fit_margin >= 0:
        line["fitted_capacity_fp32"] = fitted_capacity(args, H, A, B[0], r32, stream)
    if args.kappa2 > 0:
        line["kappa2"] = second_kappa(args, H, X[0], stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        iters_full = max(result["fp64"]["iters"]) if "fp64" in result else max(r32["iters"])
        line["cpu_baseline"] = cpu_baseline(args.n, args.kappa, args.leaf, args.eps, args.restart, args.tol,
                                            args.cpu_level, N, iters_full)
        ref = oracle_full_size(args)
        if ref:
            line["cpu_baseline"]["full_size_oracle"] = ref
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
