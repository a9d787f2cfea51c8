#!/usr/bin/env python3
"""Benchmark: 6D steady T^2S^2 tensor-train solve to relative residual 1e-8 on one MI355X.

Workload (one "step" = one complete cold-start solve of the whole hot path:
1D ingredients already built, operator TT-matrix, sweeps with local solves,
truncations, enrichment, interface updates and the FP64 residual test):
  -eps Lap u + beta . grad u = f on [-1,1]^6, u = 0 on the boundary,
  N = 32 GLL nodes per dimension (30 interior unknowns, 7.3e8 interior
  unknowns in total, never formed), eps = 1e-3, beta = seeded unit vector
  (seed 0), f = 8-term separable Gaussian mixture (exact TT rank 8),
  superconsistent collocation, stop at ||f - L x|| / ||f|| <= 1e-8 (FP64).

Prints ONE JSON line.  value = seconds per solve (lower is better).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SOLVE_OPTS = dict(tol=3e-10, target=9e-9, max_sweeps=40, kick=24, init_rank=64, check_every=0, seed=0)
RANK_CAP = 256
WORKLOAD = "6d_N32_eps1e-3_gauss8_seed0"

# MI355X peaks used for the roofline (published figures)
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def _hbm_classes():
    return {"ttm_matvec", "kron_trisolve"}


def roofline_entry(name: str, st: dict, traffic=None) -> dict:
    avg_s = st["ms"] / max(st["launches"], 1) / 1e3
    per_launch_bytes = st["bytes"] / max(st["launches"], 1)
    per_launch_flops = st["flops"] / max(st["launches"], 1)
    if name in _hbm_classes():
        achieved = per_launch_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
        return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "launches": st["launches"],
                "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": per_launch_bytes}
    achieved = per_launch_flops / avg_s / 1e12 if avg_s > 0 else 0.0
    # the real FP64 GEMM runs on the matrix cores (V_MFMA_F64_16X16X4_F64);
    # the other classes on the vector ALUs
    bound = "mfma" if name == "gemm_f64" else "alu"
    return {"kernel": name, "bound": bound, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic, "launches": st["launches"],
            "avg_launch_us": avg_s * 1e6, "algorithmic_flops_per_launch": per_launch_flops}


# source file of each kernel class (the traffic counters are valid for one version of it)
KERNEL_SOURCE = {"schur_qr": "schur.hip", "gemm_f64": "gemm.hip", "jacobi_svd": "dense_small.hip",
                 "hessenberg": "dense_small.hip", "hess_solve": "kron_hess.hip", "ttm_matvec": "tt_kernels.hip"}


def kernel_source_sha1(kernel: str):
    import hashlib
    name = KERNEL_SOURCE.get(kernel)
    if name is None:
        return None
    path = os.path.join(ROOT, "paper_2506_04732_amd", "csrc", name)
    if not os.path.exists(path):
        return None
    with open(path, "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()


def load_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if present
    and taken on the current source of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{WORKLOAD}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except Exception:
        return None
    if rec.get("kernel_source_sha1") != kernel_source_sha1(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_solve(prob, threads, opts=None, cap=None):
    """The oracle's full solve of one instance (FP64 NumPy AMEn with exact
    Kronecker local solves), stopped by the GPU solve's rule (FP64 residual
    <= target): (seconds, info, BLAS threads used).  opts / cap: the solve
    options and rank cap (default: the 6D bench workload's)."""
    opts = SOLVE_OPTS if opts is None else opts
    cap = RANK_CAP if cap is None else cap
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import amen as oamen
    from oracle import collocation as col
    from oracle import tt as ott
    ops = col.build_ops(prob.d, prob.N, prob.eps, prob.beta, prob.scheme)
    Es, Ms = col.interior_factors(ops)
    A = ott.kron_sum_ttm(Es, Ms)
    b = ott.separable_to_tt(col.gauss_rhs_factors(ops, prob.gauss.amp, prob.gauss.centre, prob.gauss.width))
    rng = np.random.default_rng(opts["seed"])
    r0 = opts["init_rank"]
    ms = [n - 2 for n in prob.N]
    rs = [1] + [min(r0, 30 ** min(l, prob.d - l)) for l in range(1, prob.d)] + [1]
    x0 = [rng.standard_normal((rs[l], ms[l], rs[l + 1])) for l in range(prob.d)]
    with threadpool_limits(limits=threads):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        t0 = time.perf_counter()
        _, info = oamen.solve(A, b, x0=x0, tol=opts["tol"], target=opts["target"],
                              max_sweeps=opts.get("max_sweeps", 40), kick=opts["kick"], rank_cap=cap,
                              local_solver="kron", kron_factors=(Es, Ms), stop_on_residual=True)
        t = time.perf_counter() - t0
    return t, info, int(used)


def cpu_baseline(prob, one_thread: bool = True) -> dict:
    """The oracle as it stands, timed on the host cores on the whole bench
    workload (not a sample): once with every BLAS thread, once with one."""
    t_all, info, used = _oracle_solve(prob, None)
    print(f"cpu baseline: oracle full solve {t_all:.1f} s on {used} threads, {info['sweeps']} sweeps",
          file=sys.stderr, flush=True)
    out = {"value": t_all, "unit": "s", "cores": used, "kind": "oracle",
           "sample": f"the whole 6D N=32 solve (not a sample): oracle AMEn from a seeded rank-"
                     f"{SOLVE_OPTS['init_rank']} NumPy start, stopped at FP64 residual <= {SOLVE_OPTS['target']}",
           "sweeps": info["sweeps"], "residual": info["residual"], "ranks": info["ranks"],
           "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count()}
    if one_thread:
        t1, info1, used1 = _oracle_solve(prob, 1)
        print(f"cpu baseline: oracle full solve {t1:.1f} s on {used1} thread", file=sys.stderr, flush=True)
        out.update({"value_1thread": t1, "sweeps_1thread": info1["sweeps"], "residual_1thread": info1["residual"]})
    return out


# overlap off: with many instances in flight the GPU is already full, and
# overlap mode factors both interfaces (twice the Francis work) and adds two
# streams per instance onto the same hardware queues
BATCH_OPTS = dict(tol=1e-10, target=1e-8, max_sweeps=30, kick=8, init_rank=8, check_every=0, seed=0, overlap=False)


def bench_batched(args, rank: int):
    """256 uneven instances (d in {4,5,6}, N_l in [16,48], eps in [1e-4,1e-1]),
    each solved to residual 1e-8 under rank cap 128, `workers` at a time on
    concurrent streams.  value = seconds for the whole batch."""
    # HIP maps a process's streams onto this many hardware queues (4 by
    # default); concurrent instances need one each to overlap.  Set before
    # the runtime starts (torch is imported below); 16 <= the 32 allowed.
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(4, args.workers)))
    import numpy as np
    import torch
    import paper_2506_04732_amd as t2s2
    import workloads
    from paper_2506_04732_amd import TT, sources

    insts = workloads.batched_instances(256)
    cap = insts[0].rank_cap
    probs = [t2s2.Problem(q.d, q.N, q.eps, q.beta, q.scheme, rank_cap=cap) for q in insts]
    fs = [sources.gaussians(p, q.gauss.amp, q.gauss.centre, q.gauss.width)
          for p, q in zip(probs, insts)]
    outs = [TT.empty(p.m, cap) for p in probs]
    for _ in range(args.warmup):
        t2s2.solve_batched(probs[:16], fs[:16], outs=outs[:16], workers=args.workers, **BATCH_OPTS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = t2s2.solve_batched(probs, fs, outs=outs, workers=args.workers, **BATCH_OPTS)
        print(f"batched step {k + 1}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    seq = None
    if args.seq_baseline:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i, (p, f, x) in enumerate(zip(probs, fs, outs)):
            p.solve(f, out=x, **BATCH_OPTS)
            if i % 32 == 31:
                print(f"sequential baseline: {i + 1} instances, {time.perf_counter() - t1:.1f} s", file=sys.stderr,
                      flush=True)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t1
    conv = sum(r.converged for r in res)
    # outside the timed region: the first 64 instances again on one stream
    # with every kernel class event-timed, for the dominant class's roofline
    # (with 16 streams in flight an event pair would also time the waits
    # behind other streams' kernels)
    t2s2.timing_classes(None)
    t2s2.timing_enable(True)
    t2s2.solve_batched(probs[:64], fs[:64], outs=outs[:64], workers=1, **BATCH_OPTS)
    torch.cuda.synchronize()
    full = t2s2.timing_read()
    t2s2.timing_enable(False)
    dominant = max(full, key=lambda k: full[k]["ms"])
    roof = roofline_entry(dominant, full[dominant])
    roof["sample"] = "the first 64 instances on one stream, every kernel class event-timed"
    cpu = None
    if not args.no_cpu_baseline and rank == 0:
        # the oracle on a bounded sample: the first instances in order until
        # ~30 s of host time, the mean scaled to the whole batch
        times, used, last = [], 1, None
        for q in insts[:8]:
            t, info, used = _oracle_solve(q, None, opts=BATCH_OPTS, cap=cap)
            times.append(t)
            last = info
            print(f"cpu baseline: oracle instance {len(times) - 1}: {t:.1f} s, {info['sweeps']} sweeps",
                  file=sys.stderr, flush=True)
            if sum(times) >= 30.0:
                break
        n = len(times)
        cpu = {"value": sum(times) / n * len(insts), "unit": "s", "cores": used, "kind": "oracle",
               "sample": f"the first {n} of {len(insts)} instances solved by the oracle (mean "
                         f"{sum(times) / n:.1f} s each, same options and rank cap), scaled to {len(insts)}",
               "sample_times_s": times, "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count()}
    out = {
        "metric": "batched TT solves: seconds for 256 uneven instances to rel. resid 1e-8",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched256_d4-6_N16-48_eps1e-4-1e-1_gauss4", "instances": len(insts),
                   "workers": args.workers, "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "rank_cap": cap, **{k: v for k, v in BATCH_OPTS.items()}},
        "instances_per_s": len(insts) / sec,
        "converged": conv,
        "max_rank_p50": float(np.median([max(r.ranks) for r in res])),
        "sequential_s": seq,
        "speedup_vs_sequential": (seq / sec) if seq else None,
        "kernels": {k: {"ms_64_instances": v["ms"], "launches": v["launches"]} for k, v in full.items()
                    if v["launches"]},
        "roofline": roof, "cpu_baseline": cpu,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


WARM_OPTS = dict(tol=1e-10, target=1e-8, max_sweeps=30, kick=8, init_rank=8, check_every=0, seed=0)


def warm_leg(train: int, test: int, epochs: int, workers: int, log=True) -> dict:
    """Learned warm start, 7D N=24: solve train + test instances (batched),
    train the 3x256 network on the training solutions (rank-8 targets), then
    solve each held-out instance cold and warm (BF16 inference, residual
    judge)."""
    import numpy as np
    import torch
    import paper_2506_04732_amd as t2s2
    import workloads
    from paper_2506_04732_amd import sources, warmstart

    d, N, r8, cap = 7, 24, 8, 128
    ntr, nte = train, test
    t0 = time.perf_counter()
    insts = [workloads.warm_instance(10 ** 6 + i) for i in range(ntr + nte)]
    # training instances are generated in chunks and released once their
    # rank-8 targets are taken (each problem holds its own device buffers);
    # the held-out problems are kept for the cold and warm solves
    targets = []
    probs, fs = [], []
    for k in range(0, ntr + nte, 64):
        chunk = insts[k:min(k + 64, ntr + nte)]
        cp = [t2s2.Problem(q.d, q.N, q.eps, q.beta, q.scheme, rank_cap=cap) for q in chunk]
        cf = [sources.gaussians(p, q.gauss.amp, q.gauss.centre, q.gauss.width) for p, q in zip(cp, chunk)]
        res = t2s2.solve_batched(cp, cf, workers=workers, **WARM_OPTS)
        targets += [warmstart.solution_target(p, r.x, r8) for p, r in zip(cp, res)]
        for j in range(len(chunk)):
            if k + j >= ntr:
                probs.append(cp[j])
                fs.append(cf[j])
        del cp, cf, res
        if log:
            print(f"warm7d: solved {len(targets)} / {ntr + nte} in {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                  flush=True)
    t_gen = time.perf_counter() - t0
    m = [N - 2] * d
    T = torch.stack(targets)
    del targets
    X = torch.from_numpy(warmstart.features([q.meta["params"] for q in insts])).cuda()
    net = warmstart.Network([X.shape[1], 256, 256, 256, warmstart.flat_size(m, r8)], seed=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = net.train(X[:ntr].contiguous(), T[:ntr].contiguous(), m, r8, epochs=epochs, batch=32, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    if log:
        print(f"warm7d: trained {epochs} epochs in {t_train:.0f} s, loss {hist[0]:.3f} -> {hist[-1]:.3f}",
              file=sys.stderr, flush=True)
    Xte, Tte = X[ntr:].contiguous(), T[ntr:].contiguous()
    held, _ = warmstart.fit_loss(net.infer_bf16(Xte).contiguous(), Tte, m, r8)
    base, _ = warmstart.fit_loss(T[:ntr].mean(0, keepdim=True).expand(nte, -1).contiguous(), Tte, m, r8)
    cold_s, warm_s, cold_sw, warm_sw, used, rho_w, rho_c, conv_w = [], [], [], [], [], [], [], []
    for i in range(nte):
        p, f = probs[i], fs[i]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rc = p.solve(f, **WARM_OPTS)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        y = net.infer_bf16(Xte[i:i + 1].contiguous())
        x0 = warmstart.unpack(y[0].contiguous(), m, r8, cap=cap)
        rw = p.solve(f, x0=x0, warm_judge=True, **WARM_OPTS)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        cold_s.append(tb - ta)
        warm_s.append(tc - tb)
        cold_sw.append(rc.sweeps)
        warm_sw.append(rw.sweeps)
        used.append(rw.warm_start_used)
        rho_w.append(rw.warm_residual)
        rho_c.append(rw.cold_residual)
        conv_w.append(rw.converged)
    return {
        "workload": "warm7d_N24_eps1e-4-1e-2_gauss4x3", "train": ntr, "test": nte, "epochs": epochs, "rank": r8,
        "rank_cap": cap, **WARM_OPTS,
        "cold_s_mean": float(np.mean(cold_s)), "warm_s_mean": float(np.mean(warm_s)),
        "sweeps_cold_mean": float(np.mean(cold_sw)), "sweeps_warm_mean": float(np.mean(warm_sw)),
        "sweeps_cold": cold_sw, "sweeps_warm": warm_sw, "warm_used": int(sum(used)),
        "warm_converged": int(sum(conv_w)),
        "heldout_fit_loss_median": float(held.median().item()),
        "mean_target_fit_loss_median": float(base.median().item()),
        "warm_residual_median": float(np.median(rho_w)), "cold_residual_median": float(np.median(rho_c)),
        "train_loss_first_last": [hist[0], hist[-1]], "generate_s": t_gen, "train_s": t_train,
    }


def bench_warm(args, rank: int):
    """The warm-start workload as its own line.  value = mean seconds per
    held-out warm solve (inference incl.)."""
    leg = warm_leg(args.train, args.test, args.epochs, args.workers)
    out = {
        "metric": "learned warm start, 7D N=24: seconds per held-out solve to rel. resid 1e-8 (warm incl. BF16 "
                  "inference)",
        "value": leg["warm_s_mean"], "unit": "s", "n_gpus": 1, "steps": args.test, "warmup": 0,
        "ms_per_step": leg["warm_s_mean"] * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64 solve, f32 train, bf16 infer", "data": "synthetic",
        "config": {"workload": leg["workload"], "train": args.train, "test": args.test, "epochs": args.epochs},
        **{k: v for k, v in leg.items() if k != "workload"},
        "roofline": None, "cpu_baseline": None,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


STAB_OPTS = dict(tol=1e-10, target=1e-8, max_sweeps=20, kick=4, init_rank=4, check_every=1, seed=0)


def _transport_profile(x, eps, beta):
    """Exact solution of beta phi' - eps phi'' = 1 on [-1, 1], phi(+-1) = 0, beta > 0
    (written without overflow): (x + 1)/beta - (2/beta) (e^{a(x+1)} - 1)/(e^{2a} - 1), a = beta/eps."""
    import numpy as np
    a = beta / eps
    frac = np.exp(a * (x - 1.0)) * (-np.expm1(-a * (x + 1.0))) / (-np.expm1(-2.0 * a))
    return (x + 1.0) / beta - (2.0 / beta) * frac


def _sign_changes(v, rel_floor=1e-12):
    import numpy as np
    dv = np.diff(v)
    dv = dv[np.abs(dv) > rel_floor * np.max(np.abs(v))]
    s = np.sign(dv)
    return int(np.count_nonzero(s[1:] != s[:-1])) if s.size >= 2 else 0


def stability_map(d=6, Ns=(8, 12, 16, 24, 32), ratios=(1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6), workers=16,
                  cap=64, log=True):
    """Plain collocation vs superconsistent collocation on the transport-
    dominated problem with the separable exact solution u = prod_l phi_l(x_l)
    (f = sum_l prod_{k != l} phi_k): for every (N, eps / |beta L|) both
    schemes are solved (batched) and the sign changes of the nodal differences
    along the line through the grid centre in direction 1 are counted on the
    GPU's fiber (the exact profile has one)."""
    import numpy as np
    import paper_2506_04732_amd as t2s2
    from paper_2506_04732_amd import TT
    beta = np.full(d, 1.0 / np.sqrt(d))
    cases, probs, fs = [], [], []
    for N in Ns:
        for ratio in ratios:
            eps = 2.0 * ratio          # |beta| = 1, L = 2
            for scheme in (t2s2.SCHEME_SC, t2s2.SCHEME_PLAIN):
                p = t2s2.Problem(d, N, eps, beta, scheme, rank_cap=cap)
                th = [p.colloc(l) for l in range(d)]
                phis = [_transport_profile(th[l], eps, beta[l]) for l in range(d)]
                terms = [[np.ones(N - 2) if k == l else phis[k] for k in range(d)] for l in range(d)]
                cores = []
                for l in range(d):
                    r0, r1 = (1 if l == 0 else d), (1 if l == d - 1 else d)
                    c = np.zeros((r0, N - 2, r1))
                    for t in range(d):
                        c[0 if l == 0 else t, :, 0 if l == d - 1 else t] = terms[t][l]
                    cores.append(c)
                cases.append((N, ratio, scheme))
                probs.append(p)
                fs.append(TT.from_numpy(cores))
    t0 = time.perf_counter()
    res = []
    for k in range(0, len(probs), 32):
        res += t2s2.solve_batched(probs[k:k + 32], fs[k:k + 32], workers=workers, **STAB_OPTS)
        if log:
            print(f"stability: solved {len(res)} / {len(probs)} in {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
    t_solve = time.perf_counter() - t0
    rows = []
    for (N, ratio, scheme), p, r in zip(cases, probs, res):
        eps = 2.0 * ratio
        mid = N // 2 - 1                                   # interior index of GLL node N // 2
        fib = p.tt_fiber(r.x, 0, [mid] * d)
        prof = np.concatenate([[0.0], fib, [0.0]])         # boundary values g = 0
        x = t2s2.nodes(N, eps, beta[0], scheme)[0]
        xc = x[N // 2]
        exact = _transport_profile(x, eps, beta[0]) * np.prod(
            [_transport_profile(np.array([xc]), eps, beta[k])[0] for k in range(1, d)])
        exact[0] = exact[-1] = 0.0
        rows.append({"N": N, "eps_over_beta_L": ratio, "scheme": "SC" if scheme == t2s2.SCHEME_SC else "plain",
                     "sign_changes": _sign_changes(prof), "exact_sign_changes": _sign_changes(exact),
                     "line_max_err": float(np.max(np.abs(prof - exact)) / np.max(np.abs(exact))),
                     "converged": bool(r.converged), "residual": r.residual, "max_rank": max(r.ranks),
                     "sweeps": r.sweeps})
    return {"d": d, "beta": "ones / sqrt(d)", "rows": rows, "solve_s": t_solve}


def bench_stability(args, rank: int):
    m = stability_map(workers=args.workers)
    sc = [r for r in m["rows"] if r["scheme"] == "SC"]
    pl = [r for r in m["rows"] if r["scheme"] == "plain"]
    out = {"metric": "stability map, 6D: oscillation counts of plain vs superconsistent collocation",
           "value": m["solve_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": m["solve_s"] * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "stability6d_transport_closed_form", **STAB_OPTS},
           "sc_oscillatory": sum(r["sign_changes"] > r["exact_sign_changes"] for r in sc),
           "plain_oscillatory": sum(r["sign_changes"] > r["exact_sign_changes"] for r in pl),
           "cases_per_scheme": len(sc), "map": m["rows"], "roofline": None, "cpu_baseline": None}
    if rank == 0:
        print(json.dumps(out), flush=True)


ST_OPTS = dict(tol=1e-9, target=1e-8, max_sweeps=30, kick=8, init_rank=8, check_every=0, seed=0)


def bench_spacetime(args, rank: int):
    """Unified space-time formulation in 7D (6 space dimensions + time):
    du/dt - eps Lap u + beta(x) . grad u = f on [-1,1]^6 x [0, 1], u = 0 on the
    spatial boundary, u(., 0) = 0, with the paper's variable advection
    beta_l(x_l) = sin(pi x_l) (as its degree-11 Legendre series) and the source
    f = e^t prod_l sin(pi x_l) (rank 1); N = 16 nodes per space dimension, 12 in
    time, eps = 1e-3.  value = seconds per solve to residual 1e-8."""
    import numpy as np
    import torch
    import paper_2506_04732_amd as t2s2
    from numpy.polynomial import legendre as npleg
    from paper_2506_04732_amd import TT
    d, N, Nt, eps, T, cap = 6, 16, 12, 1e-3, 1.0, 128
    xs = np.linspace(-1, 1, 4001)
    bcoef = npleg.legfit(xs, np.sin(np.pi * xs), 11)
    p = t2s2.SpaceTimeProblem([N] * d + [Nt], [0] * d + [1], eps, [bcoef] * d, T=T, rank_cap=cap)
    rows = [p.colloc(l) for l in range(d + 1)]
    f = TT.from_numpy([np.sin(np.pi * rows[l]).reshape(1, -1, 1) for l in range(d)]
                      + [np.exp(rows[d]).reshape(1, -1, 1)])
    g = TT.from_numpy([np.zeros((1, N, 1)) for _ in range(d)] + [np.zeros((1, Nt, 1))])
    x = TT.empty(p.m, cap)
    for _ in range(args.warmup):
        p.solve(f, g=g, out=x, **ST_OPTS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [p.solve(f, g=g, out=x, **ST_OPTS) for _ in range(args.steps)]
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    r = res[-1]
    out = {"metric": "7D space-time TT solve seconds to rel. resid 1e-8", "value": sec, "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "spacetime7d_N16_Nt12_eps1e-3_beta_sinpix", "space_dims": d, "N": N, "Nt": Nt,
                      "eps": eps, "T": T, "rank_cap": cap, **ST_OPTS},
           "converged": r.converged, "residual": r.residual, "sweeps": r.sweeps, "final_ranks": r.ranks,
           "phase_ms": r.phase_ms, "unknowns": int(np.prod([float(v) for v in p.m])),
           "roofline": None, "cpu_baseline": None}
    if rank == 0:
        print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-1thread", action="store_true", help="6d: skip the one-thread oracle run")
    ap.add_argument("--no-warm", action="store_true", help="6d: skip the learned warm-start leg")
    ap.add_argument("--warm-train", type=int, default=192, help="6d line's warm leg: training instances")
    ap.add_argument("--warm-test", type=int, default=8, help="6d line's warm leg: held-out instances")
    ap.add_argument("--warm-epochs", type=int, default=100, help="6d line's warm leg: epochs")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--kick", type=int, default=None, help="6d: enrichment rank (default 24)")
    ap.add_argument("--init-rank", type=int, default=None, help="6d: rank of the seeded random start (default 64)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="6d: arithmetic of the local solves (mixed: FP32 factorisations inside FP64 refinement)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="6d: every factorisation on the solve's stream (no side-stream eigendecompositions)")
    ap.add_argument("--workload", choices=["6d", "batched256", "warm7d", "stability", "spacetime7d"], default="6d",
                    help="6d: the 6D N=32 solve (default); batched256: 256 uneven instances solved concurrently; "
                         "warm7d: learned warm start on 7D N=24 (train on solver solutions, held-out cold vs warm)")
    ap.add_argument("--train", type=int, default=1024, help="warm7d: training instances")
    ap.add_argument("--test", type=int, default=32, help="warm7d: held-out instances")
    ap.add_argument("--epochs", type=int, default=200, help="warm7d: training epochs")
    ap.add_argument("--workers", type=int, default=16, help="batched256 / warm7d: concurrent instances")
    ap.add_argument("--seq-baseline", action="store_true",
                    help="batched256: also time the 256 instances solved one after another")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 8 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(8):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8,
                          "launches": 8}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs one solve on one GPU; --gpus {args.gpus} is not supported (the solve is a single-GPU "
              f"workload and the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.workload == "batched256":
        return bench_batched(args, rank)
    if args.workload == "warm7d":
        return bench_warm(args, rank)
    if args.workload == "stability":
        return bench_stability(args, rank)
    if args.workload == "spacetime7d":
        return bench_spacetime(args, rank)

    import torch
    import paper_2506_04732_amd as t2s2
    import workloads
    from paper_2506_04732_amd import TT, sources

    prob = workloads.steady_6d(0, 32)
    if args.no_overlap:
        SOLVE_OPTS["overlap"] = False
    if args.kick is not None:
        SOLVE_OPTS["kick"] = args.kick
    if args.init_rank is not None:
        SOLVE_OPTS["init_rank"] = args.init_rank
    if args.precision == "mixed":
        SOLVE_OPTS["precision"] = t2s2.PRECISION_MIXED
    p = t2s2.Problem(prob.d, prob.N, prob.eps, prob.beta, prob.scheme, rank_cap=RANK_CAP)
    f = sources.gaussians(p, prob.gauss.amp, prob.gauss.centre, prob.gauss.width)
    x = TT.empty(p.m, RANK_CAP)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        p.solve(f, out=x, **SOLVE_OPTS)
    # one solve with every kernel class event-timed (each timed launch costs
    # two host-side event records), outside the timed region: per-class
    # breakdown and the dominant class
    t2s2.timing_classes(None)
    t2s2.timing_enable(True)
    p.solve(f, out=x, **SOLVE_OPTS)
    full = t2s2.timing_read()
    t2s2.timing_enable(False)
    dominant = max(full, key=lambda k: full[k]["ms"])
    kernels = {k: {"ms_per_solve": v["ms"], "launches_per_solve": v["launches"]}
               for k, v in full.items() if v["launches"]}
    # the timed region: only the dominant class and the TT-matvec are
    # event-timed (the roofline figures come from these same steps)
    results = []
    t2s2.timing_classes([dominant, "ttm_matvec"])
    t2s2.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(p.solve(f, out=x, **SOLVE_OPTS))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = t2s2.timing_read()
    t2s2.timing_enable(False)
    t2s2.timing_classes(None)
    sec = (t1 - t0) / args.steps
    last = results[-1]

    roof = roofline_entry(dominant, stats[dominant], load_traffic(dominant))
    ttmv = roofline_entry("ttm_matvec", stats["ttm_matvec"]) if stats["ttm_matvec"]["launches"] else None

    check = {"library_residual": last.residual, "converged": all(r.converged for r in results)}
    if not args.no_oracle_check:
        from oracle import collocation as col
        from oracle import tt as ott
        ops = col.build_ops(prob.d, prob.N, prob.eps, prob.beta, prob.scheme)
        Es, Ms = col.interior_factors(ops)
        b = ott.separable_to_tt(col.gauss_rhs_factors(ops, prob.gauss.amp, prob.gauss.centre, prob.gauss.width))
        check["oracle_residual"] = ott.residual_norm(ott.kron_sum_ttm(Es, Ms), last.x.to_numpy(), b)

    out = {
        "metric": "6D TT solve seconds to rel. resid 1e-8; HBM GB/s; sweeps warm vs cold",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "d": prob.d, "N": prob.N[0], "eps": prob.eps, "source_rank": 8,
                   "target_residual": 1e-8, "stop_at": SOLVE_OPTS["target"], "tol": SOLVE_OPTS["tol"],
                   "kick": SOLVE_OPTS["kick"], "init_rank": SOLVE_OPTS["init_rank"], "rank_cap": RANK_CAP},
        "sweeps_cold": last.sweeps,
        "sweeps_warm": None,
        "warm_start": None,
        "final_ranks": last.ranks,
        "residual": last.residual,
        "phase_ms": last.phase_ms,
        "overlap": SOLVE_OPTS.get("overlap", True),
        "precision": args.precision,
        "refinement_steps": last.refinement_steps, "fp64_fallbacks": last.fp64_fallbacks,
        "refinement_capped": last.refinement_capped, "max_eig_cond": last.max_eig_cond,
        "roofline": roof,
        "ttm_matvec_hbm": ttmv,
        "kernels": kernels,
        "check": check,
    }
    if rank == 0 and not args.no_warm:
        # the learned warm start is defined on its own family (7D N=24, the
        # network's 20 inputs); sweeps warm vs cold are reported there
        leg = warm_leg(args.warm_train, args.warm_test, args.warm_epochs, args.workers)
        out["warm_start"] = leg
        out["sweeps_warm"] = {"workload": leg["workload"], "cold": leg["sweeps_cold_mean"],
                              "warm": leg["sweeps_warm_mean"], "time_cold_s": leg["cold_s_mean"],
                              "time_warm_s": leg["warm_s_mean"]}
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, one_thread=not args.no_cpu_1thread)
    else:
        out["cpu_baseline"] = None
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
