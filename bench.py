#!/usr/bin/env python3
"""Benchmark: KKT solves/s at FP64 relative residual 1e-6 on one MI355X.

Workload (default, the largest single-GPU configuration): 48^3 hex elements x
96 time steps (34,235,859 unknowns), a = exp(0.5 g) with g a seeded smooth
random field, two moving Gaussian sources, 125 lattice sensors, 1% noise,
beta = 1e-4; two-level space-time RAS: fine 4x4x4x8 subdomains, overlap 1,
ILU(0) with FP64 factors; coarse mesh 12^3 x 24 with the exact block LU in
time (FP64); FGMRES(50) to rtol 1e-6.

One step = one source-identification solve: new noisy sensor data for the
same operator (fresh noise draw) -> right-hand side -> FGMRES from x0 = 0 to
rtol 1e-6.  The operator assembly, the ILU(0) setup and the coarse setup are
done once per operator and reported separately (setup_ms).  Inputs are
resident in HBM when the timed region starts.

Prints one JSON line.  --gpus must be 1: the solver runs on a single GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "cube32x64": "32^3 x 64 (7,007,715 unknowns), one-level RAS 4x4x4x8 overlap 2 ILU(0), GMRES(50), rtol 1e-6",
    "cube8x16": "8^3 x 16 (37,179 unknowns), one-level RAS 2x2x2x2 overlap 1 ILU(0), GMRES(30), rtol 1e-6",
    "cube48x96": "48^3 x 96 (34,235,859 unknowns), two-level: RAS 4x4x4x8 overlap 1 ILU(0), coarse 12^3 x 24 "
                 "(coarse solve: {coarse}), FGMRES(50), rtol 1e-6",
}


# HBM bytes per ras_apply launch measured with the FETCH_SIZE and WRITE_SIZE
# counters (one pass each, `bench.py --kernels-only --config cube48x96`), each scaled by what the
# same counter reads for a 1 GiB device-to-device copy (FETCH x 2.000,
# WRITE x 1.000).  Valid only for the apply-kernel source the counters were
# taken on: a different source hash reports null.
COUNTED_TRAFFIC = {
    ("cube48x96", "f64"): {"ras_hip_sha256": "e48983e44b784066381bec0d7df973906755a792fc95997204a7a2ba2b632143",
                           "read_bytes": 45259019.0 * 2.0 * 1024, "write_bytes": 1060281.1 * 1.0 * 1024},
}


def counted_traffic(config, precision):
    import hashlib
    rec = COUNTED_TRAFFIC.get((config, precision))
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_1508_06103_amd", "csrc", "ras.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["ras_hip_sha256"]:
            return None
    return rec["read_bytes"] + rec["write_bytes"]


def percentile(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v), p))


def algorithmic_apply_bytes(pre, prob):
    """Bytes one ras_apply must move: every factor block once, r gathered on
    every overlapping box, z written once on the owned rows."""
    import numpy as np
    boxes = pre.boxes()
    vol = np.prod(boxes[:, 12:16] - boxes[:, 8:12], axis=1).astype(np.int64)
    return int(pre.factor_bytes + 24 * int(vol.sum()) + 24 * prob.V)


def host_info():
    """Host CPU: threads this process may use and the CPU model."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, model


def cpu_baseline(prob, cfg, iters, sample_subs=2, seed=0):
    """The CPU oracle on a bounded sample of the same workload, on all host cores.

    Per Arnoldi step the oracle does one fine RAS application (every
    subdomain's ILU(0) solve), one matvec (two with the coarse level, whose
    multiplicative combination needs F y), one CGS2 orthogonalisation and, for
    two-level, one exact coarse solve (forward and backward block sweeps with
    the dense LU factors of the Schur complements).  Sample: one full matvec;
    the ILU(0) factors of `sample_subs` of the largest subdomains, solved by
    as many threads as the host gives this process at once (the oracle's C
    solves release the GIL), scaled to every subdomain; one CGS2 step at half
    the restart length on 1/8 of the vector, scaled by 8; two triangular solve
    pairs with a dense LU of the coarse block order, scaled to the block
    sweeps.  The sum, times the GPU's iteration count, gives solves/s.  Setup
    (factorisations) and the coarse transfers are not included.
    """
    import numpy as np
    import scipy.linalg as sla
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import kkt, ras as oras
    threads, model = host_info()
    with threadpool_limits(limits=threads):
        terms = kkt.kkt_terms(prob)
        rng = np.random.default_rng(seed)
        x = rng.standard_normal(prob.unknowns)
        t = time.perf_counter()
        kkt.apply_terms(terms, x)
        t_mv = time.perf_counter() - t
        subs = oras.subdomains(prob, cfg.parts, cfg.overlap)
        vols = np.array([sd.rows for sd in subs])
        pick = sorted(np.argsort(-vols, kind="stable")[:sample_subs].tolist())
        R = oras.RAS(prob, cfg.parts, cfg.overlap, terms=terms, subset=pick)
        work = [pick[i % len(pick)] for i in range(threads)]
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda sid: R.solve_sub(sid, x), work))   # warm
            t = time.perf_counter()
            list(ex.map(lambda sid: R.solve_sub(sid, x), work))
            t_round = time.perf_counter() - t
        rounds = -(-len(subs) // threads)
        t_ras = t_round * rounds
        j = cfg.restart // 2
        n8 = prob.unknowns // 8
        V = rng.standard_normal((j + 1, n8))
        w = rng.standard_normal(n8)
        t = time.perf_counter()
        h1 = V @ w
        w = w - V.T @ h1
        h2 = V @ w
        w = w - V.T @ h2
        np.linalg.norm(w)
        t_orth = 8 * (time.perf_counter() - t)
        del V
        t_coarse, nmv, coarse_txt = 0.0, 1, ""
        if cfg.coarse_factor:
            fac = cfg.coarse_factor
            nb = 3 * np.prod([k // f + 1 for k, f in zip(prob.n, fac[:3])])
            nlev = prob.M // fac[3] + 1
            A = rng.standard_normal((nb, nb)) + nb * np.eye(nb)
            lu = sla.lu_factor(A)
            rhs = rng.standard_normal(nb)
            sla.lu_solve(lu, rhs)
            t = time.perf_counter()
            for _ in range(2):
                sla.lu_solve(lu, rhs)
            t_ls = (time.perf_counter() - t) / 2
            t_coarse = (2 * nlev - 1) * t_ls
            nmv = 2
            coarse_txt = (f", coarse block sweeps {2 * nlev - 1} x {t_ls * 1e3:.1f} ms triangular solve pairs of order "
                          f"{nb}")
    per_iter = t_ras + nmv * t_mv + t_orth + t_coarse
    return {
        "value": 1.0 / (iters * per_iter), "unit": "solves/s", "cores": threads, "kind": "oracle",
        "cpu_model": model,
        "sample": (f"{nmv} x one full matvec ({t_mv:.2f} s, SciPy, one thread), ILU(0) solves of the {len(pick)} "
                   f"largest of {len(subs)} subdomains on {threads} threads at once ({t_round:.3f} s per round, "
                   f"x{rounds} rounds), one CGS2 step at j={j} ({t_orth:.2f} s, scaled from 1/8 of the vector)"
                   f"{coarse_txt}; per-iteration {per_iter:.2f} s x {iters} GPU iterations; setup (factorisations) "
                   f"and coarse transfers not included"),
    }


def oracle_full_solve(st, seed=0):
    """A complete oracle solve of the small configuration (8^3 x 16, 37,179
    unknowns, one-level RAS 2x2x2x2 overlap 1, GMRES(30) to 1e-6), setup and
    solve timed separately, next to the GPU solving the same system."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits
    from oracle import kkt, ras as oras, krylov
    from workloads.generate import make_problem
    prob, cfg = make_problem("cube8x16")
    threads, _ = host_info()
    with threadpool_limits(limits=threads):
        t = time.perf_counter()
        terms = kkt.kkt_terms(prob)
        F = kkt.assemble(prob, terms=terms)
        b = kkt.rhs(prob)
        R = oras.RAS(prob, cfg.parts, cfg.overlap, terms=terms)
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        xo, so = krylov.gmres(lambda v: F @ v, R.apply, b, restart=cfg.restart, rtol=cfg.rtol)
        t_solve = time.perf_counter() - t
    op = st.KKTOperator(prob)
    pre = st.RAS(op, cfg.parts, cfg.overlap)
    x = torch.zeros_like(op.b)
    times = []
    for _ in range(6):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, sg = st.solve(op, pre, op.b, x, restart=cfg.restart, rtol=cfg.rtol)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    pre.close()
    op.close()
    return {"workload": "cube8x16: " + WORKLOADS["cube8x16"], "oracle_setup_s": t_setup, "oracle_solve_s": t_solve,
            "oracle_iters": so.iters, "oracle_solves_per_s": 1.0 / t_solve, "gpu_solve_ms": 1e3 * min(times[1:]),
            "gpu_iters": sg.iters, "gpu_vs_oracle_rel_l2": err}


def time_kernels(op, pre, reps, coarse=None):
    """Average ras_apply, kkt_matvec and coarse_apply durations, from HIP
    events recorded on the stream the library launches on (torch's current
    stream)."""
    import torch
    stream = torch.cuda.current_stream()
    r = torch.randn(op.n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps
    out = {"ras_apply": timed(lambda: pre.apply(r, z, stream=stream)),
           "kkt_matvec": timed(lambda: op.matvec(r, z, stream=stream))}
    if coarse is not None:
        out["coarse_apply"] = timed(lambda: coarse.apply(r, z, stream=stream))
    # a plain device-to-device copy of 1 GiB: the measured streaming peak
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out["copy_1gib"] = timed(lambda: dst.copy_(src))
    del src, dst
    return out


def kernels_only(op, pre, prob, reps):
    """Kernel timing plus a plain copy of known size (the reference point that
    converts the FETCH_SIZE / WRITE_SIZE counters to bytes)."""
    import torch
    km = time_kernels(op, pre, reps)
    apply_ms, matvec_ms = km["ras_apply"], km["kkt_matvec"]
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"ras_apply_ms": apply_ms, "kkt_matvec_ms": matvec_ms,
                      "ras_apply_algorithmic_bytes": algorithmic_apply_bytes(pre, prob),
                      "copy_bytes_each_way": src.numel() * 8, "reps": reps}), flush=True)


def auto_parts(prob, box=8):
    """Subdomains per axis so that owned boxes are about `box` nodes wide."""
    L = [k + 1 for k in prob.n] + [prob.M + 1]
    return tuple(max(1, int(round(l / box))) for l in L)


def batch_parts(prob, how):
    """(parts, overlap) of an uneven-batch instance: the autotuned table
    (paper_1508_06103_amd/parts_table.json), or boxes of about 8, 12 or 16
    nodes per axis ("box8", "box12", "box16") with overlap 1."""
    if how == "tuned":
        from paper_1508_06103_amd.tune import parts_for
        return parts_for(prob)
    return auto_parts(prob, box=int(how[3:])), 1


def run_batch(args):
    """Batched uneven instances: solves/s of the whole batch per step, FP32
    preconditioners inside FP64 FGMRES(50), against the same instances solved
    one at a time in plain FP64 GMRES(50)."""
    import numpy as np
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import batch_instances, redraw_noise
    probs = batch_instances(count=args.instances, base_seed=3000)
    unknowns = sum(p.unknowns for p in probs)
    print(f"[bench] batch: {len(probs)} instances, {unknowns} unknowns", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ops = [st.KKTOperator(p) for p in probs]
    pres = [st.RAS(op, *batch_parts(p, args.parts), precision=st.F32) for op, p in zip(ops, probs)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for op in ops]
    xs = [torch.zeros_like(b) for b in bs]
    count = len(probs)

    def step(k):
        for i, (p, op) in enumerate(zip(probs, ops)):
            op.rhs(redraw_noise(p, 5000 + k * count + i), out=bs[i])
            xs[i].zero_()
        return st.solve_batch(ops, pres, bs, xs, restart=50, rtol=1e-6)[1]

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    times, its = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        sts = step(args.warmup + k)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        assert all(s.converged and s.rel_res_true <= 1e-6 for s in sts)
        its += [s.iters for s in sts]
        print(f"[bench] batch step {k}: {times[-1]*1e3:.0f} ms, iterations {min(its)}..{max(its)}",
              file=sys.stderr, flush=True)
    total = time.perf_counter() - t_start
    value = count * args.steps / total
    # baseline: the same instances one at a time, plain FP64 (factors rebuilt per instance, setup not timed),
    # with ~8-node boxes, which suit single small solves better than the batch's tuned (larger) boxes
    base_t, base_its = 0.0, []
    for i, (p, op) in enumerate(zip(probs, ops)):
        pre64 = st.RAS(op, *batch_parts(p, "box8"), precision=st.F64)
        op.rhs(redraw_noise(p, 5000 + args.warmup * count + i), out=bs[i])
        xs[i].zero_()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, s = st.solve(op, pre64, bs[i], xs[i], restart=50, rtol=1e-6)
        torch.cuda.synchronize()
        base_t += time.perf_counter() - ts
        base_its.append(s.iters)
        pre64.close()
    base = count / base_t
    print(f"[bench] one at a time FP64: {base_t*1e3:.0f} ms for {count} solves", file=sys.stderr, flush=True)
    return {
        "metric": "KKT solves/s at FP64 rel. residual 1e-6; p50/p99 latency; GMRES iterations",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / f32 preconditioner", "data": "synthetic (seeded uneven instances, fresh noise per step)",
        "config": {"workload": f"batch of {count} uneven instances: n in {{8,12,16,20,24}}, M in {{16,24,32,48}}, "
                               f"1-3 sources, 27-64 sensors, "
                               f"{'autotuned subdomains and overlap per size class' if args.parts == 'tuned' else '~8-node subdomains, overlap 1'}, "
                               f"FGMRES(50)",
                   "unknowns": unknowns},
        "p50_ms": 1e3 * percentile(times, 50), "p99_ms": 1e3 * percentile(times, 99),
        "gmres_iters": float(np.mean(its)), "setup_ms": 1e3 * t_setup,
        "factor_bytes_total": int(sum(p.factor_bytes for p in pres)),
        "baseline_one_at_a_time_fp64": {"value": base, "unit": "solves/s", "gmres_iters": float(np.mean(base_its))},
        "speedup_vs_one_at_a_time_fp64": value / base,
    }


def make_coarse(st, op, fac, how, precision):
    """Coarse level of the served 32^3 x 64 requests: the exact block LU in time
    (requests on one operator share its passes over the dense blocks), or the
    paper's coarse GMRES(4) to 0.1 with a coarse RAS 2x2x2x4, overlap 1."""
    if how == "lu":
        return st.Coarse(op, fac, method=st.COARSE_LU, precision=precision)
    return st.Coarse(op, fac, (2, 2, 2, 4), overlap=1, maxit=4, rtol=0.1, precision=precision,
                     method=st.COARSE_GMRES_RAS)


def run_coarse(args):
    """Coarse corrections y = I_c^h F_c^{-1} I_h^c x with the exact block LU:
    the one-vector path against the multi-right-hand-side path (one pass over
    the dense blocks for q vectors), for the coarse levels of the served
    32^3 x 64 requests (8^3 x 16) and of cube48x96 (12^3 x 24), FP32 and FP64
    blocks, and the wall time of each coarse setup.  Apply times are
    HIP-event averages on the stream of the launches."""
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import make_problem
    out = {}
    for name, kw in (("cube32x64", dict(seed=4, lattice=3)), ("cube48x96", {})):
        prob, _ = make_problem(name, **kw)
        op = st.KKTOperator(prob)
        fac = (4, 4, 4, 4)
        nb = 3 * (prob.n[0] // 4 + 1) ** 3
        nlev = prob.M // 4 + 1
        for prec, esz in ((st.F32, 4), (st.F64, 8)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C = st.Coarse(op, fac, method=st.COARSE_LU, precision=prec)
            torch.cuda.synchronize()
            setup_ms = 1e3 * (time.perf_counter() - t0)
            blocks = esz * nb * nb * (2 * nlev - 1)
            x = torch.randn(16, op.n, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            x0, y0 = x[0].contiguous(), torch.empty_like(x[0])
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

            def timed(fn, reps=5):
                fn()
                torch.cuda.synchronize()
                ev[0].record()
                for _ in range(reps):
                    fn()
                ev[1].record()
                torch.cuda.synchronize()
                return ev[0].elapsed_time(ev[1]) / reps

            rec = {"nb": nb, "levels": nlev, "block_bytes": blocks, "setup_ms": setup_ms,
                   "one_vector_ms": timed(lambda: C.apply(x0, y0))}
            for q in (1, 2, 4, 8, 16):
                rec[f"multi_q{q}_ms"] = timed(lambda: C.apply_multi(x[:q], y[:q]))
            key = f"{name}_coarse_{'f32' if esz == 4 else 'f64'}"
            out[key] = rec
            print(f"[bench] {key}: " + ", ".join(f"{k} {v:.3f}" if isinstance(v, float) else f"{k} {v}"
                                                  for k, v in rec.items()), file=sys.stderr, flush=True)
            C.close()
            del x, y, x0, y0
            torch.cuda.empty_cache()
        op.close()
    top = out["cube48x96_coarse_f32"]
    return {"metric": "coarse corrections/s (exact block-LU coarse solve, 16 right-hand sides per pass)",
            "value": 16e3 / top["multi_q16_ms"], "unit": "corrections/s", "n_gpus": 1, "steps": 5, "warmup": 1,
            "ms_per_step": top["multi_q16_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 vectors / f32 blocks", "data": "synthetic (random vectors)",
            "config": {"workload": "coarse level 12^3 x 24 of cube48x96 (6591 unknowns per level, 25 levels)"},
            "coarse": out}


def run_overlap(args):
    """The overlap study of the paper's two-level method (Section 4, the table
    of overlap sizes): fine mesh 40^3 elements x 40 time steps (--overlap-mesh),
    coarse mesh 20^3 x 20 (factor 2 in space and time), FGMRES(50) to 1e-6;
    fine overlap 1, 2, 4.  Subdomain solves ILU(k) with k = --overlap-ilu (the paper: 0); coarse
    solve the paper's GMRES(4) to 0.1 with the coarse RAS on the same 4x4x4x4
    subdomains, coarse overlap 1 (--coarse gmres, default here), or the exact
    block LU (--coarse lu).  Synthetic cube32x64-style sources and 64 lattice
    sensors (all on coarse nodes).  Reports iterations and solve time per
    overlap."""
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import make_problem, redraw_noise
    m = args.overlap_mesh
    prob, _ = make_problem("cube32x64", n=m, M=m, lattice=4 if m % 5 == 0 else 3)
    prec = st.F64 if args.precision == "f64" else st.F32
    op = st.KKTOperator(prob)
    parts, fac = (4, 4, 4, 4), (2, 2, 2, 2)
    coarse_how = args.coarse if args.coarse_set else "gmres"
    if coarse_how == "lu":
        C = st.Coarse(op, fac, method=st.COARSE_LU, precision=prec)
    else:
        C = st.Coarse(op, fac, parts, overlap=1, maxit=4, rtol=0.1, precision=prec, method=st.COARSE_GMRES_RAS)
    b = op.rhs(redraw_noise(prob, 77))
    rows = []
    for delta in (1, 2, 4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = st.RAS(op, parts, delta, precision=prec, ilu_level=args.overlap_ilu)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        times = []
        for rep in range(2):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s = st.solve(op, pre, b, x, coarse=C, restart=50, rtol=1e-6, flexible=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            assert s.converged and s.rel_res_true <= 1e-6
        rows.append({"overlap": delta, "iters": s.iters, "solve_ms": 1e3 * min(times), "ras_setup_ms": 1e3 * t_setup,
                     "factor_gb": pre.factor_bytes / 1e9})
        print(f"[bench] overlap {delta}, ILU({args.overlap_ilu}), coarse {coarse_how}: {s.iters} its, solve "
              f"{1e3 * min(times):.1f} ms, setup {1e3 * t_setup:.1f} ms, factors {pre.factor_bytes / 1e9:.2f} GB",
              file=sys.stderr, flush=True)
        pre.close()
    coarse_txt = "exact block LU" if coarse_how == "lu" else \
        "GMRES(4) rtol 0.1 with coarse RAS 4x4x4x4 overlap 1"
    return {"metric": f"FGMRES iterations and solve time vs fine overlap (two-level, ILU({args.overlap_ilu}))",
            "value": rows[0]["iters"], "unit": "iterations at overlap 1", "n_gpus": 1, "steps": 2, "warmup": 0,
            "ms_per_step": rows[0]["solve_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": args.precision, "data": "synthetic (seeded moving-Gaussian sources, 64 lattice sensors, 1% noise)",
            "config": {"workload": f"{m}^3 x {m} ({prob.unknowns} unknowns), RAS 4x4x4x4 ILU({args.overlap_ilu}), "
                                   f"coarse {m // 2}^3 x {m // 2} {coarse_txt}, FGMRES(50), rtol 1e-6"},
            "sweep": rows}


def run_ilu(args):
    """The fill-level study of the paper's two-level method (Section 4, the
    table of ILU(k) levels).  Default mesh: the paper's 41^3 nodes x 41 time
    levels (8,477,283 unknowns, `--ilu-mesh 40`), 4x4x4x4 = 256 subdomains with
    overlap 1, coarse mesh 21^3 x 21 (factor 2 in space and time) with the
    paper's coarse GMRES(4) to 0.1 and coarse RAS 4x4x4x4 overlap 1, ILU(0);
    FGMRES(50) to 1e-6.  Fine subdomain solves ILU(k) for the levels given per
    factor precision (the default levels are those whose factors fit the
    device at this mesh).  Synthetic cube32x64-style sources and 64 lattice
    sensors (on coarse nodes).  Reports iterations, solve time, time per
    iteration, factor bytes and the apply's bandwidth per k."""
    import numpy as np
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import make_problem, redraw_noise
    m = args.ilu_mesh
    prob, _ = make_problem("cube32x64", n=m, M=m, lattice=4 if m % 5 == 0 else 3)
    op = st.KKTOperator(prob)
    parts, fac = (4, 4, 4, 4), (2, 2, 2, 2)
    b = op.rhs(redraw_noise(prob, 78))
    rows = []
    plan = [("f32", args.ilu_levels_f32), ("f64", args.ilu_levels_f64)]
    for prec_name, levels in plan:
        levels = [int(k) for k in levels.split(",") if k != ""]
        if not levels:
            continue
        prec = st.F32 if prec_name == "f32" else st.F64
        C = st.Coarse(op, fac, parts, overlap=1, maxit=4, rtol=0.1, precision=prec, method=st.COARSE_GMRES_RAS)
        for k in levels:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pre = st.RAS(op, parts, 1, precision=prec, ilu_level=k)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            print(f"[bench] {prec_name} ILU({k}) setup {t_setup:.1f} s, factors {pre.factor_bytes / 1e9:.1f} GB",
                  file=sys.stderr, flush=True)
            times = []
            for rep in range(2):
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, s = st.solve(op, pre, b, x, coarse=C, restart=50, rtol=1e-6, flexible=True)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                assert s.converged and s.rel_res_true <= 1e-6
            km = time_kernels(op, pre, 5)
            abytes = algorithmic_apply_bytes(pre, prob)
            kname = apply_kernel_name(pre, prec_name) if k == 0 else \
                f"iluk_apply_kernel<{'float' if prec == st.F32 else 'double'}>"
            row = {"precision": prec_name, "ilu_level": k, "iters": s.iters, "solve_ms": 1e3 * min(times),
                   "ms_per_iter": 1e3 * min(times) / s.iters, "ras_setup_ms": 1e3 * t_setup,
                   "factor_gb": pre.factor_bytes / 1e9, "ras_apply_ms": km["ras_apply"],
                   "ras_apply_gbs": abytes / (km["ras_apply"] * 1e-3) / 1e9, "ras_apply_kernel": kname}
            rows.append(row)
            print(f"[bench] {prec_name} ILU({k}): {s.iters} its, solve {row['solve_ms']:.0f} ms "
                  f"({row['ms_per_iter']:.2f} ms/it), setup {row['ras_setup_ms']:.0f} ms, factors "
                  f"{row['factor_gb']:.1f} GB, apply {row['ras_apply_ms']:.2f} ms ({row['ras_apply_gbs']:.0f} GB/s)",
                  file=sys.stderr, flush=True)
            pre.close()
            torch.cuda.empty_cache()
        C.close()
    first = rows[0]
    return {"metric": "FGMRES iterations and time per iteration vs ILU fill level k (two-level)",
            "value": first["iters"], "unit": f"iterations at ILU({first['ilu_level']}), {first['precision']} factors",
            "n_gpus": 1, "steps": 2, "warmup": 0, "ms_per_step": first["solve_ms"], "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64 outer / f32 and f64 factors",
            "data": "synthetic (seeded moving-Gaussian sources, lattice sensors, 1% noise)",
            "config": {"workload": f"{m + 1}^3 nodes x {m + 1} levels ({prob.unknowns} unknowns), RAS 4x4x4x4 overlap 1 "
                                   f"ILU(k), coarse {m // 2 + 1}^3 x {m // 2 + 1} GMRES(4) rtol 0.1 with coarse RAS "
                                   "4x4x4x4 overlap 1, FGMRES(50), rtol 1e-6"},
            "sweep": rows}


def run_serve(args):
    """Poisson request stream through the server (continuous batching, FP32
    preconditioners, FP64 FGMRES(50)); 90% of requests on 16 operators drawn
    from the batch distribution, 10% on the 32^3 x 64 operator with the
    two-level preconditioner.  The one-at-a-time FP64 baseline serves the same
    arrivals first come first served, one solve at a time."""
    import numpy as np
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import batch_instances, make_problem, redraw_noise
    pool = batch_instances(count=16, base_seed=3000)
    large, _ = make_problem("cube32x64", seed=4, lattice=3)   # 27 sensors, all on coarse nodes
    specs = [(p, batch_parts(p, args.parts), None) for p in pool] + [(large, ((4, 4, 4, 8), 1), (4, 4, 4, 4))]
    t0 = time.perf_counter()
    built = []
    for p, (parts, delta), fac in specs:
        op = st.KKTOperator(p)
        pre = st.RAS(op, parts, delta, precision=st.F32)
        C = make_coarse(st, op, fac, args.coarse, st.F32) if fac else None
        built.append((p, op, pre, C))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(4)
    n = args.requests
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=n))
    which = [len(pool) if rng.uniform() < 0.1 else int(rng.integers(len(pool))) for _ in range(n)]
    datas = [redraw_noise(built[w][0], 4000 + k) for k, w in enumerate(which)]
    srv = st.Server(restart=50, rtol=1e-6, device_bytes=96 << 30, max_active=64)
    print(f"[bench] serve: {n} requests at {args.rate}/s, setup {t_setup:.1f} s", file=sys.stderr, flush=True)
    lat, its, pending = [], [], {}
    nxt = 0
    t_begin = time.perf_counter()
    while len(lat) < n:
        now = time.perf_counter() - t_begin
        while nxt < n and arrivals[nxt] <= now:
            p, op, pre, C = built[which[nxt]]
            pending[srv.submit(op, pre, datas[nxt], coarse=C)] = nxt
            nxt += 1
        if pending:
            srv.step()
            tnow = time.perf_counter() - t_begin
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    k = pending.pop(t)
                    assert r[1].converged and r[1].rel_res_true <= 1e-6
                    lat.append(tnow - arrivals[k])
                    its.append(r[1].iters)
        elif nxt < n:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t_begin)))
    t_end = time.perf_counter() - t_begin
    value = n / (t_end - arrivals[0])
    print(f"[bench] served: {value:.2f} solves/s, p50 {1e3*percentile(lat, 50):.0f} ms, "
          f"p99 {1e3*percentile(lat, 99):.0f} ms", file=sys.stderr, flush=True)
    # one at a time, plain FP64: measured service times, first come first served
    svc, base64 = [], {}
    for k in range(n):
        p, op, pre, C = built[which[k]]
        (parts, delta), fac = specs[which[k]][1], specs[which[k]][2]
        if fac is None:
            parts, delta = batch_parts(p, "box8")   # one at a time: ~8-node boxes suit single small solves
        if which[k] not in base64:
            base64[which[k]] = (st.RAS(op, parts, delta, precision=st.F64),
                                make_coarse(st, op, fac, args.coarse, st.F64) if fac else None)
        pre64, C64 = base64[which[k]]
        b = op.rhs(datas[k])
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, s = st.solve(op, pre64, b, x, coarse=C64, restart=50, rtol=1e-6, flexible=C64 is not None)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - ts)
    finish, blat = 0.0, []
    for k in range(n):
        finish = max(finish, arrivals[k]) + svc[k]
        blat.append(finish - arrivals[k])
    base = n / (finish - arrivals[0])
    return {
        "metric": "KKT solves/s at FP64 rel. residual 1e-6; p50/p99 latency; GMRES iterations",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": n, "warmup": 0,
        "ms_per_step": 1e3 * (t_end - arrivals[0]) / n, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 outer / f32 preconditioner",
        "data": "synthetic (seeded request stream, fresh noise per request)",
        "config": {"workload": f"served stream: {n} Poisson requests at {args.rate}/s; 90% on 16 uneven operators "
                               f"(n 8-24, M 16-48, {'autotuned' if args.parts == 'tuned' else '~8-node'} subdomains), "
                               f"10% on 32^3 x 64 with two-level RAS (coarse 8^3 x 16, "
                               f"{'exact block LU' if args.coarse == 'lu' else 'GMRES(4)+RAS'})"},
        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99), "gmres_iters": float(np.mean(its)),
        "setup_ms": 1e3 * t_setup,
        "baseline_one_at_a_time_fp64": {"value": base, "unit": "solves/s", "p50_ms": 1e3 * percentile(blat, 50),
                                        "p99_ms": 1e3 * percentile(blat, 99)},
    }


def build_single(st, prob, cfg, precision, coarse_how):
    """Operator, preconditioner and coarse level of one workload, timed
    (coarse_how None: no coarse level)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = st.KKTOperator(prob)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    pre = st.RAS(op, cfg.parts, cfg.overlap, precision=precision)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    coarse, t_coarse = None, 0.0
    if cfg.coarse_factor and coarse_how is not None:
        t0 = time.perf_counter()
        if coarse_how == "lu":
            coarse = st.Coarse(op, cfg.coarse_factor, method=st.COARSE_LU, precision=precision)
        else:
            # coarse RAS with as many subdomains as the fine level, overlap 1; GMRES(4) to 0.1 (Section 4)
            coarse = st.Coarse(op, cfg.coarse_factor, cfg.parts, overlap=1, maxit=4, rtol=0.1, precision=precision,
                               method=st.COARSE_GMRES_RAS)
        torch.cuda.synchronize()
        t_coarse = time.perf_counter() - t0
    setup = {"assemble": 1e3 * t_asm, "ras_setup": 1e3 * t_setup, "coarse_setup": 1e3 * t_coarse}
    print(f"[bench] assemble {t_asm*1e3:.1f} ms, ras_setup {t_setup*1e3:.1f} ms, coarse_setup {t_coarse*1e3:.1f} ms, "
          f"factors {pre.factor_bytes/1e9:.2f} GB, apply kernel rows per phase {pre.apply_rows}", file=sys.stderr,
          flush=True)
    return op, pre, coarse, setup


def timed_solves(st, prob, cfg, op, pre, coarse, steps, warmup, flexible, tag, seed0=1000):
    """warmup + steps solves with fresh noise; per-step wall times (s) and iterations."""
    import torch
    from workloads.generate import redraw_noise
    b = torch.empty(op.n, dtype=torch.float64, device="cuda")
    x = torch.zeros(op.n, dtype=torch.float64, device="cuda")

    def step(k):
        op.rhs(redraw_noise(prob, seed0 + k), out=b)
        x.zero_()
        return st.solve(op, pre, b, x, coarse=coarse, restart=cfg.restart, rtol=cfg.rtol, maxit=cfg.maxit,
                        flexible=flexible)[1]

    for w in range(warmup):
        s = step(w)
        print(f"[bench] {tag} warmup {w}: {s.iters} its, {s.ms:.1f} ms, res {s.rel_res_true:.2e}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    times, its = [], []
    t_start = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        s = step(warmup + k)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        its.append(s.iters)
        assert s.converged and s.rel_res_true <= cfg.rtol, s
        print(f"[bench] {tag} step {k}: {s.iters} its, {times[-1]*1e3:.1f} ms, res {s.rel_res_true:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return times, its, time.perf_counter() - t_start


def apply_kernel_name(pre, prec_name):
    t = "double" if prec_name == "f64" else "float"
    rows = pre.apply_rows
    return f"apply_ring_kernel<{t}, {rows}>" if rows else f"apply_kernel<{t}>"


def roofline_of(prob, pre, apply_ms, config, prec_name, copy_ms=None):
    """Roofline entry of the apply; with copy_ms (a 1 GiB device copy, read
    plus write) also the fraction of that measured streaming rate."""
    apply_bytes = algorithmic_apply_bytes(pre, prob)
    achieved = apply_bytes / (apply_ms * 1e-3) / 1e9
    out = {"kernel": f"ras_apply ({apply_kernel_name(pre, prec_name)})", "bound": "hbm", "achieved": achieved,
           "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
           "traffic": counted_traffic(config, prec_name), "algorithmic_bytes": apply_bytes}
    if copy_ms:
        copy_gbps = 2.0 * (1 << 30) / (copy_ms * 1e-3) / 1e9
        out["measured_copy_GBps"] = copy_gbps
        out["frac_of_measured_copy"] = achieved / copy_gbps
    return out


def mixed_precision_extra(st, prob, cfg, args, op, pre, coarse):
    """The same workload with FP32 ILU factors and FP32 coarse blocks inside FP64
    FGMRES: solves/s, and the C and f error of the mixed solution against the
    plain FP64 one (same data; op, pre, coarse are the FP64 handles) and
    against a tight FP64 solve (rtol 1e-10).  Closes the FP64 handles before
    building the FP32 ones."""
    import numpy as np
    import torch
    from workloads.generate import redraw_noise
    out = {}
    b = op.rhs(redraw_noise(prob, 999))
    sols = {}

    def solve(tag, op, pre, coarse, rtol):
        x = torch.zeros_like(b)
        _, s = st.solve(op, pre, b, x, coarse=coarse, restart=cfg.restart, rtol=rtol, maxit=cfg.maxit, flexible=True)
        assert s.converged, (tag, s)
        sols[tag] = x.cpu().numpy().reshape(-1, 3)
        out[f"{tag}_iters"] = s.iters
        out[f"{tag}_rel_res_true"] = s.rel_res_true
        print(f"[bench] {tag}: {s.iters} its, res {s.rel_res_true:.2e}", file=sys.stderr, flush=True)

    solve("f64", op, pre, coarse, cfg.rtol)
    solve("f64_tight", op, pre, coarse, 1e-10)
    pre.close()
    if coarse is not None:
        coarse.close()
    op.close()
    torch.cuda.empty_cache()
    op, pre, coarse, setup = build_single(st, prob, cfg, st.F32, args.coarse)
    solve("mixed", op, pre, coarse, cfg.rtol)
    times, its, total = timed_solves(st, prob, cfg, op, pre, coarse, 3, 1, True, "mixed", seed0=2000)
    out.update({"value": 3 / total, "unit": "solves/s", "ms_per_step": 1e3 * total / 3,
                "gmres_iters": float(np.mean(its)), "setup_ms": setup})
    km = time_kernels(op, pre, args.apply_reps, coarse)
    out["kernels_ms"] = km
    out["roofline"] = roofline_of(prob, pre, km["ras_apply"], args.config, "f32", km.get("copy_1gib"))
    pre.close()
    if coarse is not None:
        coarse.close()
    op.close()
    torch.cuda.empty_cache()

    def rel(a, ref, c):
        return float(np.linalg.norm(a[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]))
    out["error"] = {"C_vs_f64": rel(sols["mixed"], sols["f64"], 0), "f_vs_f64": rel(sols["mixed"], sols["f64"], 2),
                    "C_vs_tight": rel(sols["mixed"], sols["f64_tight"], 0),
                    "f_vs_tight": rel(sols["mixed"], sols["f64_tight"], 2),
                    "f64_C_vs_tight": rel(sols["f64"], sols["f64_tight"], 0),
                    "f64_f_vs_tight": rel(sols["f64"], sols["f64_tight"], 2)}
    print(f"[bench] mixed vs FP64: {out['error']}", file=sys.stderr, flush=True)
    return out


def one_level_extra(st, args):
    """cube32x64 (7.0 M unknowns), one-level FP64 GMRES(50): a short run."""
    import numpy as np
    import torch
    from workloads.generate import make_problem
    prob, cfg = make_problem("cube32x64")
    op, pre, coarse, setup = build_single(st, prob, cfg, st.F64, "lu")
    times, its, total = timed_solves(st, prob, cfg, op, pre, None, 3, 1, False, "cube32x64")
    km = time_kernels(op, pre, args.apply_reps)
    out = {"workload": "cube32x64: " + WORKLOADS["cube32x64"], "value": 3 / total, "unit": "solves/s",
           "ms_per_step": 1e3 * total / 3, "gmres_iters": float(np.mean(its)), "setup_ms": setup, "kernels_ms": km,
           "roofline": roofline_of(prob, pre, km["ras_apply"], "cube32x64", "f64", km.get("copy_1gib"))}
    pre.close()
    op.close()
    torch.cuda.empty_cache()
    return out


def run_kernels_only(args):
    import paper_1508_06103_amd as st
    from workloads.generate import make_problem
    prob, cfg = make_problem(args.config)
    prec = st.F64 if args.precision == "f64" else st.F32
    op, pre, coarse, setup = build_single(st, prob, cfg, prec, None)   # no coarse level: its setup is not timed here
    kernels_only(op, pre, prob, args.apply_reps)


def run_single(args):
    import numpy as np
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import make_problem
    t0 = time.perf_counter()
    prob, cfg = make_problem(args.config)
    t_gen = time.perf_counter() - t0
    prec = st.F64 if args.precision == "f64" else st.F32
    print(f"[bench] {args.config}: {prob.unknowns} unknowns, parts {cfg.parts}, overlap {cfg.overlap}, "
          f"generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    op, pre, coarse, setup = build_single(st, prob, cfg, prec, args.coarse)
    flexible = prec == st.F32 or coarse is not None
    times, its, total = timed_solves(st, prob, cfg, op, pre, coarse, args.steps, args.warmup, flexible, "main")
    km = time_kernels(op, pre, args.apply_reps, coarse)
    value = args.steps / total
    mean_its = float(np.mean(its))
    coarse_txt = ("exact block LU in time, FP64" if prec == st.F64 else "exact block LU in time, FP32") \
        if args.coarse == "lu" else "GMRES(4) rtol 0.1 with coarse RAS 4x4x4x8 overlap 1"
    res = {
        "metric": "KKT solves/s at FP64 rel. residual 1e-6; p50/p99 latency; GMRES iterations",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == st.F64 else "f64 outer / f32 preconditioner",
        "data": "synthetic (seeded moving-Gaussian sources, lattice sensors, fresh 1% noise per step)",
        "config": {"workload": f"{args.config}: " + WORKLOADS[args.config].format(coarse=coarse_txt),
                   "unknowns": prob.unknowns, "subdomains": pre.nsub, "precision": args.precision},
        "p50_ms": 1e3 * percentile(times, 50), "p99_ms": 1e3 * percentile(times, 99),
        "gmres_iters": mean_its, "setup_ms": setup, "kernels_ms": km,
        "roofline": roofline_of(prob, pre, km["ras_apply"], args.config, args.precision, km.get("copy_1gib")),
    }
    if not args.no_extras and args.config == "cube48x96" and args.precision == "f64":
        res["mixed_f32_preconditioner"] = mixed_precision_extra(st, prob, cfg, args, op, pre, coarse)
    else:
        pre.close()
        if coarse is not None:
            coarse.close()
        op.close()
    torch.cuda.empty_cache()
    if not args.no_extras:
        if args.config != "cube32x64":
            res["cube32x64_one_level_f64"] = one_level_extra(st, args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(prob, cfg, int(round(mean_its)))
        print("[bench] oracle full solve of cube8x16", file=sys.stderr, flush=True)
        res["oracle_full_solve_cube8x16"] = oracle_full_solve(st)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="cube48x96", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--apply-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="single mode: skip the FP32-preconditioner run of cube48x96 and the cube32x64 run")
    ap.add_argument("--kernels-only", action="store_true",
                    help="no solves: time ras_apply, kkt_matvec and a plain 1 GiB device copy (for counter runs)")
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "coarse", "overlap", "ilu"],
                    help="single: one operator, one solve per step (default); batch: 64 uneven instances per "
                         "step; serve: Poisson request stream through the server; coarse: the exact coarse "
                         "solve with one and with several right-hand sides; overlap: the paper's overlap study "
                         "of the two-level method; ilu: the paper's ILU fill-level study of the two-level method")
    ap.add_argument("--coarse", default="lu", choices=["lu", "gmres"],
                    help="two-level configurations: exact block-LU coarse solve, or the paper's coarse GMRES(4)+RAS")
    ap.add_argument("--overlap-ilu", type=int, default=0, help="overlap mode: ILU level of the fine subdomain solves")
    ap.add_argument("--overlap-mesh", type=int, default=40, help="overlap mode: elements per axis and time steps")
    ap.add_argument("--ilu-mesh", type=int, default=40, help="ilu mode: elements per axis and time steps")
    ap.add_argument("--ilu-levels-f32", default="0,1,2", help="ilu mode: fill levels k run with FP32 factors")
    ap.add_argument("--ilu-levels-f64", default="0,1", help="ilu mode: fill levels k run with FP64 factors")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--parts", default="tuned", choices=["tuned", "box8", "box12", "box16"],
                    help="batch/serve partitions: the autotuned table, or boxes of about 8, 12 or 16 nodes per "
                         "axis with overlap 1")
    ap.add_argument("--requests", type=int, default=100)
    ap.add_argument("--rate", type=float, default=50.0, help="serve mode: arrivals per second")
    args = ap.parse_args()
    args.coarse_set = any(a == "--coarse" or a.startswith("--coarse=") for a in sys.argv[1:])
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.mode == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.mode == "coarse":
        print(json.dumps(run_coarse(args)), flush=True)
        return
    if args.mode == "overlap":
        print(json.dumps(run_overlap(args)), flush=True)
        return
    if args.mode == "ilu":
        print(json.dumps(run_ilu(args)), flush=True)
        return
    if args.kernels_only:
        run_kernels_only(args)
        return
    print(json.dumps(run_single(args)), flush=True)


if __name__ == "__main__":
    main()
