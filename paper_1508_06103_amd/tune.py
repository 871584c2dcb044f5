"""Subdomain-partition autotuner for the uneven batched instances.

For every size class (n, M) of the uneven batch (n in {8, 12, 16, 20, 24}
elements per axis, M in {16, 24, 32, 48} time steps) the tuner times batched
FGMRES(50) solves (FP32 preconditioners, rtol 1e-6) of a few seeded
instances of that class under candidate partitions: owned boxes of about 6,
8 or 12 nodes per spatial axis and 8 or 16 time levels, overlap 1 or 2.  The
fastest candidate per class goes into ``parts_table.json`` beside this file,
with its time and mean iteration count; ``parts_for`` reads the table.

    python -m paper_1508_06103_amd.tune [--out FILE] [--instances K]

The table is what the batched and served benchmarks use, and it records the
partition of every class so that each run can be reproduced.
"""
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "parts_table.json")
SPACE_BOXES = (6, 8, 12)
TIME_BOXES = (8, 16)
OVERLAPS = (1, 2)


def _parts(nodes, box):
    return max(1, int(round(nodes / box)))


def candidates(n, M):
    """Distinct (parts, overlap) candidates for a class: parts = (px, py, pz, pt)."""
    out = []
    for bs in SPACE_BOXES:
        for bt in TIME_BOXES:
            p = _parts(n + 1, bs)
            parts = (p, p, p, _parts(M + 1, bt))
            for d in OVERLAPS:
                if (parts, d) not in out:
                    out.append((parts, d))
    return out


def _load():
    with open(TABLE) as f:
        return json.load(f)


def parts_for(prob):
    """(parts, overlap) for an instance of the uneven batch, from the tuned
    table (the class with the nearest n, then the nearest M)."""
    tab = _load()["classes"]
    n = prob.n[0]
    M = prob.M
    keys = [tuple(int(v) for v in k.split("x")) for k in tab]
    kn, kM = min(keys, key=lambda k: (abs(k[0] - n), abs(k[1] - M)))
    rec = tab[f"{kn}x{kM}"]
    return tuple(rec["parts"]), int(rec["overlap"])


def _time_candidate(st, torch, probs, ops, parts, overlap):
    pres = [st.RAS(op, parts, overlap, precision=st.F32) for op in ops]
    xs = [torch.zeros(op.n, dtype=torch.float64, device="cuda") for op in ops]
    st.solve_batch(ops, pres, None, xs, restart=50, rtol=1e-6)   # first run: engine and graphs
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = st.solve_batch(ops, pres, None, xs, restart=50, rtol=1e-6)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ok = all(s.converged for s in stats)
    its = sum(s.iters for s in stats) / len(stats)
    for p in pres:
        p.close()
    return ms, its, ok


def main(argv=None):
    import argparse
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import BATCH_M, BATCH_N, class_instances

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--instances", type=int, default=4)
    args = ap.parse_args(argv)
    classes = {}
    for n in BATCH_N:
        for M in BATCH_M:
            probs = class_instances(n, M, count=args.instances)
            ops = [st.KKTOperator(p) for p in probs]
            best = None
            for parts, d in candidates(n, M):
                ms, its, ok = _time_candidate(st, torch, probs, ops, parts, d)
                print(f"[tune] {n}x{M} parts {parts} overlap {d}: {ms:.1f} ms, {its:.1f} its"
                      f"{'' if ok else ' (not converged)'}", flush=True)
                if ok and (best is None or ms < best["ms"]):
                    best = {"parts": list(parts), "overlap": d, "ms": round(ms, 2), "iters": round(its, 1)}
            for op in ops:
                op.close()
            classes[f"{n}x{M}"] = best
            print(f"[tune] {n}x{M}: {best}", flush=True)
    out = {"what": "batched FGMRES(50) solve time of the instances of each class, FP32 RAS(ILU(0)), rtol 1e-6",
           "instances_per_class": args.instances, "device": torch.cuda.get_device_name(0), "classes": classes}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[tune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
