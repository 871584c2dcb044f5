"""Subdomain-partition autotuner for the uneven batched instances.

Two modes, both writing ``parts_table.json`` beside this file (``parts_for``
reads it; the batched and served benchmarks use it):

* in the mix (``--in-mix``, the default table): a tuning batch of 64
  instances drawn like the benchmark's uneven batch but with other seeds is
  solved as one batched FGMRES(50) (FP32 preconditioners, rtol 1e-6), and the
  partition of each size class (n, M) present is chosen by coordinate
  descent on the batch's solve time: starting from owned boxes of about 12
  nodes per axis, each class in turn tries boxes of about 8, 12 or 16 nodes
  per spatial axis and 8, 12 or 16 time levels (overlap 1) and keeps a
  candidate that shortens the whole batch by more than 0.5%.  In a full
  batch the GPU is busy anyway, so the partition that wins is the one with
  the fewest, largest boxes that still converge fast.  One workgroup
  applies a box, streaming its factors at about 20-28 GB/s, so a box with
  more than a compute unit's share of a full batch's factor bytes outlasts
  the rest of the launch: candidates whose largest box holds more FP32
  factor bytes than ``--max-box-mb`` (150 MB: 38 GB of factors over 256
  compute units) are not tried, and a class whose boxes of about 12 nodes
  exceed it starts from its candidate with the fewest boxes under it.
* per class (without ``--in-mix``): a few seeded instances of each class
  are timed alone as a batch under candidate partitions (owned boxes of
  about 6, 8, 12 or 16 nodes per spatial axis and 8 or 16 time levels,
  overlap 1 or 2), and the fastest wins.  Alone, a class favours more,
  smaller boxes, which keep the GPU busy.

    python -m paper_1508_06103_amd.tune [--in-mix] [--out FILE] [--instances K]

The table records every class's partition, so each run can be reproduced.
"""
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "parts_table.json")
SPACE_BOXES = (6, 8, 12, 16)
TIME_BOXES = (8, 16)
OVERLAPS = (1, 2)


def _parts(nodes, box):
    return max(1, int(round(nodes / box)))


MIX_SPACE_BOXES = (8, 12, 16)
MIX_TIME_BOXES = (8, 12, 16)


def box_parts(n, M, box, tbox=None):
    """Parts (px, py, pz, pt) for owned boxes of about `box` nodes per spatial
    axis and `tbox` (default `box`) time levels."""
    p = _parts(n + 1, box)
    return (p, p, p, _parts(M + 1, tbox or box))


def mix_candidates(n, M):
    out = []
    for bs in MIX_SPACE_BOXES:
        for bt in MIX_TIME_BOXES:
            parts = box_parts(n, M, bs, bt)
            if parts not in out:
                out.append(parts)
    return out


MAX_BOX_MB = 150.0


def max_box_bytes(n, M, parts, overlap=1, elem=4):
    """Factor bytes of the largest subdomain box of a partition: on every axis
    the longest range of a part (the even split, the first parts one node
    longer) grown by the overlap and clipped to the mesh; RAS(ILU(0)) stores
    a 3 x 3 block for every pair of box nodes at most one apart on every axis."""
    size = 9 * elem
    for L, p in zip((n + 1, n + 1, n + 1, M + 1), parts):
        q, r = divmod(L, p)
        cuts = [k * q + min(k, r) for k in range(p + 1)]
        ext = max(min(L, cuts[k + 1] + overlap) - max(0, cuts[k] - overlap) for k in range(p))
        size *= 3 * ext - 2
    return size


def mix_start(n, M, cap_mb=MAX_BOX_MB):
    """Starting partition of a class in the mix: boxes of about 12 nodes, or,
    if their largest box exceeds the cap, the candidate under it with the
    fewest boxes."""
    start = box_parts(n, M, 12)
    if max_box_bytes(n, M, start) <= cap_mb * 1e6:
        return start
    under = [p for p in mix_candidates(n, M) if max_box_bytes(n, M, p) <= cap_mb * 1e6]
    return min(under, key=lambda p: (p[0] * p[1] * p[2] * p[3], p)) if under else start


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


def _tune_in_mix(st, torch, args):
    """Coordinate descent of the classes' partitions on the time of one
    batched solve of a whole tuning batch (see the module docstring)."""
    from workloads.generate import BATCH_M, BATCH_N, batch_instances
    probs = batch_instances(count=args.count, base_seed=args.seed)
    cls = [(p.n[0], p.M) for p in probs]
    ops = [st.KKTOperator(p) for p in probs]
    work = {}
    for p, c in zip(probs, cls):
        work[c] = work.get(c, 0) + p.unknowns
    order = sorted(work, key=lambda c: -work[c])
    cap = args.max_box_mb * 1e6
    choice = {c: mix_start(c[0], c[1], args.max_box_mb) for c in order}
    pres = [st.RAS(op, choice[c], 1, precision=st.F32) for op, c in zip(ops, cls)]

    def run():
        xs = [torch.zeros(op.n, dtype=torch.float64, device="cuda") for op in ops]
        st.solve_batch(ops, pres, None, xs, restart=50, rtol=1e-6)   # engine and graphs
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, stats = st.solve_batch(ops, pres, None, xs, restart=50, rtol=1e-6)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, all(s.converged for s in stats), [s.iters for s in stats]

    best, ok, its = run()
    print(f"[tune] mix of {len(probs)}: start (boxes of ~12 nodes) {best:.1f} ms", flush=True)
    for c in order:
        idx = [i for i in range(len(probs)) if cls[i] == c]
        for parts in mix_candidates(*c):
            if parts == choice[c] or max_box_bytes(c[0], c[1], parts) > cap:
                continue
            old = [pres[i] for i in idx]
            for i in idx:
                pres[i] = st.RAS(ops[i], parts, 1, precision=st.F32)
            ms, ok, its_c = run()
            keep = ok and ms < best * 0.995
            print(f"[tune] {c[0]}x{c[1]} parts {parts}: batch {ms:.1f} ms{' (kept)' if keep else ''}", flush=True)
            if keep:
                best, choice[c], its = ms, parts, its_c
                for q in old:
                    q.close()
            else:
                for i, q in zip(idx, old):
                    pres[i].close()
                    pres[i] = q
    classes = {}
    for n in BATCH_N:
        for M in BATCH_M:
            c = (n, M)
            mine = [its[i] for i in range(len(probs)) if cls[i] == c]
            classes[f"{n}x{M}"] = {"parts": list(choice.get(c, mix_start(n, M, args.max_box_mb))), "overlap": 1,
                                   "in_tuning_batch": len(mine),
                                   "iters": round(sum(mine) / len(mine), 1) if mine else None}
    for q in pres:
        q.close()
    for op in ops:
        op.close()
    return {"what": "partition per class chosen in the mix: coordinate descent on the batched FGMRES(50) solve "
                    "time of a whole tuning batch (FP32 RAS(ILU(0)), rtol 1e-6), no box above max_box_mb of "
                    "FP32 factors; classes absent from it keep their starting partition",
            "tuning_batch": {"count": args.count, "base_seed": args.seed, "batch_ms": round(best, 1)},
            "max_box_mb": args.max_box_mb,
            "device": torch.cuda.get_device_name(0), "classes": classes}


def main(argv=None):
    import argparse
    import torch
    import paper_1508_06103_amd as st
    from workloads.generate import BATCH_M, BATCH_N, class_instances

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--instances", type=int, default=4)
    ap.add_argument("--in-mix", action="store_true", help="tune on one batched solve of a whole tuning batch")
    ap.add_argument("--count", type=int, default=64, help="--in-mix: instances in the tuning batch")
    ap.add_argument("--seed", type=int, default=5000, help="--in-mix: base seed of the tuning batch")
    ap.add_argument("--max-box-mb", type=float, default=MAX_BOX_MB,
                    help="--in-mix: largest box's FP32 factor bytes (MB) a candidate may have")
    args = ap.parse_args(argv)
    if args.in_mix:
        out = _tune_in_mix(st, torch, args)
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
        print(f"[tune] wrote {args.out}", flush=True)
        return 0
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
