"""Benchmark: batched X-Drop seed extension on one MI355X.

One step = one xdrop_extend_batch over the whole synthetic batch (both
extensions of every seed, combine included), inputs already resident in HBM.
Prints one JSON line: GCUPS (paper definition: sum over seeds of |q|*|t| per
second), alignments/s, the roofline of the dominant kernel (integer VALU
bound), the CPU oracle timed on a bounded sample, and a short serving run
(p50/p99 request latency under Poisson arrivals).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
INT32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic int32 operations per live cell (2 gap adds, diagonal add,
# substitution select, 2 max, prune compare and select, running max)
OPS_PER_CELL = 9

METRIC = ("GCUPS + alignments/s (int32, bit-exact) and p50/p99 latency in "
          "serving loop")
DEFAULT_WORKLOAD = "protein-500k"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_tokens(text: str) -> str:
    """C++ source with its comments dropped and every run of white space made
    one blank: what the compiler sees, so that an edit of comments or layout
    leaves it unchanged.  Comment marks inside string and character
    literals are left alone."""
    import re
    pat = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/',
                     re.S)
    out = pat.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ",
                  text)
    return " ".join(out.split())


def kernel_source_digest() -> str:
    """sha256 of the kernel sources' code (comments and layout left out): HBM
    byte counters stored under profiles/ apply only to the kernel code they
    were taken on."""
    import hashlib
    h = hashlib.sha256()
    for rel in ("paper_2304_08662_amd/csrc/xdrop_kernels.hip",
                "paper_2304_08662_amd/csrc/xdrop_internal.h"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
        h.update(b"\0")
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the wave kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel source sha256") != kernel_source_digest():
        return None
    try:
        return int(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def scoring_for(xdrop, scheme):
    if scheme.alphabet == 4 and scheme.matrix is None:
        return xdrop.ScoringSpec(xdrop.DNA2, 4, scheme.match, scheme.mismatch,
                                 scheme.gap, scheme.X)
    return xdrop.ScoringSpec(xdrop.BYTE, scheme.alphabet, 0, 0, scheme.gap,
                             scheme.X, matrix=scheme.full_matrix())


def cpu_baseline(batch, scheme, target_s: float, gpu_cells_per_seed):
    """Oracle on a bounded sample of the same workload (~target_s seconds)."""
    import oracle
    n = len(batch.seeds)
    rng = np.random.default_rng(7)
    order = rng.permutation(n)
    # size the sample from the live cells the GPU reported (oracle ~4e8
    # cells/s per 8 threads here; a first probe corrects the estimate)
    sc = oracle.Scoring(scheme.full_matrix(), scheme.gap, scheme.X)
    probe = batch.subset(order[:min(n, 50)])
    t0 = time.perf_counter()
    _, th = oracle.batch(probe.codes, probe.offsets, probe.seeds, sc)
    dt = time.perf_counter() - t0
    per_seed = dt / max(len(probe.seeds), 1)
    k = int(min(n, max(50, target_s / max(per_seed, 1e-6))))
    sample = batch.subset(order[:k])
    # a workload smaller than the target runs whole, repeated
    reps, dt = 0, 0.0
    while reps == 0 or (dt < target_s / 2 and reps < 40):
        t0 = time.perf_counter()
        out, th = oracle.batch(sample.codes, sample.offsets, sample.seeds, sc)
        dt += time.perf_counter() - t0
        reps += 1
    cells = sample.gcups_cells() * reps
    return {"value": round(cells / dt / 1e9, 3), "unit": "GCUPS",
            "cores": int(th), "kind": "oracle",
            "sample": f"{k} of {n} seeds (random, seed 7) x {reps}, "
                      f"{dt:.1f} s, {int(out['cells'].sum())} live cells per "
                      f"pass, aln/s {k * reps / dt:.1f}"}


def serving_run(xdrop, n_requests: int, rates=(0.8,), budget=64 << 30):
    """Poisson request stream (1-4096 pairs, log-uniform; DNA 1k-generator or
    protein-generator pairs drawn from two pools), served twice: with every
    request carrying its own copy of its sequences, and with the pools
    resident once as sequence sets that requests seed against.  Saturation
    throughput from a closed burst, host-to-device bytes of each, then
    p50/p99 latency of the resident-set form at the given fractions of its
    saturation."""
    from paper_2304_08662_amd import inputs
    rng = inputs.rng_for(5)
    pools = inputs.request_pools(rng, 8192)
    refs = list(inputs.request_refs(rng, n_requests, 0.0, 8192))
    n_aln = sum(len(idx) for _, _, idx in refs)
    cells = 0
    for _, w, idx in refs:
        pool = pools[w][0]
        L = pool.lengths()
        cells += int(np.sum(L[pool.seeds["q"][idx]].astype(np.int64) *
                            L[pool.seeds["t"][idx]]))
    scs = [scoring_for(xdrop, sch) for _, sch in pools]

    def burst(srv, submit):
        t0 = time.perf_counter()
        tk = [submit(i) for i in range(n_requests)]
        for i, t in enumerate(tk):
            srv.wait(t, len(refs[i][2]))
        return time.perf_counter() - t0

    out = {"requests": n_requests, "alignments": n_aln}
    # every request with its own sequences
    own = [pools[w][0].subset(idx) for _, w, idx in refs]
    packed = [(b.packed() if b.alphabet == 4 else b.codes) for b in own]
    srv = xdrop.Server(0, budget_bytes=budget)
    sat = burst(srv, lambda i: srv.submit(packed[i], own[i].offsets,
                                          own[i].seeds, scs[refs[i][1]]))
    out["own_copies"] = {"saturation_aln_per_s": round(n_aln / sat, 1),
                         "saturation_gcups": round(cells / sat / 1e9, 1),
                         "h2d_bytes": srv.stats()["h2d_bytes"]}
    srv.close()
    del own, packed
    # the pools resident once; requests seed against them
    srv = xdrop.Server(0, budget_bytes=budget)
    sids = [srv.put_sequences(p.packed() if p.alphabet == 4 else p.codes,
                              p.offsets, xdrop.DNA2 if p.alphabet == 4
                              else xdrop.BYTE) for p, _ in pools]
    seeds = [pools[w][0].seeds[idx] for _, w, idx in refs]

    def submit_ref(i):
        w = refs[i][1]
        return srv.submit(None, None, seeds[i], scs[w], seq_set=sids[w])

    sat = burst(srv, submit_ref)
    sat_req_per_s = n_requests / sat
    st = srv.stats()
    res = {"saturation_req_per_s": round(sat_req_per_s, 1),
           "saturation_aln_per_s": round(n_aln / sat, 1),
           "saturation_gcups": round(cells / sat / 1e9, 1),
           "h2d_bytes": st["h2d_bytes"], "reused_bytes": st["reused_bytes"],
           "rates": []}
    for frac in rates:
        rate = frac * sat_req_per_s
        gaps = np.random.default_rng(11).exponential(1.0 / rate, n_requests)
        arrive = np.cumsum(gaps)
        lat = np.zeros(n_requests)
        pending = {}
        start = time.perf_counter()
        i = 0
        while i < n_requests or pending:
            now = time.perf_counter() - start
            while i < n_requests and arrive[i] <= now:
                pending[submit_ref(i)] = i
                i += 1
            done = []
            for t, j in pending.items():
                if srv.poll(t, len(refs[j][2])) is not None:
                    lat[j] = time.perf_counter() - start - arrive[j]
                    done.append(t)
            for t in done:
                del pending[t]
            if not done:
                time.sleep(20e-6)
        wall = time.perf_counter() - start
        res["rates"].append({
            "fraction_of_saturation": frac,
            "req_per_s": round(rate, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "aln_per_s": round(n_aln / wall, 1),
            "gcups": round(cells / wall / 1e9, 1)})
    st = srv.stats()
    res["max_batches_in_flight"] = st["max_batches_in_flight"]
    res["admitted_while_busy"] = st["admitted_while_busy"]
    srv.close()
    out["resident_sets"] = res
    out["h2d_bytes_saved"] = out["own_copies"]["h2d_bytes"] - res["h2d_bytes"]
    return out


def load_workload(name: str, scale: float):
    """The seeded workload, kept in /tmp between runs on one host (the
    generator is deterministic; the protein one takes tens of seconds)."""
    from paper_2304_08662_amd import inputs
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"),
                        f"xdrop_bench_{name}_{scale}.npz")
    if os.path.exists(path):
        z = np.load(path)
        batch = inputs.Batch(z["codes"], z["offsets"], z["seeds"],
                             int(z["alphabet"]))
        _, scheme = inputs.workload(name, 1e-9)  # (one pair: the scoring)
        return batch, scheme
    batch, scheme = inputs.workload(name, scale)
    tmp = path + ".tmp.npz"
    np.savez(tmp, codes=batch.codes, offsets=batch.offsets, seeds=batch.seeds,
             alphabet=batch.alphabet)
    os.replace(tmp, path)
    return batch, scheme


UNMEASURED = {
    "dna-100k": ("not run on the GPU: a GPU run of its parity case (on a "
                 "build with a since removed 16-cell wave kernel) did not "
                 "finish and no cause has been shown, so the case stays off "
                 "the GPU; its results are checked on the CPU build of the "
                 "kernel sources only"),
}


def time_steps(ctx, args_dev, sc, res, opts, stream, steps, warmup):
    """Mean ms per step over `steps` batches (HIP events on the launch
    stream, bracketed by device synchronisation), after `warmup`."""
    import torch
    for _ in range(warmup):
        ctx.extend_batch(*args_dev, sc, res, opts, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.extend_batch(*args_dev, sc, res, opts, stream=stream)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps


def phase_times(ctx, args_dev, sc, res, opts, stream, steps):
    """Per-phase ms (HIP events on the launch stream around each kernel of
    the sequence), averaged over `steps` further batches."""
    ctx.set_timing(True)
    for _ in range(steps):
        ctx.extend_batch(*args_dev, sc, res, opts, stream=stream)
    stream.synchronize()
    phase_sum, nb = ctx.last_timing()
    ctx.set_timing(False)
    assert nb == steps
    return np.array(phase_sum) / nb


def other_workload(xdrop, ctx, name, steps, stream):
    """Automatic and plain-form step times of another workload."""
    from paper_2304_08662_amd import inputs
    batch, scheme = load_workload(name, 1.0)
    n = len(batch.seeds)
    packed = batch.packed() if batch.alphabet == 4 else batch.codes
    dev = xdrop.to_device(packed, batch.offsets, batch.seeds)
    res = xdrop.result_buffer(n)
    sc = scoring_for(xdrop, scheme)
    stream.wait_stream(__import__("torch").cuda.current_stream())
    ms, _ = time_steps(ctx, dev, sc, res, None, stream, steps, 2)
    got = xdrop.results_to_numpy(res, n)
    assert (got["status"] == 0).all()
    plain_ms, _ = time_steps(ctx, dev, sc, res, xdrop.options(variant=3),
                             stream, steps, 1)
    o = ctx.resolve_options(sc, n)
    live = int(got["cells"].sum())
    return {"ms_per_step": round(ms, 4),
            "gcups": round(batch.gcups_cells() / (ms / 1e3) / 1e9, 1),
            "alignments_per_s": round(n / (ms / 1e3), 1),
            "live_gcups": round(live / (ms / 1e3) / 1e9, 1),
            "form": {"variant": o.variant, "tile": o.tile, "chunk": o.chunk},
            "plain_ms_per_step": round(plain_ms, 4),
            "seeds": n, "X": scheme.X}


def block_tier_probe(args):
    """The block tier alone: unrelated random pairs of equal length with no
    X-drop (X = 2^31 - 1), so every extension runs all m + n antidiagonals
    and its band grows to the full matrix width; the WORKGROUP form puts
    every extension on the block tier from the first antidiagonal.  Per-phase
    HIP events on the launch stream; ns per antidiagonal of one extension =
    the tier's time / (m + n)."""
    import numpy as np
    import torch
    from paper_2304_08662_amd import inputs, xdrop
    ctx = xdrop.Context(0)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    shapes = [(1, 1000, 4), (1, 2000, 4), (256, 1000, 4), (1024, 1000, 4),
              (256, 1000, 20)]
    for npairs, length, alpha in shapes:
        rng = np.random.default_rng(5)
        pairs = [(rng.integers(0, alpha, length).astype(np.uint8),
                  rng.integers(0, alpha, length).astype(np.uint8), 0, 0, 0)
                 for _ in range(npairs)]
        batch = inputs._assemble(pairs, alpha, {})
        if alpha == 4:
            scheme = inputs.Scheme(4, 1, -1, -1, 2**31 - 1)
        else:
            scheme = inputs.Scheme(
                20, gap=-2, X=2**31 - 1,
                matrix=inputs.stand_in_substitution_matrix())
        sc = scoring_for(xdrop, scheme)
        packed = batch.packed() if alpha == 4 else batch.codes
        dev = xdrop.to_device(packed, batch.offsets, batch.seeds)
        res = xdrop.result_buffer(len(batch.seeds))
        opts = xdrop.options(xdrop.VARIANT_WORKGROUP)
        for _ in range(args.warmup):
            ctx.extend_batch(*dev, sc, res, opts, stream=stream)
        stream.synchronize()
        # (phases: prep, wave kernel, handed-on extensions, block tier and
        # device-memory tier, combine)
        ph = phase_times(ctx, dev, sc, res, opts, stream, args.steps)
        steps = 2 * length  # antidiagonals of one extension (m + n)
        print(json.dumps({
            "block_tier": {"pairs": npairs, "length": length,
                           "alphabet": alpha,
                           "workgroup_ms": round(float(ph[3]), 4),
                           "ns_per_antidiagonal":
                               round(float(ph[3]) * 1e6 / steps, 1),
                           "tiers": ctx.last_stats()}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="0.5,0.8,0.95")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the automatic choice without tuning first "
                         "(by default the launch form, tile and chunk are "
                         "tuned on the batch before the timed steps)")
    ap.add_argument("--tuning", default=None, metavar="PATH",
                    help="tuning cache (JSON lines): read instead of tuning "
                         "if it exists, else written by the tuning run")
    ap.add_argument("--others", default="dna-1k,dna-tail",
                    help="other workloads timed after the headline one")
    ap.add_argument("--block-tier", action="store_true",
                    help="only time the block tier (bands of 513-2,048 "
                         "cells) on unrelated random pairs with no X-drop "
                         "and exit: one JSON line per batch shape")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB five "
                         "times (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU "
              "path (the work would shard by seeds, with no exchange "
              "between GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.workload in UNMEASURED:
        print(f"{args.workload}: {UNMEASURED[args.workload]}", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_08662_amd import inputs, xdrop
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written":
                          nbytes, "copies": 5}), flush=True)
        return
    if args.block_tier:
        block_tier_probe(args)
        return
    log(f"generating {args.workload} x{args.scale}")
    batch, scheme = load_workload(args.workload, args.scale)
    n = len(batch.seeds)
    packed = batch.packed() if batch.alphabet == 4 else batch.codes
    dev = xdrop.to_device(packed, batch.offsets, batch.seeds)
    res = xdrop.result_buffer(n)
    ctx = xdrop.Context(0)
    sc = scoring_for(xdrop, scheme)
    given = args.variant or args.tile or args.chunk
    opts = xdrop.options(args.variant, args.tile, args.chunk) if given else None
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    tuned = None
    if args.tuning and os.path.exists(args.tuning) and not given:
        ctx.load_tuning(args.tuning)
        o = ctx.resolve_options(sc, n)
        tuned = {"variant": o.variant, "tile": o.tile, "chunk": o.chunk,
                 "from": args.tuning}
    elif not args.no_autotune and not given:
        log("autotune")
        t0 = time.perf_counter()
        best = ctx.autotune(*dev, sc, res, cache_path=args.tuning,
                            stream=stream)
        stream.synchronize()
        tuned = {"variant": best.variant, "tile": best.tile,
                 "chunk": best.chunk,
                 "seconds": round(time.perf_counter() - t0, 2)}
        log(f"tuned {tuned}")
    ms_step, wall_step = time_steps(ctx, dev, sc, res, opts, stream,
                                    args.steps, args.warmup)
    got = xdrop.results_to_numpy(res, n)
    assert (got["status"] == 0).all(), "unexpected per-seed status"
    live = int(got["cells"].sum())
    cells = batch.gcups_cells()
    gcups = cells / (ms_step / 1e3) / 1e9
    phase = phase_times(ctx, dev, sc, res, opts, stream, args.steps)
    # the plain form (one launched wave per extension, no queue) on the same
    # batch: the baseline the persistent form is compared with
    plain_ms, _ = time_steps(ctx, dev, sc, res, xdrop.options(variant=3),
                             stream, max(2, args.steps // 2), 1)
    form = ctx.resolve_options(sc, n, opts)
    # (1) the first extension kernel: the row or 16-bit kernel in those
    # forms, else the wave kernel; (2) the wave kernel on the extensions
    # that kernel handed on
    names = ["prep", "extend", "extend_handed_on", "workgroup", "combine"]
    dom = int(np.argmax(phase))
    achieved = OPS_PER_CELL * live / (phase[dom] / 1e3) / 1e12
    stats = ctx.last_stats()
    log(f"step {ms_step:.3f} ms  wall/step {wall_step * 1e3:.3f} ms  plain "
        f"{plain_ms:.3f} ms  phases {dict(zip(names, np.round(phase, 4)))}  "
        f"tiers {stats}")

    out = {
        "metric": METRIC,
        "value": round(gcups, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "scale": args.scale,
                   "seeds": n, "X": scheme.X, "alphabet": scheme.alphabet},
        "alignments_per_s": round(n / (ms_step / 1e3), 1),
        "live_gcups": round(live / (ms_step / 1e3) / 1e9, 1),
        "live_cells": live,
        "form": {"variant": form.variant, "tile": form.tile,
                 "chunk": form.chunk},
        "plain_ms_per_step": round(plain_ms, 4),
        "speedup_vs_plain": round(plain_ms / ms_step, 3),
        "phase_ms": dict(zip(names, [round(float(x), 4) for x in phase])),
        "tiers": stats,
        "tuned": tuned,
        "roofline": {"bound": "alu", "kernel": names[dom],
                     "achieved": round(achieved, 3),
                     "peak": round(INT32_PEAK_TOPS, 1), "unit": "TOP/s",
                     "frac": round(achieved / INT32_PEAK_TOPS, 4),
                     "traffic": measured_traffic(args.workload)},
        "unmeasured": UNMEASURED,
    }
    others = [w for w in args.others.split(",") if w and w != args.workload]
    if others:
        out["other_workloads"] = {}
        for w in others:
            log(f"other workload {w}")
            out["other_workloads"][w] = other_workload(
                xdrop, ctx, w, 20 if w == "dna-1k" else 5, stream)
    ctx.close()
    if args.serve_requests > 0:
        log("serving run")
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        out["serving"] = serving_run(xdrop, args.serve_requests, rates)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(batch, scheme, args.cpu_seconds,
                                           live / n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
