"""Benchmark of the find-or-put hot path on one MI355X.

Default workload (one step = clear the table, then find-or-put the whole
batch): 2^28 two-word keys, 2^27 distinct keys each occurring twice in a
seeded shuffled order, into a table of 2^28 slots (load factor 0.5 at the
end).  Inputs are resident in HBM before the timed region; the step runs on
the current stream and is timed with HIP events.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the find-or-put kernel) and the CPU oracle timed on a bounded sample.

Extra modes (not the default): --sweep (bucket words x subgroup x keys per
subgroup at load factors 0.5 and 0.9) and --probe (random-access bandwidth of
granules of 4..256 bytes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("states explored/sec + find-or-put Mops/s, % HBM roofline; batched vs single")
HBM_PEAK_GBS = 8000.0
GRANULE = 64  # assumed random-access granule in bytes (see the probe mode)
SEED = 1801058570


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28, help="log2 of the number of keys")
    ap.add_argument("--bucket", type=int, default=32)
    ap.add_argument("--subgroup", type=int, default=8)
    ap.add_argument("--kps", type=int, default=1, help="keys in flight per subgroup")
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--hashes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--explore", action="store_true",
                    help="explore random networks (see --net) instead of the find-or-put batch")
    ap.add_argument("--net", action="append", default=[],
                    help="seed:procs:nstates:live:degree:sinkprob (repeatable)")
    ap.add_argument("--cap", type=float, default=1e9, help="table capacity in states (explore)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter scale reference)")
    return ap.parse_args()


def algorithmic_bytes_per_op(w: int, B: int, probes_per_op: float, new_frac: float) -> float:
    """Key read + status write + one granule-rounded bucket read per probe +
    the write-back of the claimed granule for new keys."""
    return 4 * w + 1 + probes_per_op * max(4 * B, GRANULE) + new_frac * GRANULE


def run_fop(gx, torch, keys, n_distinct, B, G, U, alpha, H, steps, warmup):
    """Time `steps` steps of (clear, find-or-put); returns a dict of figures."""
    n = keys.shape[0]
    cap = int(n_distinct / alpha + 0.999999)
    t = gx.Table(2, B, cap, subgroup=G, keys_per_subgroup=U, max_hashes=H)
    st = torch.empty(n, dtype=torch.uint8, device=keys.device)
    n_new = torch.zeros(1, dtype=torch.int64, device=keys.device)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        t.clear(stream)
        if ev:
            ev[1].record(stream)
        t.find_or_put(keys, st, n_new, stream)
        if ev:
            ev[2].record(stream)

    for _ in range(warmup):
        n_new.zero_()
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_new.zero_()
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(steps):
        step(evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    clear_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
    fop_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / steps
    s = t.stats()  # figures of the last step (clear resets them)
    new_last = int((st == gx.GX_NEW).sum().item())
    full_last = int((st == gx.GX_FULL).sum().item())
    info = t.info
    t.close()
    probes = s.probes / max(1, s.lookups)
    return dict(total_ms=total_ms, ms_per_step=total_ms / steps, clear_ms=clear_ms,
                fop_ms=fop_ms, probes_per_op=probes, new=new_last, full=full_last,
                max_hash_index=s.max_hash_index, n_new_sum=int(n_new.item()),
                table_bytes=info.bytes, n_slots=info.n_slots, H=info.max_hashes,
                B=B, G=G, U=U, alpha=alpha)


def measured_traffic(args):
    """HBM bytes per find-or-put launch from the committed rocprofv3 counter
    summary, when it was taken on the same kernel source and configuration
    (otherwise None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "fop_kernel_2p28_B32_G8_U1_traffic.json")
    try:
        meta = json.load(open(path))
    except (OSError, ValueError):
        return None
    csrc = os.path.join(ROOT, "paper_1801_05857_amd", "csrc")
    src = "".join(open(os.path.join(csrc, f)).read() for f in ("gx_device.hpp", "gx_fop_kernel.hpp"))
    cfg = {"log2n": args.log2n, "bucket_words": args.bucket, "subgroup": args.subgroup,
           "keys_per_subgroup": args.kps, "alpha": args.alpha}
    if meta.get("source_sha256") != hashlib.sha256(src.encode()).hexdigest() or meta.get("config") != cfg:
        return None
    return float(meta["traffic_bytes_per_launch"])


def cpu_baseline(target_s: float = 15.0):
    """The oracle (std::unordered_set insertion, one thread) on a bounded
    sample of the same workload shape: a stream of 2^k distinct two-word keys
    each occurring twice, shuffled; k is chosen from a 2^22-key calibration run
    so that the measured run takes about target_s."""
    import math

    import oracle
    import workloads as W

    def timed(k):
        keys = W.duplicated_stream(1 << k, 2, 2, seed=SEED)
        s = oracle.OracleSet(2)
        t0 = time.perf_counter()
        s.insert(keys)
        return keys.shape[0], time.perf_counter() - t0

    n0, dt0 = timed(21)
    k = int(round(math.log2(max(1.0, target_s * n0 / dt0 / 2))))
    k = max(21, min(26, k))
    n, dt = timed(k)
    return {"value": round(n / dt / 1e6, 3), "unit": "Mops/s", "cores": 1, "kind": "oracle",
            "sample": f"std::unordered_set insertion of 2^{k + 1} two-word keys "
                      f"(2^{k} distinct, each twice, shuffled), one thread, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1801_05857_amd as gx
    import workloads as W

    gx.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.probe:
        buf = torch.empty(1 << 29, dtype=torch.int32, device=dev)  # 2 GiB
        buf.fill_(1)
        sink = torch.zeros(1, dtype=torch.int64, device=dev)
        for g in (4, 8, 16, 32, 64, 128, 256):
            n_reads = (1 << 31) // g if g >= 64 else (1 << 26)
            gx.gather_probe(buf, g, n_reads, 7, sink)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            gx.gather_probe(buf, g, n_reads, 7, sink)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            print(json.dumps({"probe_granule_bytes": g, "reads": n_reads, "ms": ms,
                              "Greads_per_s": n_reads / ms / 1e6,
                              "GB_per_s_useful": n_reads * g / ms / 1e6}), flush=True)
        return

    if args.explore:
        for spec in args.net or ["1:12:64:5:3:0.2"]:
            seed, P, ns, live, deg, sink = spec.split(":")
            net = W.random_lts(int(seed), int(P), int(ns), int(live), int(deg), 32, 0.25,
                               float(sink))
            w = gx.network_words(net)
            t = gx.Table(w, args.bucket, int(args.cap), subgroup=args.subgroup,
                         keys_per_subgroup=args.kps, max_hashes=args.hashes or 64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                # first run: sizes the table-resident buffers; the timed run
                # explores into the cleared table with every buffer resident
                gx.explore(net, t)
                cold = time.perf_counter() - t0
                t.clear()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = gx.explore(net, t)
                dt = time.perf_counter() - t0
                s = t.stats()
                per_state = (r.n_transitions / max(1, r.n_states))
                S = t.info.slot_words
                bps = per_state * max(4 * args.bucket, GRANULE) + 8 * S + GRANULE
                print(json.dumps({"net": spec, "words": w, "states": r.n_states,
                                  "transitions": r.n_transitions, "levels": len(r.levels),
                                  "max_level": int(r.levels.max()), "deadlocks": len(r.deadlocks),
                                  "seconds": round(dt, 4), "cold_seconds": round(cold, 4),
                                  "states_per_s": round(r.n_states / dt),
                                  "succ_per_state": round(per_state, 2),
                                  "probes_per_lookup": round(s.probes / max(1, s.lookups), 4),
                                  "algo_GBps": round(r.n_states * bps / dt / 1e9, 1),
                                  "load": round(r.n_states / t.info.n_slots, 3)}), flush=True)
            except gx.GxError as e:
                print(json.dumps({"net": spec, "error": str(e),
                                  "seconds": round(time.perf_counter() - t0, 3)}), flush=True)
            t.close()
        return

    n = 1 << args.log2n
    n_distinct = n // 2
    keys, _ = W.duplicated_stream_torch(n_distinct, 2, SEED, dev)
    torch.cuda.synchronize()

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        a.fill_(3)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.sweep:
        for alpha, H in ((0.5, 8), (0.9, 128)):
            for B in (8, 16, 32, 64):
                for G in (8, 16, 32, 64):
                    for U in (1, 2, 4, 8):
                        r = run_fop(gx, torch, keys, n_distinct, B, G, U, alpha, H, 2, 1)
                        bpo = algorithmic_bytes_per_op(2, B, r["probes_per_op"], 0.5)
                        r["Mops_per_s"] = n / r["fop_ms"] / 1e3
                        r["algo_GBps"] = n * bpo / r["fop_ms"] / 1e6
                        r["roofline_frac"] = r["algo_GBps"] / HBM_PEAK_GBS
                        print(json.dumps(r), flush=True)
        return

    H = args.hashes or (8 if args.alpha <= 0.5 else 128)
    r = run_fop(gx, torch, keys, n_distinct, args.bucket, args.subgroup, args.kps, args.alpha,
                H, args.steps, args.warmup)
    if r["new"] != n_distinct or r["full"] != 0:
        raise SystemExit(f"result check failed: {r['new']} new, {r['full']} full")
    bpo = algorithmic_bytes_per_op(2, args.bucket, r["probes_per_op"], 0.5)
    achieved = n * bpo / (r["fop_ms"] * 1e-3) / 1e9
    value = n / (r["ms_per_step"] * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"isolated find-or-put: 2^{args.log2n} two-word keys, "
                         f"2^{args.log2n - 1} distinct each inserted twice, shuffled; "
                         f"table cleared then filled to load factor {args.alpha}"),
            "bucket_words": args.bucket, "subgroup": args.subgroup,
            "keys_per_subgroup": args.kps, "max_hashes": r["H"],
            "table_slots": r["n_slots"], "table_bytes": r["table_bytes"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "algorithmic_bytes_per_launch": round(n * bpo),
            "kernel": "fop_kernel",
            "kernel_ms": round(r["fop_ms"], 4),
            "bytes_per_op": round(bpo, 2),
            "probes_per_op": round(r["probes_per_op"], 4),
        },
        "find_or_put_Mops_per_s_kernel": round(n / (r["fop_ms"] * 1e-3) / 1e6, 1),
        "clear_ms": round(r["clear_ms"], 4),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
