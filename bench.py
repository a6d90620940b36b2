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

import numpy as np

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
    ap.add_argument("--subgroup", type=int, default=4)
    ap.add_argument("--kps", type=int, default=1, help="keys in flight per subgroup")
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--hashes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-explore", action="store_true", help="skip the exploration leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served leg")
    ap.add_argument("--no-alpha9", action="store_true", help="skip the load factor 0.9 run")
    ap.add_argument("--no-dup", action="store_true", help="skip the duplication sweep")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--probe-gib", type=int, action="append", default=[],
                    help="footprint of the gather probe in GiB (repeatable; default 2)")
    ap.add_argument("--explore", action="store_true",
                    help="explore random networks (see --net) instead of the find-or-put batch")
    ap.add_argument("--net", action="append", default=[],
                    help="seed:procs:nstates:live:degree:sinkprob (repeatable)")
    ap.add_argument("--cap", type=float, default=1e9, help="table capacity in states (explore)")
    ap.add_argument("--local-dedup", action="store_true",
                    help="explore with the per-wavefront duplicate filter")
    ap.add_argument("--batch", action="store_true",
                    help="batched exploration of --batch-n uneven random networks")
    ap.add_argument("--batch-n", type=int, default=1024)
    ap.add_argument("--batch-bucket", type=int, default=0, help="0: autotuned per instance")
    ap.add_argument("--batch-subgroup", type=int, default=0, help="0: autotuned per instance")
    ap.add_argument("--batch-kps", type=int, default=0, help="0: autotuned per instance")
    ap.add_argument("--serve", action="store_true",
                    help="served exploration: Poisson request streams at 0.1-1.2x saturation")
    ap.add_argument("--serve-n", type=int, default=1000, help="requests per rate")
    ap.add_argument("--serve-rates", default="0.1,0.25,0.5,0.75,1.0,1.2",
                    help="Poisson rates as multiples of saturation (empty: saturation only)")
    ap.add_argument("--tiny", action="store_true",
                    help="only the tiny configuration")
    ap.add_argument("--explore-large", action="store_true",
                    help="only the large plain-path exploration (3.3e9 states)")
    ap.add_argument("--dup-sweep", action="store_true",
                    help="isolated insertion of 2^27 one-word keys at duplication 1..100")
    ap.add_argument("--token-ring", action="store_true",
                    help="explore Token Ring instances of 2..16 nodes")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter scale reference)")
    ap.add_argument("--fop-only", action="store_true",
                    help="only the timed find-or-put steps (for profiling)")
    return ap.parse_args()


def algorithmic_bytes_per_op(w: int, B: int, probes_per_op: float, new_frac: float) -> float:
    """Key read + status write + one granule-rounded bucket read per probe +
    the write-back of the claimed granule for new keys."""
    return 4 * w + 1 + probes_per_op * max(4 * B, GRANULE) + new_frac * GRANULE


def run_fop_sub_batches(gx, torch, keys, n_distinct, B, G, U, alpha, H, sub):
    """The same insertion into a cleared table as back-to-back launches of
    `sub` keys each on one stream (fastest of two runs after a warm-up):
    returns (ms, NEW count, FULL count)."""
    n = keys.shape[0]
    cap = int(n_distinct / alpha + 0.999999)
    t = gx.Table(2, B, cap, subgroup=G, keys_per_subgroup=U, max_hashes=H)
    st = torch.empty(n, dtype=torch.uint8, device=keys.device)
    stream = torch.cuda.current_stream()
    best = None
    for rep in range(3):
        t.clear(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for lo in range(0, n, sub):
            t.find_or_put(keys[lo:lo + sub], st[lo:lo + sub], None, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if rep:
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
    new = int((st == gx.GX_NEW).sum().item())
    full = int((st == gx.GX_FULL).sum().item())
    t.close()
    return best, new, full


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

    path = os.path.join(ROOT, "profiles", f"fop_kernel_2p{args.log2n}_B{args.bucket}_G{args.subgroup}"
                                          f"_U{args.kps}_traffic.json")
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


def measured_explore_traffic():
    """HBM bytes per exploration of the large workload from the committed
    rocprofv3 counter summary, when it was taken on the same kernel and
    driver sources and table configuration (otherwise None)."""
    import hashlib

    import workloads as W

    path = os.path.join(ROOT, "profiles", "explore_large_random_12x64_B16_G4_traffic.json")
    try:
        meta = json.load(open(path))
    except (OSError, ValueError):
        return None
    csrc = os.path.join(ROOT, "paper_1801_05857_amd", "csrc")
    src = "".join(open(os.path.join(csrc, f)).read() for f in meta["source_files"])
    cfg = dict(W.LARGE_EXPLORE, table_slots=W.LARGE_TABLE_SLOTS)
    if meta.get("source_sha256") != hashlib.sha256(src.encode()).hexdigest() or meta.get("config") != cfg:
        return None
    return float(meta["traffic_bytes_per_exploration"])


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


def claim_ceiling(gx, torch, mode: int, gib: int = 2, n_ops: int = 1 << 28):
    """Operations per second of gx_claim_probe over a `gib` GiB buffer: mode 1
    device-scope compare-and-swaps at random 64-byte granules, mode 2 an
    8-byte read each with a compare-and-swap in the same granule for every
    other one (find-or-put of keys half of which are new)."""
    buf = torch.full((gib << 27,), -1, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    gx.claim_probe(buf, mode, n_ops, 7, sink)
    torch.cuda.synchronize()
    buf.fill_(-1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    gx.claim_probe(buf, mode, n_ops, 11, sink)
    e1.record()
    torch.cuda.synchronize()
    rate = n_ops / (e0.elapsed_time(e1) * 1e-3)
    del buf
    torch.cuda.empty_cache()
    return rate


def random_read_ceiling(gx, torch, granule: int, gib: int = 2):
    """Random reads of `granule` bytes per second over a `gib` GiB buffer
    (gx_gather_probe): the achievable ceiling of one bucket probe."""
    buf = torch.empty(gib << 28, dtype=torch.int32, device="cuda")
    buf.fill_(1)
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    n_reads = max(1 << 24, (1 << 31) // granule)
    gx.gather_probe(buf, granule, n_reads, 7, sink)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    gx.gather_probe(buf, granule, n_reads, 7, sink)
    e1.record()
    torch.cuda.synchronize()
    rate = n_reads / (e0.elapsed_time(e1) * 1e-3)
    del buf
    torch.cuda.empty_cache()
    return rate


def run_tiny(gx, torch, W, reps=100):
    """The tiny configuration (four 8-state cycles with two rendezvous, one
    word, table of 2^16 words, buckets of 32): microseconds per exploration,
    median of `reps` after warm-up."""
    # the network's ctypes view is built once, as a C caller builds its
    # gx_network once for repeated calls
    net = gx.network_view(W.tiny_cycles())
    t = gx.Table(1, 32, 1 << 16, subgroup=8, max_hashes=16)
    times = []
    for k in range(reps + 3):
        t.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gx.explore(net, t)
        if k >= 3:
            times.append(time.perf_counter() - t0)
    t.close()
    times.sort()
    return {"workload": "tiny: 4 cyclic processes of 8 states, 2 rendezvous, w=1, table 2^16 words",
            "states": r.n_states, "levels": len(r.levels),
            # the closed form: 8^4 states, 21 levels, 4 tau steps everywhere plus
            # 2 x 64 joint jumps
            "matches_closed_form": (r.n_states, len(r.levels), r.n_transitions) == (4096, 21,
                                                                                     16512),
            "us_per_explore": round(times[len(times) // 2] * 1e6, 1)}


def cpu_explore_baseline(W):
    """The oracle BFS (std::unordered_set, one thread) on the large workload's
    family at a size it finishes in seconds (4 live states per process)."""
    import oracle

    net = W.large_random_network(live=4)
    t0 = time.perf_counter()
    r = oracle.explore(net)
    dt = time.perf_counter() - t0
    return {"value": round(r.n_states / dt), "unit": "states/s", "cores": 1, "kind": "oracle",
            "sample": f"BFS of the large workload's family with 4 live states per process "
                      f"({r.n_states} states, {r.n_transitions} transitions), one thread, "
                      f"{dt:.1f} s"}


def host_threads() -> int:
    """Host threads the CPU oracle may use: the cores this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_explore_all_cores(W):
    """The oracle's dense-bitmap BFS (oracle.explore_dense) on every host
    thread: the large workload's family at 6 live states per process."""
    import oracle

    threads = host_threads()
    net = W.large_random_network(live=6)
    t0 = time.perf_counter()
    r = oracle.explore_dense(net, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(r.n_states / dt), "unit": "states/s", "cores": threads,
            "kind": "oracle",
            "sample": f"dense-bitmap BFS of the large workload's family with 6 live states per "
                      f"process ({r.n_states} states, {r.n_transitions} transitions), "
                      f"{threads} threads, {dt:.1f} s"}


def cpu_batch_all_cores(W, budget_s: float = 10.0):
    """The oracle's dense-bitmap BFS on every host thread over the batched
    workload's instances in order, until about budget_s seconds have passed."""
    import oracle

    threads = host_threads()
    nets, _ = W.batch_networks(1024, 11)
    states = done = 0
    t0 = time.perf_counter()
    for net in nets:
        states += oracle.explore_dense(net, threads=threads).n_states
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(states / dt), "unit": "states/s", "cores": threads, "kind": "oracle",
            "sample": f"dense-bitmap BFS of the first {done} of the 1024 batched networks "
                      f"({states} states), {threads} threads, {dt:.1f} s"}


def explore_bytes_per_state(f: float, B: int, S: int) -> float:
    """Algorithmic HBM bytes per explored state: its f successors each probe
    one bucket (at least a 64-byte granule), the state is read from its
    frontier and written to the next one (4S bytes each way), and its claim
    writes back one granule."""
    return f * max(4 * B, GRANULE) + 2 * 4 * S + GRANULE


def successor_buffer_bytes_per_state(f: float, w: int) -> float:
    """HBM bytes per explored state that the two-kernel level adds on top of
    the algorithmic ones: every successor is written to the successor buffer
    and read back by the probe kernel (its w words each way; without the
    local duplicate filter the buffer holds w words per successor, not the
    slot's S).  Overhead of this implementation, not counted in the
    roofline."""
    return f * 2 * 4 * w


def roofline_of(states: int, bytes_per_state_total: float, seconds: float) -> dict:
    """Roofline fields of an exploration leg: algorithmic bytes over wall time
    against the 8 TB/s HBM peak."""
    gbps = bytes_per_state_total / seconds / 1e9
    return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_state": round(bytes_per_state_total / max(1, states), 1)}


def run_explore_leg(gx, torch, W, live=8, slots=None):
    """States explored per second on the large plain-path workload (12
    processes of 64 declared states, 3-word vectors, 3.3e9 reachable states,
    192 GB table) in the table configuration W.LARGE_EXPLORE, with the
    table's buffers resident (a first exploration sizes them), timed on the
    second exploration into the cleared table."""
    net = W.large_random_network(live)
    w = gx.network_words(net)
    slots = slots or W.LARGE_TABLE_SLOTS
    cfg = dict(W.LARGE_EXPLORE)
    B = cfg.pop("bucket_words")
    torch.cuda.empty_cache()
    t = gx.Table(w, B, slots, **cfg)
    t0 = time.perf_counter()
    gx.explore(net, t)
    cold = time.perf_counter() - t0
    t.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = gx.explore(net, t)
    dt = time.perf_counter() - t0
    st = t.stats()
    info = t.info
    f = r.n_transitions / r.n_states
    S = info.slot_words
    bps = explore_bytes_per_state(f, B, S)
    t.close()
    out = {"workload": (f"random network: 12 processes x 64 declared states ({live} live), "
                        f"out-degree 3, 32 labels, 25% rendezvous, seed 1, sink 0.15; "
                        f"{w}-word vectors; table {info.n_slots} slots "
                        f"({info.bytes / 1e9:.0f} GB), buckets of {B} words, subgroup "
                        f"{cfg['subgroup']}, {cfg['keys_per_subgroup']} key(s) in flight"),
           "states": r.n_states, "transitions": r.n_transitions, "levels": len(r.levels),
           "seconds": round(dt, 4), "cold_seconds": round(cold, 4),
           "states_per_s": round(r.n_states / dt),
           "lookups_per_s": round(r.n_transitions / dt),
           "successors_per_state": round(f, 2),
           "probes_per_lookup": round(st.probes / max(1, st.lookups), 4),
           "load_factor": round(r.n_states / info.n_slots, 3),
           "roofline": roofline_of(r.n_states, r.n_states * bps, dt),
           "successor_buffer_bytes_per_state": round(successor_buffer_bytes_per_state(f, w), 1)}
    traffic = measured_explore_traffic() if live == 8 and slots == W.LARGE_TABLE_SLOTS else None
    out["roofline"]["traffic"] = traffic
    out["roofline"]["traffic_unit"] = ("HBM bytes per exploration (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                       "scaled per access kind)")
    if traffic:
        out["roofline"]["measured_hbm_GBps"] = round(traffic / dt / 1e9, 1)
    return out


DUP_GRID = ((32, 32, 1), (4, 4, 1), (8, 4, 1), (16, 4, 1), (32, 4, 1), (8, 8, 1), (16, 8, 1),
            (32, 8, 1), (64, 8, 1), (64, 16, 1), (64, 64, 1))
DUPLICATIONS = (1, 2, 4, 8, 16, 21, 32, 50, 64, 100)


def run_dup_sweep(gx, torch, W, log2n=27, alpha=0.5, grid=DUP_GRID, dups=DUPLICATIONS):
    """The isolated insertion experiment of Sec. 5.1 / Fig. 6 at MI355X scale:
    a stream of 2^27 one-word keys in which every distinct key occurs d times
    (d = 1 .. 100), inserted into an empty table sized for load factor alpha
    at the end.  (32, 32, 1) is the paper's static design (a bucket of 32
    integers probed by a warp-sized group of 32 lanes, GH), (4, 4, 1) its
    configurable bucket of 4 integers with a group of 4 (GH-cbs); the rest
    are this library's other bucket and subgroup sizes."""
    n = 1 << log2n
    rows = []
    for dup in dups:
        n_distinct = n // dup
        keys, _ = W.duplicated_stream_torch(n_distinct, dup, SEED, "cuda", w=1)
        m = keys.shape[0]
        st = torch.empty(m, dtype=torch.uint8, device="cuda")
        for B, G, U in grid:
            t = gx.Table(1, B, int(n_distinct / alpha) + 1, subgroup=G, keys_per_subgroup=U,
                         max_hashes=32)
            t.find_or_put(keys, st)  # warm-up
            best = None
            for _ in range(2):
                t.clear()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                t.find_or_put(keys, st)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
            s = t.stats()
            rows.append({"duplication": dup, "bucket_words": B, "subgroup": G,
                         "keys_per_subgroup": U, "keys": m, "ms": round(best, 3),
                         "Mops_per_s": round(m / best / 1e3, 1),
                         "new": s.stored, "full": s.full})
            t.close()
        del keys, st
    torch.cuda.empty_cache()
    return rows


def dup_sweep_summary(rows) -> dict:
    """Fig. 6 in brief: G ops/s of GH (B32, 32 lanes) and GH-cbs (B4, 4
    lanes) and of the fastest configuration, per duplication."""
    out = []
    for dup in sorted({r["duplication"] for r in rows}):
        rr = [r for r in rows if r["duplication"] == dup]
        gh = next(r for r in rr if (r["bucket_words"], r["subgroup"]) == (32, 32))
        cbs = next(r for r in rr if (r["bucket_words"], r["subgroup"]) == (4, 4))
        best = max(rr, key=lambda r: r["Mops_per_s"])
        out.append({"duplication": dup, "GH_B32_g32_Gops": round(gh["Mops_per_s"] / 1e3, 2),
                    "GH_cbs_B4_g4_Gops": round(cbs["Mops_per_s"] / 1e3, 2),
                    "cbs_over_GH": round(cbs["Mops_per_s"] / gh["Mops_per_s"], 2),
                    "best": f"B{best['bucket_words']}-g{best['subgroup']}",
                    "best_Gops": round(best["Mops_per_s"] / 1e3, 2),
                    "wrong_new_counts": sum(int(r["new"] != r["keys"] // dup or r["full"] != 0)
                                            for r in rr)})
    return {"workload": "2^27 one-word keys, each distinct key d times, shuffled; table for "
                        "load 0.5 at the end; GH = buckets of 32 words probed by 32 lanes, "
                        "GH-cbs = buckets of 4 words probed by 4 lanes (Fig. 6)",
            "rows": out}


def run_token_ring(gx, torch, W, sizes=range(2, 17)):
    """Table 1 (right): Token Ring of N nodes, states and states/s per N."""
    rows = []
    for n in sizes:
        net = W.token_ring(n)
        states = 2 * n * 3 ** (n - 1)
        w = gx.network_words(net)
        t = gx.Table(w, 32, max(64, 2 * states), subgroup=8, keys_per_subgroup=1, max_hashes=16)
        gx.explore(net, t)  # sizes the resident buffers
        t.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gx.explore(net, t)
        dt = time.perf_counter() - t0
        rows.append({"token_ring_nodes": n, "words": w, "states": r.n_states,
                     "closed_form": states, "levels": len(r.levels), "seconds": round(dt, 4),
                     "states_per_s": round(r.n_states / dt)})
        t.close()
    return rows


def time_batch_runs(b, torch, reps=3):
    """Median wall time of reps whole runs of a created batch (after one
    untimed run)."""
    b.run()
    torch.cuda.synchronize()
    runs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    return sorted(runs)[len(runs) // 2]


def run_batch(gx, torch, W, n, seed=11, hashes=16, B=0, G=0, U=0):
    """Batched exploration of n uneven random networks under the stepped
    schedule (one multi-instance launch per kernel class per BFS level),
    against the persistent schedule replayed from a hipGraph and against one
    gx_explore call per instance on pre-created tables (all clear their
    tables and start over)."""
    nets, bounds = W.batch_networks(n, seed)
    caps = [2 * c for c in bounds]  # table slots: load factor at most 0.5
    t_setup = time.perf_counter()
    b = gx.Batch(nets, caps, max_hashes=hashes, bucket_words=B, subgroup=G, keys_per_subgroup=U)
    setup_s = time.perf_counter() - t_setup
    t_batch = time_batch_runs(b, torch)
    res = b.results()
    cfgs = [b.instance_config(i) for i in range(n)]
    b.close()
    with gx.Batch(nets, caps, max_hashes=hashes, bucket_words=B, subgroup=G,
                  keys_per_subgroup=U, use_graph=True) as bg:
        t_graph = time_batch_runs(bg, torch)
        res_graph = bg.results()
    # the autotuner's decisions behind the per-instance picks (per slot width,
    # for the combined capacity of its instances), and the same batch at the
    # fixed default configuration
    tuner = {}
    if not (B or G or U):
        foot = {}
        for nt, c in zip(nets, caps):
            w = gx.network_words(nt)
            S = 4 if w >= 3 else w
            f = foot.setdefault(S, [w, 0, 0])
            f[1] += c
            f[2] += 1
        for S, (w, total, cnt) in sorted(foot.items()):
            t = gx.autotune_capacity(w, total)
            tuner[f"slot_words_{S}"] = {
                "instances": cnt, "combined_capacity": total, "size_class": t["size_class"],
                "pick": f"B{t['bucket_words']}-G{t['subgroup']}",
                "ns_per_key": round(t["ns_per_key"], 4),
                "ns_per_key_default_B16_G4": round(t["ns_per_key_default"], 4),
                "ns_per_key_runner_up": round(t["ns_per_key_runner_up"], 4),
                "margin": round(t["ns_per_key_runner_up"] / t["ns_per_key"] - 1, 4)}
        with gx.Batch(nets, caps, max_hashes=hashes, bucket_words=16, subgroup=4,
                      keys_per_subgroup=1) as bf:
            t_fixed = time_batch_runs(bf, torch)
    graph_mismatch = sum(1 for (s1, r1), (s2, r2) in zip(res, res_graph)
                         if s1 != s2 or (r1 is not None and (r1.n_states != r2.n_states or
                                                             r1.levels.tolist() != r2.levels.tolist())))
    ok = [r for st, r in res if st == gx.GX_OK]
    states = sum(r.n_states for r in ok)
    trans = sum(r.n_transitions for r in ok)
    algo_bytes = sum(r.n_states * explore_bytes_per_state(r.n_transitions / max(1, r.n_states),
                                                          cfg[0], 4 if r.words_per_state == 3
                                                          else r.words_per_state)
                     for (st, r), cfg in zip(res, cfgs) if st == gx.GX_OK)
    # one exploration per instance, tables, buffers and the networks' ctypes
    # views resident (the batch marshals its networks once, at creation)
    views = [gx.network_view(nt) for nt in nets]
    tables = [gx.Table(gx.network_words(nt), B, c, subgroup=G, keys_per_subgroup=U,
                       max_hashes=hashes) for nt, c, (B, G, U) in zip(views, caps, cfgs)]
    for nt, t in zip(views, tables):
        try:
            gx.explore(nt, t)  # sizes each table's resident buffers
        except gx.GxError:
            pass
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single_states = 0
    mismatch = 0
    single_failed = 0
    for k, (nt, t) in enumerate(zip(views, tables)):
        t.clear()
        try:
            r = gx.explore(nt, t)
        except gx.GxError:
            single_failed += 1
            continue
        single_states += r.n_states
        st, rb = res[k]
        if (st != gx.GX_OK or rb.n_states != r.n_states or rb.levels.tolist() != r.levels.tolist()
                or rb.n_transitions != r.n_transitions
                or not np.array_equal(rb.deadlocks, r.deadlocks)):
            mismatch += 1
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    for t in tables:
        t.close()
    from collections import Counter
    return {"batched": {
        "workload": f"{n} random networks, 3-10 processes of 4-64 states, reachable sizes "
                    "log-uniform 1e3-1e7 (live-state products), stepped schedule: one "
                    "multi-instance launch per kernel class per BFS level",
        "instances": n, "ok": len(ok), "states": states, "transitions": trans,
        "seconds": round(t_batch, 4), "states_per_s": round(states / t_batch),
        "roofline": roofline_of(states, algo_bytes, t_batch),
        "persistent_graph_seconds": round(t_graph, 4),
        "persistent_graph_states_per_s": round(states / t_graph),
        "persistent_graph_differing": graph_mismatch,
        "fixed_B16_G4_seconds": round(t_fixed, 4) if tuner else None,
        "tuned_vs_fixed_B16_G4": round(t_fixed / t_batch, 3) if tuner else None,
        "autotuner": tuner,
        "one_launch_per_instance_seconds": round(t_single, 4),
        "one_launch_per_instance_states_per_s": round(single_states / t_single),
        "speedup_vs_one_launch_per_instance": round(t_single / t_batch, 2),
        "instances_differing_from_single": mismatch,
        "single_failed": single_failed,
        "setup_seconds": round(setup_s, 2),
        "configs": {f"B{B}-G{G}-U{U}": c for (B, G, U), c in Counter(cfgs).items()}}}


def load_served_pool():
    """Exact results of the served request pool, computed by the CPU oracle
    and stored by tests/golden/make_served_pool.py: {index: dict}."""
    rows = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "served_pool.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x) for x in line.split()]
        rows[v[0]] = {"words": v[1], "states": v[2], "transitions": v[3], "deadlocks": v[4],
                      "levels": v[7:]}
    return rows


def _wrong(st, r, want, gx) -> int:
    """1 when a served result differs from the oracle's (state, transition and
    deadlock counts and every level count), else 0."""
    return int(st != gx.GX_OK or r.n_states != want["states"]
               or r.n_transitions != want["transitions"]
               or len(r.deadlocks) != want["deadlocks"]
               or r.levels.tolist() != want["levels"])


def run_serve(gx, torch, W, n_req=1000, seed=5, rates=(0.1, 0.25, 0.5, 0.75, 1.0, 1.2),
              budget_gib=200):
    """Served exploration: requests drawn (seeded) from a pool of 256 random
    networks with reachable sizes spread log-uniformly over 1e4-1e8 and 1- to
    4-word vectors (W.served_networks(256, 5)), each declaring the product of
    its live-state counts as its bound.  Measured: the saturation rate (all
    n_req requests submitted at once), then Poisson streams of n_req requests
    (seeded exponential gaps) at each multiple of it in ``rates``, with p50/p99
    latency from submission to result; every result is checked against the
    oracle's (tests/golden/served_pool.txt).  Reference: one gx_explore call
    per request, back to back, on a resident table in the server's kernel
    configuration (each pool network timed once on its warm table; the
    reference time is the sum over the requests)."""
    import random

    nets, _, bounds = W.served_networks(256, 5)
    want = load_served_pool()
    rng = random.Random(seed)
    reqs = [rng.randrange(len(nets)) for _ in range(n_req)]
    total_states = sum(want[i]["states"] for i in reqs)
    # one gx_explore call per pool network on a warm, resident table
    t_net = {}
    cfg_of = {}
    for i in sorted(set(reqs)):
        nt = gx.network_view(nets[i])
        w = gx.network_words(nt)
        tb, tg, _ = gx.autotune(w, 0.5)  # the server's kernel configuration
        cfg_of[i] = (tb, 4 if w == 3 else w)
        t = gx.Table(w, tb, max(64, 2 * want[i]["states"]), subgroup=tg, keys_per_subgroup=1,
                     max_hashes=16)
        gx.explore(nt, t)  # sizes its resident buffers
        t.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gx.explore(nt, t)
        t_net[i] = time.perf_counter() - t0
        if _wrong(gx.GX_OK, r, want[i], gx):
            raise SystemExit(f"served pool network {i}: gx_explore differs from the oracle")
        t.close()
    torch.cuda.empty_cache()
    single = sum(t_net[i] for i in reqs)
    algo = sum(want[i]["states"] * explore_bytes_per_state(
        want[i]["transitions"] / max(1, want[i]["states"]), *cfg_of[i]) for i in reqs)
    out = {"workload": (f"{n_req} requests drawn from 256 random networks, reachable sizes "
                        f"log-uniform 1e4-1e8 ({min(want[i]['states'] for i in reqs)}-"
                        f"{max(want[i]['states'] for i in reqs)} drawn), 1-4-word vectors, "
                        "declared bound = product of live-state counts; Poisson arrivals"),
           "requests": n_req, "states_per_rate": total_states,
           "one_call_per_request_states_per_s": round(total_states / single)}
    with gx.Server(budget_gib << 30, max_hashes=16) as srv:
        # all at once: the saturation rate
        t0 = time.perf_counter()
        ids = [srv.submit(nets[i], bounds[i]) for i in reqs]
        bad = 0
        for rid, i in zip(ids, reqs):
            st, r, _ = srv.poll(rid)
            bad += _wrong(st, r, want[i], gx)
        burst = time.perf_counter() - t0
        rate_sat = n_req / burst
        out["saturation"] = {"seconds": round(burst, 3), "requests_per_s": round(rate_sat, 2),
                             "states_per_s": round(total_states / burst),
                             "wrong_results": bad,
                             "vs_one_call_per_request": round(single / burst, 2),
                             "roofline": roofline_of(total_states, algo, burst)}
        print(json.dumps({"served": "saturation", **out["saturation"]}), file=sys.stderr,
              flush=True)
        out["rates"] = []
        for mult in rates:
            lam = mult * rate_sat
            t_arr, times = 0.0, []
            for _ in range(n_req):
                t_arr += rng.expovariate(lam)
                times.append(t_arr)
            ids = []
            start = time.perf_counter()
            for i, ta in zip(reqs, times):
                now = time.perf_counter() - start
                if ta > now:
                    time.sleep(ta - now)
                ids.append(srv.submit(nets[i], bounds[i]))
            lat, bad = [], 0
            for rid, i in zip(ids, reqs):
                st, r, l = srv.poll(rid)
                lat.append(l)
                bad += _wrong(st, r, want[i], gx)
            wall = time.perf_counter() - start
            lat.sort()
            stt = srv.stats()
            row = {"rate_vs_saturation": mult, "rate_per_s": round(lam, 2),
                   "seconds": round(wall, 3), "states_per_s": round(total_states / wall),
                   "p50_latency_s": round(lat[len(lat) // 2], 4),
                   "p99_latency_s": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4),
                   "wrong_results": bad, "retried": stt["retried"],
                   "vs_one_call_per_request": round(single / wall, 2)}
            out["rates"].append(row)
            print(json.dumps({"served": "poisson", **row}), file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "gx runs on one GPU; sharding across GPUs is not implemented, so --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1801_05857_amd as gx
    import workloads as W

    gx.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy:
        # one plain device copy of 1 GiB: the reference that scales the HBM
        # byte counters of a profiled run
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        a.fill_(3)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    if args.probe:
        for gib in args.probe_gib or [2]:
            buf = torch.empty(gib << 28, dtype=torch.int32, device=dev)
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
                print(json.dumps({"footprint_GiB": gib, "probe_granule_bytes": g,
                                  "reads": n_reads, "ms": ms,
                                  "Greads_per_s": n_reads / ms / 1e6,
                                  "GB_per_s_useful": n_reads * g / ms / 1e6}), flush=True)
            del buf
            torch.cuda.empty_cache()
            for mode, what in ((1, "compare-and-swap at a random 64-byte granule"),
                               (2, "8-byte read, compare-and-swap in that granule for every "
                                   "other operation")):
                rate = claim_ceiling(gx, torch, mode, gib)
                print(json.dumps({"footprint_GiB": gib, "claim_probe": what,
                                  "Gops_per_s": round(rate / 1e9, 3)}), flush=True)
        return

    if args.dup_sweep:
        rows = run_dup_sweep(gx, torch, W)
        for row in rows:
            print(json.dumps(row), flush=True)
        print(json.dumps(dup_sweep_summary(rows)), flush=True)
        return
    if args.token_ring:
        for row in run_token_ring(gx, torch, W):
            print(json.dumps(row), flush=True)
        return
    if args.batch:
        print(json.dumps(run_batch(gx, torch, W, args.batch_n, B=args.batch_bucket,
                                   G=args.batch_subgroup, U=args.batch_kps)), flush=True)
        return
    if args.serve:
        rates = tuple(float(x) for x in args.serve_rates.split(",") if x.strip())
        print(json.dumps(run_serve(gx, torch, W, args.serve_n, rates=rates)), flush=True)
        return
    if args.tiny:
        print(json.dumps(run_tiny(gx, torch, W)), flush=True)
        return
    if args.explore_large:
        print(json.dumps(run_explore_leg(gx, torch, W)), flush=True)
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
                gx.explore(net, t, local_dedup=args.local_dedup)
                cold = time.perf_counter() - t0
                t.clear()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = gx.explore(net, t, local_dedup=args.local_dedup)
                dt = time.perf_counter() - t0
                s = t.stats()
                per_state = (r.n_transitions / max(1, r.n_states))
                S = t.info.slot_words
                bps = explore_bytes_per_state(per_state, args.bucket, S)
                print(json.dumps({"net": spec, "words": w, "states": r.n_states,
                                  "transitions": r.n_transitions, "levels": len(r.levels),
                                  "max_level": int(r.levels.max()), "deadlocks": len(r.deadlocks),
                                  "seconds": round(dt, 4), "cold_seconds": round(cold, 4),
                                  "states_per_s": round(r.n_states / dt),
                                  "succ_per_state": round(per_state, 2),
                                  "probes_per_lookup": round(s.probes / max(1, s.lookups), 4),
                                  "algo_GBps": round(r.n_states * bps / dt / 1e9, 1),
                                  "load": round(r.n_states / t.info.n_slots, 3),
                                  "B": args.bucket, "G": args.subgroup, "U": args.kps,
                                  "local_dedup": args.local_dedup,
                                  "local_duplicates": r.local_duplicates}), flush=True)
            except gx.GxError as e:
                print(json.dumps({"net": spec, "error": str(e),
                                  "seconds": round(time.perf_counter() - t0, 3)}), flush=True)
            t.close()
        return

    t_bench = time.perf_counter()
    n = 1 << args.log2n
    n_distinct = n // 2
    keys, _ = W.duplicated_stream_torch(n_distinct, 2, SEED, dev)
    torch.cuda.synchronize()


    if args.sweep:
        for alpha, H in ((0.5, 8), (0.9, 128)):
            for B in (8, 16, 32, 64):
                for G in (4, 8, 16, 32, 64):
                    for U in (1, 2, 4, 8):
                        if U > G or (G == 4 and B > 32):
                            continue
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
    if args.fop_only:
        print(json.dumps(out), flush=True)
        return
    # the achievable random-read rate at the bucket's size, the second
    # denominator of the roofline
    ceil = random_read_ceiling(gx, torch, max(4 * args.bucket, GRANULE))
    out["roofline"]["random_read_ceiling"] = {
        "granule_bytes": max(4 * args.bucket, GRANULE), "G_reads_per_s": round(ceil / 1e9, 2),
        "probes_per_s_frac": round(n * r["probes_per_op"] / (r["fop_ms"] * 1e-3) / ceil, 4)}
    # what the claims cost: device-scope compare-and-swaps alone, and the
    # read-then-claim mix of a stream whose keys are half new, on a buffer
    # of the table's size
    gib = max(1, int(round(r["table_bytes"] / (1 << 30))))
    cas = claim_ceiling(gx, torch, 1, gib)
    mix = claim_ceiling(gx, torch, 2, gib)
    out["roofline"]["claim_ceiling"] = {
        "footprint_GiB": gib, "G_cas_per_s": round(cas / 1e9, 2),
        "G_read_then_half_claim_ops_per_s": round(mix / 1e9, 2),
        "ops_per_s_frac_of_mix": round(n / (r["fop_ms"] * 1e-3) / mix, 4)}
    # the same keys as 2^20-key launches back to back (one batch vs sub-batches)
    sub_ms, sub_new, sub_full = run_fop_sub_batches(gx, torch, keys, n_distinct, args.bucket,
                                                    args.subgroup, args.kps, args.alpha, H,
                                                    1 << 20)
    out["sub_batches_2p20"] = {"launches": (n + (1 << 20) - 1) >> 20,
                               "Mops_per_s": round(n / (sub_ms * 1e-3) / 1e6, 1),
                               "new": sub_new, "full": sub_full}
    if args.alpha == 0.5 and not args.no_alpha9:
        r9 = run_fop(gx, torch, keys, n_distinct, args.bucket, args.subgroup, args.kps, 0.9, 128,
                     2, 1)
        out["load_factor_0.9"] = {
            "Mops_per_s_kernel": round(n / (r9["fop_ms"] * 1e-3) / 1e6, 1),
            "probes_per_op": round(r9["probes_per_op"], 4), "max_hash_index": r9["max_hash_index"],
            "full": r9["full"], "max_hashes": 128, "table_slots": r9["n_slots"]}
    def progress(leg):
        print(json.dumps({"bench_leg_done": leg, "elapsed_s": round(time.perf_counter() - t_bench, 1)}),
              file=sys.stderr, flush=True)

    progress("find-or-put")
    out["tiny"] = run_tiny(gx, torch, W)
    progress("tiny")
    del keys
    torch.cuda.empty_cache()
    if not args.no_explore:
        out["explore"] = run_explore_leg(gx, torch, W)
        progress("explore")
    if not args.no_batch:
        out.update(run_batch(gx, torch, W, args.batch_n, B=args.batch_bucket,
                             G=args.batch_subgroup, U=args.batch_kps))
        progress("batched")
    if not args.no_serve:
        out["served"] = run_serve(gx, torch, W, args.serve_n)
        progress("served")
    if not args.no_dup:
        out["duplication_sweep"] = dup_sweep_summary(run_dup_sweep(gx, torch, W))
        progress("duplication sweep")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        progress("cpu baseline")
        if not args.no_explore:
            out["cpu_baseline"]["explore"] = cpu_explore_baseline(W)
            out["cpu_baseline"]["explore_all_cores"] = cpu_explore_all_cores(W)
            progress("cpu explore baselines")
        if not args.no_batch:
            out["cpu_baseline"]["batched_all_cores"] = cpu_batch_all_cores(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
