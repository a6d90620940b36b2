"""Write batch_1024_s11.txt: the exact exploration (Sec. 3) of every network of
the batched workload, ``workloads.batch_networks(1024, 11)`` (1024 random
networks of 3-10 processes with reachable sizes spread log-uniformly over
1e3-1e7), computed by the CPU oracle alone (``oracle.explore_dense``).

One line per network:
  index words states transitions deadlocks dead_digest0 dead_digest1 levels...
Run from the repository root: ``python tests/golden/make_batch_1024.py``."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_1024_s11.txt")
N, SEED = 1024, 11


def main() -> None:
    nets, _ = W.batch_networks(N, SEED)
    t0 = time.time()
    rows = []
    for i, net in enumerate(nets):
        r = oracle.explore_dense(net)
        rows.append(" ".join(str(x) for x in (
            i, r.words, r.n_states, r.n_transitions, r.n_deadlocks, r.dead_digest[0],
            r.dead_digest[1], *[int(v) for v in r.levels])))
    lines = [
        f"# Exact BFS (Sec. 3) of workloads.batch_networks({N}, {SEED}), written by",
        "# make_batch_1024.py from oracle.explore_dense.  Columns: index words states",
        "# transitions deadlocks dead_digest0 dead_digest1 level_counts...",
        f"# ({time.time() - t0:.0f} s on {os.cpu_count()} cores)",
    ] + rows
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"{len(rows)} networks, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
