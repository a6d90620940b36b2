"""Write served_pool.txt: the exact exploration (Sec. 3) of every network of
the served workload's request pool, ``workloads.served_networks(256, 5)``
(random networks with reachable sizes spread log-uniformly over 1e4-1e8 and
1- to 4-word vectors), computed by the CPU oracle alone
(``oracle.explore_dense``).

One line per network:
  index words states transitions deadlocks dead_digest0 dead_digest1 levels...
Run from the repository root: ``python tests/golden/make_served_pool.py``
(several minutes on eight cores)."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "served_pool.txt")
POOL, SEED = 256, 5


def main() -> None:
    nets, targets, bounds = W.served_networks(POOL, SEED)
    t0 = time.time()
    lines = [
        f"# Exact BFS (Sec. 3) of workloads.served_networks({POOL}, {SEED}), written by",
        "# make_served_pool.py from oracle.explore_dense.  Columns: index words states",
        "# transitions deadlocks dead_digest0 dead_digest1 level_counts...",
    ]
    for i, net in enumerate(nets):
        r = oracle.explore_dense(net)
        lines.append(" ".join(str(x) for x in (
            i, r.words, r.n_states, r.n_transitions, r.n_deadlocks, r.dead_digest[0],
            r.dead_digest[1], *[int(v) for v in r.levels])))
        print(lines[-1][:100], flush=True)
    lines.insert(3, f"# ({time.time() - t0:.0f} s on {os.cpu_count()} cores)")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
