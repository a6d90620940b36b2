"""Write large_random_l8.txt: the exact exploration of the large plain-path
workload (12 processes of 64 declared local states, 8 live, out-degree 3,
32 labels of which 25% are 2-party rendezvous, seed 1, sink probability 0.15;
3-word vectors) computed by the CPU oracle alone (``oracle.explore_dense``, a
level-synchronous BFS over dense bitmaps, Sec. 3).

Run from the repository root: ``python tests/golden/make_large_random_l8.py``.
It needs about 26 GB of memory (three bitmaps over the 8^12 index space) and
several minutes on eight cores.  Every value written comes from the oracle."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_random_l8.txt")


def main() -> None:
    net = W.large_random_network(live=8)
    t0 = time.time()
    r = oracle.explore_dense(net, threads=int(os.environ.get("ORACLE_THREADS", "0")))
    secs = time.time() - t0
    lines = [
        "# Exact BFS (Sec. 3) of large_random_network(live=8): 12 processes x 64 declared",
        "# states, 8 live, out-degree 3, 32 labels, 25% rendezvous, seed 1, sink 0.15;",
        "# 3-word vectors.  Written by make_large_random_l8.py from oracle.explore_dense",
        f"# ({secs:.0f} s on {os.cpu_count()} cores).",
        f"states {r.n_states}",
        f"transitions {r.n_transitions}",
        f"levels {len(r.levels)}",
        "level_counts " + " ".join(str(int(x)) for x in r.levels),
        f"deadlocks {r.n_deadlocks}",
        f"digest {r.digest[0]} {r.digest[1]}",
        f"dead_digest {r.dead_digest[0]} {r.dead_digest[1]}",
        f"index_space {r.index_space}",
    ]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
