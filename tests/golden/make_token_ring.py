"""Write token_ring_13_15.txt: the exact exploration (Sec. 3) of the Token Ring
of 13, 14 and 15 nodes (Table 1, right; two-word vectors), computed by the CPU
oracle alone (``oracle.explore_dense``): states, transitions, deadlocks,
digest of the reachable set and every level count.

One line per ring:  nodes states transitions deadlocks digest0 digest1 levels...
Run from the repository root: ``python tests/golden/make_token_ring.py``
(about 12 GB of memory for the 15-node ring)."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "token_ring_13_15.txt")


def main() -> None:
    t0 = time.time()
    rows = []
    for n in (13, 14, 15):
        r = oracle.explore_dense(W.token_ring(n))
        rows.append(" ".join(str(x) for x in (n, r.n_states, r.n_transitions, r.n_deadlocks,
                                             r.digest[0], r.digest[1],
                                             *[int(v) for v in r.levels])))
        print(rows[-1][:100], flush=True)
    lines = ["# Exact BFS (Sec. 3) of workloads.token_ring(n), n = 13..15, written by",
             "# make_token_ring.py from oracle.explore_dense.  Columns: nodes states",
             "# transitions deadlocks digest0 digest1 level_counts...",
             f"# ({time.time() - t0:.0f} s on {os.cpu_count()} cores)"] + rows
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
