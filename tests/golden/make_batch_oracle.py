"""Write the oracle's answers for the 4,096-graph uneven batch.

Every instance of the batch (n uniform in [50, 800], mean degree uniform in
[4, 12]; 75% G(n, p), 25% with a planted cover of 0.3 n) is solved by the
sequential CPU oracle with a node limit of CAP tree nodes.  Each output line
is

    index n m kind status size nodes sha

where status is "exact" (size is MVC) or "cap" (the oracle stopped at the
limit; size is -1), and sha is the first 16 hex digits of the SHA-256 of the
instance's CSR, so a test can tell that the generator still makes the same
graph.  Only the oracle computes the values.

    python tests/golden/make_batch_oracle.py [processes]
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

CAP = 200_000
COUNT = 4096
SEED = 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch4096_oracle.txt")


def solve(i: int):
    from paper_2512_18334_amd import graphgen as gg
    import oracle
    g = gg.config4_instance(i, SEED)
    kind = g.name.split("_", 1)[1]
    try:
        r = oracle.mvc(g, node_limit=CAP)
        status, size, nodes = "exact", r["size"], r["nodes"]
    except oracle.OracleLimit:
        status, size, nodes = "cap", -1, CAP
    return i, g.n, g.m, kind, status, size, nodes, gg.sha256(g)[:16]


def main() -> None:
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    import oracle
    oracle.build()
    t0 = time.time()
    rows = [None] * COUNT
    with mp.Pool(procs) as pool:
        # from the last index down (the order does not matter)
        for done, r in enumerate(pool.imap_unordered(solve, range(COUNT - 1, -1, -1)), 1):
            rows[r[0]] = r
            if done % 256 == 0:
                print(f"{done}/{COUNT} after {time.time() - t0:.0f} s", flush=True)
    exact = sum(1 for r in rows if r[4] == "exact")
    with open(OUT, "w") as f:
        f.write(f"# uneven batch: {COUNT} instances, seed {SEED}; oracle node limit {CAP}\n")
        f.write(f"# {exact} exact, {COUNT - exact} at the limit; written by "
                f"tests/golden/make_batch_oracle.py\n")
        f.write("# index n m kind status size nodes sha\n")
        for r in rows:
            f.write(" ".join(str(x) for x in r) + "\n")
    print(f"wrote {OUT}: {exact} exact of {COUNT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
