"""Graph sizes across correlation orders and degrees (host only).

    python -m paper_2202_04140_amd.counts [--group o3|torus] [--p 1|2|inf]
                                          [--nu 3 4 5] [--degrees 4 6 8] [--max-seconds 30]

Builds the DAG with Algorithm 1 and with Algorithm 2 (n = 2) for every
(nu, D) and prints |K|, the node count #V, the auxiliary count #A and the
ratio #A / #V of each (the quantity the paper's numerical tests plot, Sec. 3.4).
For O(3) the radial and angular cutoffs are n_max = l_max = D.  A row is
skipped once one (nu, D) took longer than --max-seconds, since the p = 2 and
p = infinity sets grow quickly with D.
"""

from __future__ import annotations

import argparse
import math
import sys
import time

from . import GROUP_O3, GROUP_TORUS, Graph


def sizes(group: int, nu: int, D: int, p: float, algorithm: int, alg_n: int = 2) -> dict:
    """|K|, #V and #A of one host-only graph."""
    nl = D if group == GROUP_O3 else 0
    g = Graph(nu, D, nl, nl, group=group, degree_p=p, algorithm=algorithm, alg_n=alg_n, host_only=True)
    s = g.stats()
    return {"K": s["n_k"], "V": s["n_nodes"], "A": s["n_aux"]}


def table(group: int, p: float, nus, degrees, max_seconds: float = 30.0):
    """Rows (nu, D, |K|, #V1, #A1, #A1/#V1, #V2, #A2, #A2/#V2) for Algorithm 1 and 2."""
    rows = []
    for nu in nus:
        for D in degrees:
            t = time.perf_counter()
            a1 = sizes(group, nu, D, p, 1)
            a2 = sizes(group, nu, D, p, 2)
            rows.append((nu, D, a1["K"], a1["V"], a1["A"], a1["A"] / a1["V"], a2["V"], a2["A"], a2["A"] / a2["V"]))
            if time.perf_counter() - t > max_seconds:
                break
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--group", choices=["o3", "torus"], default="o3")
    ap.add_argument("--p", default="1", choices=["1", "2", "inf"])
    ap.add_argument("--nu", type=int, nargs="+", default=[3, 4, 5])
    ap.add_argument("--degrees", type=int, nargs="+", default=[4, 6, 8, 10, 12])
    ap.add_argument("--max-seconds", type=float, default=30.0)
    a = ap.parse_args(argv)
    group = GROUP_O3 if a.group == "o3" else GROUP_TORUS
    p = math.inf if a.p == "inf" else float(a.p)
    print("| nu | D | |K| | #V (Alg. 1) | #A | #A/#V | #V (Alg. 2, n = 2) | #A | #A/#V |")
    print("|---|---|---|---|---|---|---|---|---|")
    for r in table(group, p, a.nu, a.degrees, a.max_seconds):
        print(f"| {r[0]} | {r[1]} | {r[2]} | {r[3]} | {r[4]} | {r[5]:.4f} | {r[6]} | {r[7]} | {r[8]:.4f} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
