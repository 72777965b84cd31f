"""Write the small temporal-path fixtures in this folder.

The paper prints no worked example (its example graph of §1 is a figure
without values), so these fixtures are produced by exhaustive enumeration
of time-respecting walks (``oracle.brute_force``), following the path
definitions of §2.1-§2.3 and the query interval of Alg. 2.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import tiny_graph  # noqa: E402

CASES = [
    # name, seed, n, m, t_max, lam_max, source, t_alpha, t_omega
    ("dense_ties", 11, 6, 14, 6, 2, 0, 0, 12),
    ("narrow_window", 12, 7, 16, 10, 3, 1, 3, 9),
    ("multi_edges", 13, 4, 18, 8, 3, 2, 1, 14),
    ("sparse", 14, 9, 10, 20, 5, 3, 0, 30),
    ("late_start", 15, 7, 16, 12, 2, 0, 8, 16),
]


def main():
    for (name, seed, n, m, tmax, lmax, s, ta, tw) in CASES:
        g = tiny_graph(seed, n=n, m=m, t_max=tmax, lam_max=lmax)
        edges = [(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(g.src, g.dst, g.t, g.lam)]
        s = int(s) if int(np.bincount(g.src, minlength=n)[s]) else int(g.src[0])
        ea, ld, fa = oracle.brute_force(n, edges, s, ta, tw)
        doc = {
            "source_of_values": "oracle.brute_force (enumeration of time-respecting walks; "
                                "definitions of paper sections 2.1-2.3, query interval of Alg. 2)",
            "n": n, "edges": edges, "source": s, "t_alpha": ta, "t_omega": tw,
            "ea": ea, "ld": ld, "fastest": fa,
        }
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(doc, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
