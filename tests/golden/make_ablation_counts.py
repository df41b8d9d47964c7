"""Writes ablation_counts.txt: exact counts (oracle brute force, Def.
"temporal match") of the constraint-ablation workload, the reference for the
estimates' errors.  Calls only the oracle and the input generator.

    python tests/golden/make_ablation_counts.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle as O  # noqa: E402
from paper_2507_20441_amd import workloads as W  # noqa: E402


def main():
    g = W.ablation_graph()
    og = O.Graph(g.src, g.dst, g.t, g.n)
    lines = ["# exact counts of the constraint-ablation workload (workloads.ablation_graph,",
             "# delta = ABLATION['delta']), by oracle brute force; written by make_ablation_counts.py",
             f"# graph n={g.n} m={g.m}"]
    for name in W.ABLATION["motifs"]:
        c = og.brute_count(O.make_motif(W.MOTIFS[name], W.ABLATION["delta"]))
        lines.append(f"count {name} {c}")
    with open(os.path.join(HERE, "ablation_counts.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
