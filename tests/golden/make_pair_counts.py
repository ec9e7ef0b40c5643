"""Write tests/golden/pair_counts.json from the CPU oracle's brute-force
enumeration of the interaction rule (calls only oracle/).

Run from the repository root:  python tests/golden/make_pair_counts.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

CASES = [(0, 0.4), (1, 0.4), (2, 0.4), (3, 0.4), (4, 0.4), (1, 0.5), (2, 0.5), (2, 0.7), (2, 0.34), (2, 0.9)]


def main():
    out = {"source": "oracle.pair_counts (brute-force rule enumeration)", "counts": {}}
    for L, theta in CASES:
        p2p, m2l = O.pair_counts(L, theta)
        out["counts"][f"L{L}_theta{theta}"] = {"L": L, "theta": theta, "p2p": p2p,
                                               "m2l": [int(x) for x in m2l]}
        print(L, theta, p2p, list(m2l), flush=True)
    with open(os.path.join(HERE, "pair_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
