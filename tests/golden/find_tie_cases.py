"""Write tie_cases.tsv: small inputs on which the traceback's gap rule matters.

Lists seeded random pairs whose canonical alignment changes when the gap
rule "open here beats extend" is replaced by "extend beats open" for
insertions or for deletions (found by
exhaustive enumeration in tests/brute.py).  Only inputs are stored; the
tests re-derive the expected alignment by enumeration each time.
Run from the repository root: python tests/golden/find_tie_cases.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import brute  # noqa: E402


def decisions_extend_first(ops, forced_lead_ins, kind):
    # flip the in-gap choice: open(0) <-> extend(1); match-state tokens unchanged
    out, k, lead = [], len(ops), 0
    if forced_lead_ins:
        while lead < len(ops) and ops[lead] == brute.OP_I:
            lead += 1
    while k > lead:
        op = ops[k - 1]
        if op == brute.OP_M:
            out.append(1)
            k -= 1
            continue
        L = 0
        while k - L > lead and ops[k - 1 - L] == op:
            L += 1
        if op == kind:
            out += [2 if op == brute.OP_D else 3] + [0] * (L - 1) + [1]
        else:
            out += [2 if op == brute.OP_D else 3] + [1] * (L - 1) + [0]
        k -= L
    return tuple(out + [0])


def main():
    rng = np.random.default_rng(140204876)
    rows = []
    for sc, kind in [((3, 0, 2, 1), brute.OP_I), ((2, -3, 5, 2), brute.OP_I), ((1, -1, 1, 1), brute.OP_I),
                     ((5, -4, 2, 1), brute.OP_D), ((4, -2, 1, 1), brute.OP_D), ((3, -3, 1, 2), brute.OP_D)]:
        for mode in (0, 1):
            found = 0
            for _ in range(6000):
                if kind == brute.OP_D:  # deletion ties need a window longer than the read
                    m, n = int(rng.integers(2, 5)), int(rng.integers(4, 9))
                else:
                    m, n = int(rng.integers(2, 7)), int(rng.integers(2, 7))
                q = rng.integers(0, 4, m, dtype=np.uint8)
                r = rng.integers(0, 4, n, dtype=np.uint8)
                a = brute.canonical(q, r, mode, sc)
                keep = brute.decisions
                brute.decisions = lambda ops, forced_lead_ins: decisions_extend_first(ops, forced_lead_ins, kind)
                try:
                    b = brute.canonical(q, r, mode, sc)
                finally:
                    brute.decisions = keep
                if a != b:
                    rows.append((mode, sc, q, r))
                    found += 1
                    if found == 4:
                        break
    with open(os.path.join(HERE, "tie_cases.tsv"), "w") as f:
        f.write("# inputs where gap open-vs-extend ties change the canonical traceback\n")
        f.write("# mode\tmatch,mismatch,open,extend\tread\twindow\n")
        for mode, sc, q, r in rows:
            f.write("%s\t%s\t%s\t%s\n" % ("sg" if mode == 0 else "local", ",".join(map(str, sc)),
                                           "".join("ACGT"[x] for x in q), "".join("ACGT"[x] for x in r)))


if __name__ == "__main__":
    main()
