"""Readers of the text fixtures in tests/golden (values printed in the paper)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def worked_example():
    """Section 2.2 worked example: returns a dict of numpy arrays / ints."""
    lines = [ln.strip() for ln in open(os.path.join(HERE, "worked_example_n3.txt"))
             if ln.strip() and not ln.startswith("#")]
    out = {"solutions": []}
    k = 0
    while k < len(lines):
        tok = lines[k].split()
        if tok[0] == "n":
            out["n"] = int(tok[1]); k += 1
        elif tok[0] in ("H", "D", "C", "G"):
            rows = 3 if tok[0] in ("H", "D") else 9
            out[tok[0]] = np.array([[int(v) for v in lines[k + 1 + r].split()] for r in range(rows)],
                                   dtype=np.int64)
            k += 1 + rows
        elif tok[0] in ("pc", "pg"):
            out[tok[0]] = int(tok[1]); k += 1
        elif tok[0] == "solution":
            parts = [p.split() for p in lines[k][len("solution"):].split(";")]
            out["solutions"].append(dict(
                sigma=[int(v) for v in parts[0]], x=np.array([int(v) for v in parts[1]], np.uint8),
                f=int(parts[2][0]), xCx=int(parts[3][0]), xGx=int(parts[4][0]), g=int(parts[5][0])))
            k += 1
        else:
            raise ValueError(lines[k])
    return out
