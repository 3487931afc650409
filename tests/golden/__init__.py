"""Fixtures transcribed from the paper (each file states its source)."""
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def load_fig1():
    """Parse fig1_example.txt; returns a dict with 0-based pattern arrays and
    the printed symbolic data (1-based labels, as in the paper)."""
    out = {"snodes": {1: [], 2: []}}
    with open(os.path.join(_HERE, "fig1_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":") if not line.startswith("snode") else ("snode", None, line)
            if key == "n":
                out["n"] = int(rest)
            elif key == "entries":
                out["entries"] = [tuple(int(v) for v in e.split(",")) for e in rest.split()]
            elif key in ("parent", "degree", "representatives"):
                out[key] = [int(v) for v in rest.split()]
            elif key == "snode":
                parts = rest.split()
                part, rep = int(parts[1]), int(parts[2])
                fields = dict(p.split("=") for p in parts[3:])
                nset = [int(v) for v in fields["N"].split(",") if v]
                aset = [int(v) for v in fields["A"].split(",") if v]
                out["snodes"][part].append((rep, nset, aset, int(fields["parent"])))
    n = out["n"]
    cols = [[j] for j in range(n)]
    for (i, j) in out["entries"]:
        cols[j - 1].append(i - 1)
    colptr = np.zeros(n + 1, dtype=np.int64)
    rows = []
    for j in range(n):
        r = sorted(cols[j])
        rows.extend(r)
        colptr[j + 1] = colptr[j] + len(r)
    out["pattern"] = (n, colptr, np.array(rows, dtype=np.int32))
    return out
