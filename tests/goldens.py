"""Parser for the hand-derived fixtures under tests/golden/.

Line formats (``#`` starts a comment):
  d <float>                         default threshold of the file
  point <x> <y> <z>                 one point, in index order
  case min=<a> max=<b> k=<k> labels=<l0,l1,...>
  dcase d=<float|next(float)> min=<a> max=<b> k=<k> labels=<...>
  raw_skip <l0,l1,...> / raw_all <...>    raw Alg. 1 label values
  pair x y z  x y z  d=<float|next(float)> joined=<0|1>
"""

from __future__ import annotations

import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse_float32(tok: str) -> float:
    if tok.startswith("next(") and tok.endswith(")"):
        v = np.float32(tok[5:-1])
        return float(np.nextafter(v, np.float32(np.inf)))
    return float(np.float32(tok))


def _kv(tokens):
    out = {}
    for t in tokens:
        k, v = t.split("=", 1)
        out[k] = v
    return out


def load(name: str) -> dict:
    path = os.path.join(GOLDEN_DIR, name)
    res = {"d": None, "points": [], "cases": [], "pairs": [], "raw_skip": None, "raw_all": None}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "d":
                res["d"] = parse_float32(tok[1])
            elif tok[0] == "point":
                res["points"].append([float(v) for v in tok[1:4]])
            elif tok[0] in ("case", "dcase"):
                kv = _kv(tok[1:])
                res["cases"].append(dict(
                    d=parse_float32(kv["d"]) if "d" in kv else None,
                    min=int(kv["min"]), max=int(kv["max"]), k=int(kv["k"]),
                    labels=np.array([int(v) for v in kv["labels"].split(",")], dtype=np.int32)))
            elif tok[0] in ("raw_skip", "raw_all"):
                res[tok[0]] = np.array([int(v) for v in tok[1].split(",")], dtype=np.int64)
            elif tok[0] == "pair":
                a = [float(v) for v in tok[1:4]]
                b = [float(v) for v in tok[4:7]]
                kv = _kv(tok[7:])
                res["pairs"].append(dict(a=a, b=b, d=parse_float32(kv["d"]),
                                         joined=int(kv["joined"])))
            else:
                raise ValueError("unknown fixture line: %r" % line)
    res["points"] = np.array(res["points"], dtype=np.float32).reshape(-1, 3)
    for c in res["cases"]:
        if c["d"] is None:
            c["d"] = res["d"]
    return res


def all_cases():
    """(fixture name, xyz, d, min, max, k, labels) for every labelled case."""
    out = []
    for name in ("chain4.txt", "filter9.txt", "fig3_extremes.txt"):
        g = load(name)
        for c in g["cases"]:
            out.append((name, g["points"], c["d"], c["min"], c["max"], c["k"], c["labels"]))
    for name in ("threshold.txt", "predicate_order.txt"):
        g = load(name)
        for i, p in enumerate(g["pairs"]):
            xyz = np.array([p["a"], p["b"]], dtype=np.float32)
            lab = np.array([0, 0] if p["joined"] else [0, 1], dtype=np.int32)
            out.append(("%s#%d" % (name, i), xyz, p["d"], 1, 2, 1 if p["joined"] else 2, lab))
    return out

