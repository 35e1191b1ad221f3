"""Small text fixtures; each file states where its values come from."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load_edge_rows():
    """(records as R16 structured array, expected keys, expected cols[4, G]) from edge_rows.txt."""
    recs, exp = [], []
    for line in open(os.path.join(HERE, "edge_rows.txt")):
        parts = line.split()
        if not parts or parts[0].startswith("#"):
            continue
        if parts[0] == "R":
            recs.append((int(parts[1]), int(parts[2])))
        elif parts[0] == "E":
            exp.append([int(x) for x in parts[1:]])
    r = np.empty(len(recs), dtype=[("key", "<u8"), ("v", "<i8")])
    r["key"] = [k for k, _ in recs]
    r["v"] = [v for _, v in recs]
    keys = np.array([e[0] for e in exp], dtype=np.uint64)
    cols = np.array([[e[j] for e in exp] for j in range(1, 5)], dtype=np.int64)
    return r, keys, cols
