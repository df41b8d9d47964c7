"""Reader for the hand-worked fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    fx = dict(motif=[], edges=[], tree=None, center=None, before=[])
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            vals = [int(v) for v in vals]
            if key == "motif":
                fx["motif"].append(tuple(vals))
            elif key == "edge":
                fx["edges"].append(tuple(vals))
            elif key == "before":
                fx["before"].append(tuple(vals))
            elif key == "tree":
                fx["tree"] = vals
            elif key in ("delta", "center", "expect_count", "expect_weight_slot0",
                         "expect_weight_slot1"):
                fx[key] = vals[0]
            elif key == "weight_of":
                fx[key] = tuple(vals)
            else:
                raise ValueError(f"{name}: unknown key {key}")
    e = np.array(fx["edges"], dtype=np.int64)
    fx["src"] = e[:, 0].astype(np.int32)
    fx["dst"] = e[:, 1].astype(np.int32)
    fx["t"] = e[:, 2].astype(np.int64)
    fx["n"] = int(max(e[:, 0].max(), e[:, 1].max()) + 1)
    return fx
