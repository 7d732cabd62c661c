"""Loader for the stored 60-digit fixtures in tests/golden/."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_exact.json")


def load():
    with open(GOLDEN) as f:
        raw = json.load(f)
    out = {}
    for name, d in raw.items():
        conv = {k: np.array([[float.fromhex(v) for v in row] for row in d[k]]) for k in ("A", "Z", "Q", "R")}
        conv["Z"] = np.asfortranarray(conv["Z"])
        out[name] = dict(d, **conv)
    return out
