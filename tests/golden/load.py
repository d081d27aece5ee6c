"""Reader for the key/value golden fixtures in this folder."""

import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()[:2]
            out[k] = float(v)
    return out
