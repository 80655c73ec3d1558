"""Reader of the stored oracle values under tests/golden/."""
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_cube():
    causal, ent, mv = None, [], []
    with open(os.path.join(HERE, "cube_S4_T2.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            k = line.split()
            if k[0] == "causal":
                causal = int(k[1])
            elif k[0] == "entry":
                ent.append((int(k[1]), int(k[2]), float(k[3]), float(k[4])))
            elif k[0] == "matvec":
                mv.append((int(k[1]), float(k[2]), float(k[3])))
    rows = np.array([e[0] for e in ent], dtype=np.int32)
    cols = np.array([e[1] for e in ent], dtype=np.int32)
    vals = np.array([e[2] for e in ent])
    mags = np.array([e[3] for e in ent])
    mv.sort()
    y = np.array([v[1] for v in mv])
    ybound = np.array([v[2] for v in mv])
    return causal, rows, cols, vals, mags, y, ybound
