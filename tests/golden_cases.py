"""Reader for the hand-worked point-source fixtures in tests/golden/."""
import os
from fractions import Fraction

import numpy as np

from synth import Geometry

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_point_sources(name="point_source.txt"):
    cases, cur = [], None
    with open(os.path.join(HERE, name)) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = {"name": tok[1], "taps": {}}
            elif tok[0] == "grid":
                cur["grid"] = [int(tok[1]), int(tok[2]), int(tok[3]), int(tok[4]), float(tok[5]),
                               (float(tok[6]), float(tok[7]), float(tok[8]))]
            elif tok[0] == "sensor":
                cur["sensor"] = [float(t) for t in tok[1:4]]
            elif tok[0] == "timing":
                cur["timing"] = [int(tok[1])] + [float(t) for t in tok[2:6]]
            elif tok[0] == "pixel":
                cur["pixel"] = int(tok[1])
            elif tok[0] == "tap":
                cur["taps"][int(tok[1])] = float(Fraction(tok[2]))
            elif tok[0] == "end":
                nd, nx, ny, nz, h, ctr = cur["grid"]
                K, dt, t0, c, rmin = cur["timing"]
                sens = np.array([cur["sensor"][:nd]], dtype=np.float64)
                cur["geom"] = Geometry(nd, nx, ny, nz, h, ctr, sens, K, dt, t0, c, rmin)
                cases.append(cur)
                cur = None
    return cases
