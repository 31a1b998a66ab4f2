"""Writes closed_form_targets.json: the exact station values of the measured
workloads, computed by the oracle's closed forms only (the benchmark reads
them to state each kernel's error against the exact solution; the oracle
itself is never run by the benchmark's GPU legs).

  cfg2   SI prism: u, g_z and the central difference of u at h = 2 m
  cfg3   128^3 voxel grid of 5 prisms: u (the grid holds the prisms exactly)
  cfg4   the 32 voxel models: u at every station of every model

Each model's voxel grid is voxel-aligned with its prisms, so the potential of
the grid equals the prisms' closed form; the boundary data is that closed
form, so it is also the exact solution inside the box.

  python tests/golden/make_targets.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1709_07469_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "closed_form_targets.json")


def potential(prisms, G, P):
    return float(sum(oracle.prism_potential(q[:3], q[3:6], q[6], G, P) for q in np.asarray(prisms).reshape(-1, 7)))


def gz(prisms, G, P):
    return float(sum(oracle.prism_gz(q[:3], q[3:6], q[6], G, P) for q in np.asarray(prisms).reshape(-1, 7)))


def targets():
    c2 = W.cfg2()
    h = c2.h
    up, gzs, fd = [], [], []
    for P in c2.stations:
        up.append(potential(c2.prisms, c2.G, P))
        gzs.append(gz(c2.prisms, c2.G, P))
        a = P + np.array([0.0, 0.0, h])
        b = P - np.array([0.0, 0.0, h])
        fd.append((potential(c2.prisms, c2.G, a) - potential(c2.prisms, c2.G, b)) / (2.0 * h))
    c3 = W.cfg3()
    u3 = [potential(c3.model_prisms, c3.G, P) for P in c3.stations]
    u4 = [[potential(m.model_prisms, m.G, P) for P in m.stations] for m in W.cfg4()]
    return {"cfg2": {"u": up, "gz": gzs, "gz_fd_h": fd, "h": h}, "cfg3": {"u": u3}, "cfg4": {"u": u4}}


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(targets(), f)
        f.write("\n")
    print(OUT)
