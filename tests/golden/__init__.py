"""Readers of the paper's worked examples stored as small text fixtures."""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load_tab2():
    """Fig. 1 / Tab. 2 fixture: coordinates [10, 2] (float64), eps, k, the
    printed table [10, 8] (nn, nn_rank, mean, mean_rank, indeg, indeg_rank,
    kmean, kmean_rank) and the Fig. 1b edges {point: set(neighbours)}, all
    with 0-based ids."""
    params, rows, edges = {}, [], {}
    with open(os.path.join(HERE, "tab2_fig1.txt")) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "P":
                params[t[1]] = float(t[2])
            elif t[0] == "T":
                rows.append([float(v) for v in t[1:]])
            elif t[0] == "E":
                edges[int(t[1]) - 1] = {int(v) - 1 for v in t[2:]}
    rows = np.asarray(rows)
    coords = rows[:, 1:3]
    table = rows[:, 3:]
    return coords, params["eps"], int(params["k"]), table, edges


def load_fig3():
    """Fig. 3 fixture: query (2,), and [(eps, set of 0-based ids)]."""
    q, sets = None, []
    with open(os.path.join(HERE, "fig3.txt")) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "Q":
                q = np.array([float(t[1]), float(t[2])])
            elif t[0] == "S":
                sets.append((float(t[1]), {int(v) - 1 for v in t[2:]}))
    return q, sets


def exact_fp32_variant(coords, scale=100.0, shift=64.0, denom=512.0):
    """Map the Fig. 1 coordinates to x' = (100 x + 64) / 512.  All of them
    become dyadic rationals in [0, 1] whose squared differences and sums are
    exact in float32, so float32 and float64 see identical distances (the
    exact tie of point 1's third neighbour is then resolved only by id)."""
    ints = np.round(scale * np.asarray(coords, dtype=np.float64))
    return ((ints + shift) / denom).astype(np.float32)


def load_eps_select_example():
    """Sec. 3.5.2 example: n, the three top-n sets, and the printed U^min and
    U^max."""
    sets, n, umin, umax = [], 0, None, None
    with open(os.path.join(HERE, "eps_select_example.txt")) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "N":
                n = int(t[1])
            elif t[0] == "S":
                sets.append([int(v) for v in t[2:]])
            elif t[0] == "UMIN":
                umin = [float(v) for v in t[1:]]
            elif t[0] == "UMAX":
                umax = [float(v) for v in t[1:]]
    return n, sets, umin, umax
