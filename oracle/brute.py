"""Independent brute-force Tersoff energy (test infrastructure).

O(N^3), numpy, no neighbour list: for every atom i and every other atom j
(minimum image, or open boundaries when ``box`` is None) with r_ij < R+D,
zeta_ij sums over every k distinct from i and j with r_ik < R+D, then
E = 1/2 sum_i sum_j f_C(r_ij) [f_R(r_ij) + b_ij f_A(r_ij)]   (Eq. 1-3).

It is written separately from the C oracle (different language, different
loop structure) so that the two pin each other.  Forces are checked against
finite differences of this energy in the tests.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("A", "B", "lambda1", "lambda2", "lambda3", "beta", "eta",
          "c", "d", "h", "gamma", "R", "D", "m")


def _param(table, ti, tj, tk):
    e = np.asarray(table)[ti, tj, tk]
    return dict(zip(FIELDS, (float(v) for v in e)))


def _fc(r, p):
    if r < p["R"] - p["D"]:
        return 1.0
    if r < p["R"] + p["D"]:
        return 0.5 * (1.0 - math.sin(math.pi * (r - p["R"]) / (2.0 * p["D"])))
    return 0.0


def _g(cos_t, p):
    c2, d2 = p["c"] ** 2, p["d"] ** 2
    return p["gamma"] * (1.0 + c2 / d2 - c2 / (d2 + (p["h"] - cos_t) ** 2))


def energy(pos, types, box, table) -> float:
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types)
    n = pos.shape[0]
    total = 0.0
    for i in range(n):
        disp = pos - pos[i]
        if box is not None:
            L = np.asarray(box, dtype=np.float64)
            disp = disp - L * np.round(disp / L)
        dist = np.sqrt((disp ** 2).sum(axis=1))
        for j in range(n):
            if j == i:
                continue
            pij = _param(table, types[i], types[j], types[j])
            rij = dist[j]
            if not rij < pij["R"] + pij["D"]:
                continue
            zeta = 0.0
            for k in range(n):
                if k == i or k == j:
                    continue
                pk = _param(table, types[i], types[j], types[k])
                rik = dist[k]
                if not rik < pk["R"] + pk["D"]:
                    continue
                cos_t = float(disp[j] @ disp[k]) / (rij * rik)
                arg = (pk["lambda3"] * (rij - rik)) ** int(pk["m"])
                zeta += _fc(rik, pk) * _g(cos_t, pk) * math.exp(arg)
            bij = (1.0 + pij["beta"] ** pij["eta"] * zeta ** pij["eta"]) ** (-1.0 / (2.0 * pij["eta"]))
            fr = pij["A"] * math.exp(-pij["lambda1"] * rij)
            fa = -pij["B"] * math.exp(-pij["lambda2"] * rij)
            total += 0.5 * _fc(rij, pij) * (fr + bij * fa)
    return total


def neighbors(pos, box, rcut: float):
    """O(N^2) neighbour rows in numpy (list of sorted int arrays)."""
    pos = np.asarray(pos, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)
    rows = []
    for i in range(pos.shape[0]):
        d = pos - pos[i]
        d = d - L * np.round(d / L)
        r2 = (d ** 2).sum(axis=1)
        sel = np.nonzero(r2 < rcut * rcut)[0]
        rows.append(sel[sel != i])
    return rows
