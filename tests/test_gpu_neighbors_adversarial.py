"""GPU neighbour lists on inputs built to sit where the search's
single-precision pre-test is tight (Section 2: the full list with skin),
compared bit for bit with the oracle: pairs at the list radius +- a few FP64
ulps and at the pre-test's sure-accept and rejection radii +- a few float
ulps, centres at 0 and at L - ulp and unwrapped by +-L, +-2L, displacement
components within ulps of L/2 in boxes of exactly twice the list radius, and
grids with one, two and three cells per axis.  The construction of the
borderline radii follows tests/test_search_pretest.py, which checks the same
bound against an emulation of the pre-test on the CPU."""
import zlib

import numpy as np
import pytest

import oracle
from paper_1710_00882_amd import workloads as W

from gpu_helpers import say, to_dev
from test_search_pretest import adversarial_pairs, half_box_pairs, pretest

pytestmark = pytest.mark.gpu

RC = W.SI["R"] + W.SI["D"] + W.SKIN   # list radius of the silicon set: 4.0 A

# (box, designed pairs per system, systems): few enough atoms per system that
# rows stay below the 23 candidates the search's first pass holds, so the
# pre-test, not the wavefront-per-row pass, decides them
BOXES = {
    "three_cells": (np.array([12.0 + 1e-6, 12.5, 13.1]), 36, 12),
    "large": (np.array([61.3, 58.9, 44.2]), 900, 1),
    "two_cells": (np.array([8.0 + 1e-8, 10.862, 9.5]), 15, 24),
    "one_cell_exact": (np.array([8.0, 8.0, 8.0]), 9, 30),
    "mixed_axes": (np.array([8.0, 12.4, 40.0]), 72, 8),
}


def systems(name):
    L, npairs, nsys = BOXES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    _, _, _, sure, lim = pretest(np.zeros((1, 3)), np.zeros((1, 3)), L, RC)
    for _ in range(nsys):
        k = npairs if L.min() >= 3 * RC else (npairs + 1) // 2
        xi, xj = adversarial_pairs(L, RC, sure, lim, max(1, k // 3), rng, edge_prob=0.15)
        if L.min() < 3 * RC:
            a, b = half_box_pairs(L, RC, max(1, k // 3), rng)
            xi, xj = np.concatenate([xi, a]), np.concatenate([xj, b])
        yield W.System(np.concatenate([xi, xj]), np.zeros(2 * len(xi), np.int32), L), xi, xj


@pytest.mark.parametrize("name", list(BOXES))
def test_adversarial_lists_bit_exact(name):
    import torch
    from paper_1710_00882_amd import Tersoff
    L = BOXES[name][0]
    table = W.si_table()
    m = Tersoff(table)
    near = below = above = entries = 0
    for s, xi, xj in systems(name):
        p, t = to_dev(s)
        m.build_neighbors(p, t, s.box, skin=W.SKIN)
        torch.cuda.synchronize()
        off, idx = m.neighbors()
        ooff, oidx = oracle.neighbors(s.pos, s.box, RC)
        assert np.array_equal(off, ooff), f"{name}: row lengths differ"
        assert np.array_equal(idx, oidx), f"{name}: rows differ"
        d = xj - xi
        d -= np.rint(d / L) * L
        r = np.linalg.norm(d, axis=1)
        near += int(np.sum(np.abs(r - RC) < 1e-12))
        below += int(np.sum(r < RC))
        above += int(np.sum(r >= RC))
        entries += len(oidx)
    say(f"[nbr-adv] {name}: {entries} entries bit-exact; designed pairs {below} inside, {above} outside, "
        f"{near} within 1e-12 A of the radius")
    assert below > 0 and above > 0
