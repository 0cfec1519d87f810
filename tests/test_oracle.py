"""Pins of the FP64 CPU oracle against what the mathematics fixes.

The paper prints no worked numerical example, so every pin is a closed form
of a symmetric structure, an identity (F = -grad E, W = -dE/d strain), an
invariance, or agreement with the independent O(N^3) brute-force energy.
Each is chosen so that a plausible slip in the oracle fails it:
  - missing 1/2 of Eq. (1) or k = j kept in Eq. (3): closed forms, brute force;
  - a dropped or mis-signed derivative term: finite-difference forces, with
    atoms placed in the cutoff switching zone and lambda3 != 0 (m = 1, 3);
  - wrong parameter entry for mixed species: two-species brute force;
  - virial sign or index slip: strain finite differences;
  - neighbour list: cell list == brute O(N^2), and == numpy rows.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as brute
from paper_1710_00882_amd import workloads as W

SI = W.SI


def fc(r, p=SI):
    if r < p["R"] - p["D"]:
        return 1.0
    if r < p["R"] + p["D"]:
        return 0.5 - 0.5 * math.sin(math.pi / 2 * (r - p["R"]) / p["D"])
    return 0.0


def g(cos_t, p=SI):
    return p["gamma"] * (1 + p["c"] ** 2 / p["d"] ** 2 - p["c"] ** 2 / (p["d"] ** 2 + (cos_t - p["h"]) ** 2))


def bond(zeta, p=SI):
    return (1 + (p["beta"] * zeta) ** p["eta"]) ** (-1 / (2 * p["eta"]))


def pairV(r, zeta, p=SI):
    """f_C (f_R + b f_A): the bracket of Eq. (1) for one ordered pair."""
    return fc(r, p) * (p["A"] * math.exp(-p["lambda1"] * r) - bond(zeta, p) * p["B"] * math.exp(-p["lambda2"] * r))


BIG = np.array([100.0, 100.0, 100.0])


def cluster_eval(pos, table=None, types=None):
    table = W.si_table() if table is None else table
    pos = np.asarray(pos, dtype=np.float64) + 50.0
    types = np.zeros(len(pos), np.int32) if types is None else types
    return oracle.evaluate(pos, types, BIG, table)


# ------------------------------------------------------------ closed forms

def test_dimer_closed_form():
    for r in (2.35, 2.6, 2.7):       # below R - D: f_C = 1
        E, F, Wv = cluster_eval([[0, 0, 0], [r, 0, 0]])
        exact = SI["A"] * math.exp(-SI["lambda1"] * r) - SI["B"] * math.exp(-SI["lambda2"] * r)
        assert E == pytest.approx(exact, rel=1e-14)
        # F on the atom at +x is -dE/dr
        dE = -SI["lambda1"] * SI["A"] * math.exp(-SI["lambda1"] * r) + SI["lambda2"] * SI["B"] * math.exp(-SI["lambda2"] * r)
        assert F[1, 0] == pytest.approx(-dE, rel=1e-12)
        assert F[0, 0] == pytest.approx(dE, rel=1e-12)
        # virial of a pair: r * F_j along the bond
        assert Wv[0] == pytest.approx(-r * dE, rel=1e-12)


def test_dimer_switching_zone_midpoint():
    r = SI["R"]                     # f_C(R) = 1/2 exactly
    E, _, _ = cluster_eval([[0, 0, 0], [0, r, 0]])
    exact = 0.5 * (SI["A"] * math.exp(-SI["lambda1"] * r) - SI["B"] * math.exp(-SI["lambda2"] * r))
    assert E == pytest.approx(exact, rel=1e-13)
    E2, _, _ = cluster_eval([[0, 0, 0], [0, 0, SI["R"] + SI["D"] + 1e-9]])
    assert E2 == 0.0


def test_equilateral_trimer():
    r = 2.35
    pos = [[0, 0, 0], [r, 0, 0], [r / 2, r * math.sqrt(3) / 2, 0]]
    E, F, _ = cluster_eval(pos)
    # six ordered pairs, each with one k at 60 degrees: zeta = g(1/2)
    exact = 0.5 * 6 * pairV(r, g(0.5))
    assert E == pytest.approx(exact, rel=1e-13)
    assert np.abs(F.sum(axis=0)).max() < 1e-12


def test_linear_trimer():
    r = 2.35
    E, _, _ = cluster_eval([[0, 0, 0], [r, 0, 0], [2 * r, 0, 0]])
    # ends see only the middle atom (zeta = 0); the middle sees both ends at 180 degrees
    exact = 0.5 * (2 * pairV(r, 0.0) + 2 * pairV(r, g(-1.0)))
    assert E == pytest.approx(exact, rel=1e-13)


def diamond_energy_per_atom(a):
    rnn = a * math.sqrt(3) / 4
    return 0.5 * 4 * pairV(rnn, 3 * g(-1.0 / 3.0))


@pytest.mark.parametrize("cells", [(2, 2, 2), (3, 2, 4)])
def test_perfect_diamond(cells):
    a = W.SI_LATTICE
    s = W.diamond(*cells, a=a)
    E, F, Wv = oracle.evaluate(s.pos, s.types, s.box, W.si_table())
    assert E / s.n == pytest.approx(diamond_energy_per_atom(a), rel=1e-13)
    assert np.abs(F).max() < 1e-11
    # W_aa = -(a/3) dE/da per atom under uniform dilation; off-diagonals vanish
    h = 1e-3                          # five-point stencil
    f = diamond_energy_per_atom
    dEda = (-f(a + 2 * h) + 8 * f(a + h) - 8 * f(a - h) + f(a - 2 * h)) / (12 * h)
    for c in range(3):
        assert Wv[c] / s.n == pytest.approx(-a / 3 * dEda, rel=1e-8)
    assert np.abs(Wv[3:]).max() / s.n < 1e-12


def test_diamond_cohesive_energy_near_published_si():
    # Tersoff's Si(C) set gives a cohesive energy of about 4.63 eV at about 5.43 A
    e = diamond_energy_per_atom(W.SI_LATTICE)
    assert -4.64 < e < -4.62
    grid = np.linspace(5.40, 5.46, 601)
    amin = grid[np.argmin([diamond_energy_per_atom(a) for a in grid])]
    assert abs(amin - 5.432) < 2e-3


# ---------------------------------------------------- test parameter sets

def stress_table(m=1, lam3=1.3):
    """Si with lambda3 != 0 and a wide switching zone (many pairs in it)."""
    return W.table_from_species([dict(SI, lambda3=lam3, m=m, R=2.55, D=0.35)])


def stress_two_species(lam3=0.9):
    s0 = dict(SI, lambda3=lam3, R=2.55, D=0.35)
    s1 = dict(W.species_variant(s0, 0.9, 1.04), lambda3=0.5 * lam3, h=-0.3, c=8.0e4, eta=0.7)
    return W.table_from_species([s0, s1])


def jittered_cell(seed, ntypes=1, jitter=0.15):
    return W.diamond(2, 2, 2, jitter=jitter, seed=seed, ntypes=ntypes)


def random_cluster(n, seed, spread=2.2):
    """Small cluster with pair distances spread over the switching zone."""
    g_ = W.rng(seed)
    pts = [np.zeros(3)]
    while len(pts) < n:
        base = pts[g_.integers(len(pts))]
        v = g_.normal(size=3)
        cand = base + v / np.linalg.norm(v) * g_.uniform(spread, 2.85)
        if min(np.linalg.norm(cand - p) for p in pts) > 1.9:
            pts.append(cand)
    return np.array(pts)


# ------------------------------------------------------- brute force O(N^3)

@pytest.mark.parametrize("seed", [11, 12])
def test_brute_force_periodic(seed):
    s = jittered_cell(seed)
    for table in (W.si_table(), stress_table(1), stress_table(3)):
        E, _, _ = oracle.evaluate(s.pos, s.types, s.box, table)
        Eb = brute.energy(s.pos, s.types, s.box, table)
        assert E == pytest.approx(Eb, rel=1e-13, abs=1e-12)


def test_brute_force_two_species():
    s = jittered_cell(21, ntypes=2)
    for table in (W.two_species_table(), stress_two_species()):
        E, _, _ = oracle.evaluate(s.pos, s.types, s.box, table)
        Eb = brute.energy(s.pos, s.types, s.box, table)
        assert E == pytest.approx(Eb, rel=1e-13, abs=1e-12)


def test_brute_force_cluster():
    pos = random_cluster(9, seed=5)
    types = np.array([0, 1, 0, 1, 1, 0, 0, 1, 0], np.int32)
    for table, t in ((stress_table(1), None), (stress_table(3), None), (stress_two_species(), types)):
        E, _, _ = cluster_eval(pos, table, t)
        Eb = brute.energy(pos, np.zeros(len(pos), np.int32) if t is None else t, None, table)
        assert E == pytest.approx(Eb, rel=1e-13, abs=1e-12)


# ------------------------------------------------------ derivative identities

def fd_forces(pos, types, box, table, h=1e-5, atoms=None):
    out = np.zeros_like(pos)
    atoms = range(len(pos)) if atoms is None else atoms
    for i in atoms:
        for a in range(3):
            p = pos.copy(); p[i, a] += h
            ep = oracle.evaluate(p, types, box, table)[0]
            p[i, a] -= 2 * h
            em = oracle.evaluate(p, types, box, table)[0]
            out[i, a] = -(ep - em) / (2 * h)
    return out


@pytest.mark.parametrize("case", ["si", "lam3_m1", "lam3_m3", "two_species"])
def test_forces_are_minus_gradient(case):
    if case == "two_species":
        s = jittered_cell(31, ntypes=2, jitter=0.2)
        table = stress_two_species()
    else:
        s = jittered_cell(30, jitter=0.2)
        table = {"si": W.si_table(), "lam3_m1": stress_table(1), "lam3_m3": stress_table(3)}[case]
    E, F, _ = oracle.evaluate(s.pos, s.types, s.box, table)
    atoms = list(range(0, s.n, 7))
    Ffd = fd_forces(s.pos, s.types, s.box, table, atoms=atoms)
    err = np.abs(F[atoms] - Ffd[atoms]).max()
    assert err < 2e-6 * max(1.0, np.abs(F).max())


def test_cluster_forces_switching_zone():
    pos = random_cluster(8, seed=7) + 50.0
    types = np.zeros(len(pos), np.int32)
    table = stress_table(1)
    E, F, _ = oracle.evaluate(pos, types, BIG, table)
    Ffd = fd_forces(pos, types, BIG, table)
    assert np.abs(F - Ffd).max() < 2e-6 * max(1.0, np.abs(F).max())
    # zero net force and zero net torque for an isolated cluster
    assert np.abs(F.sum(axis=0)).max() < 1e-11
    torque = np.cross(pos - pos.mean(axis=0), F).sum(axis=0)
    assert np.abs(torque).max() < 1e-10


def test_virial_is_minus_strain_derivative_periodic():
    s = jittered_cell(40, jitter=0.2)
    table = stress_table(1)
    _, _, Wv = oracle.evaluate(s.pos, s.types, s.box, table)
    h = 1e-6
    for a in range(3):
        scale = np.ones(3); scale[a] += h
        ep = oracle.evaluate(s.pos * scale, s.types, s.box * scale, table)[0]
        scale[a] -= 2 * h
        em = oracle.evaluate(s.pos * scale, s.types, s.box * scale, table)[0]
        assert Wv[a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6, abs=1e-6)


def test_virial_shear_components_cluster():
    pos = random_cluster(8, seed=9)
    table = stress_table(3)
    _, _, Wv = cluster_eval(pos, table)
    h = 1e-6
    for comp, (a, b) in zip((3, 4, 5), ((0, 1), (0, 2), (1, 2))):
        def e(eps):
            G = np.eye(3); G[a, b] += eps
            return cluster_eval(pos @ G.T, table)[0]
        dE = (e(h) - e(-h)) / (2 * h)
        assert Wv[comp] == pytest.approx(-dE, rel=1e-6, abs=1e-6)


# -------------------------------------------------------------- invariances

def test_translation_and_image_invariance():
    s = jittered_cell(50)
    table = stress_table(1)
    E, F, Wv = oracle.evaluate(s.pos, s.types, s.box, table)
    shifted = s.pos + np.array([0.37, -1.1, 2.9])
    shifted[::3] += s.box                      # unwrapped images
    shifted[1::5] -= 2 * s.box
    E2, F2, W2 = oracle.evaluate(shifted, s.types, s.box, table)
    assert E2 == pytest.approx(E, rel=1e-13)
    assert np.abs(F2 - F).max() < 1e-10
    assert np.abs(W2 - Wv).max() < 1e-10
    assert np.abs(F.sum(axis=0)).max() < 1e-10


def test_rotation_invariance_cluster():
    pos = random_cluster(10, seed=3)
    table = stress_table(1)
    E, F, _ = cluster_eval(pos, table)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(0.3), -math.sin(0.3)], [0, math.sin(0.3), math.cos(0.3)]])
    Rm = Rz @ Rx
    E2, F2, _ = cluster_eval(pos @ Rm.T, table)
    assert E2 == pytest.approx(E, rel=1e-12)
    assert np.abs(F2 - F @ Rm.T).max() < 1e-10


def test_permutation_invariance():
    s = jittered_cell(60, ntypes=2)
    table = stress_two_species()
    E, F, Wv = oracle.evaluate(s.pos, s.types, s.box, table)
    perm = W.rng(1).permutation(s.n)
    E2, F2, W2 = oracle.evaluate(s.pos[perm], s.types[perm], s.box, table)
    assert E2 == pytest.approx(E, rel=1e-13)
    assert np.abs(F2 - F[perm]).max() < 1e-10
    assert np.abs(W2 - Wv).max() < 1e-10


def test_axis_permutation_invariance_periodic():
    s = W.diamond(3, 2, 2, jitter=0.1, seed=70)
    table = stress_table(1)
    E, F, Wv = oracle.evaluate(s.pos, s.types, s.box, table)
    order = [2, 0, 1]
    E2, F2, W2 = oracle.evaluate(s.pos[:, order], s.types, s.box[order], table)
    assert E2 == pytest.approx(E, rel=1e-13)
    assert np.abs(F2 - F[:, order]).max() < 1e-10
    assert np.allclose(W2[:3], Wv[:3][order], atol=1e-10)


# ------------------------------------------------------------ neighbour list

@pytest.mark.parametrize("cells,jitter,rcut", [((2, 2, 2), 0.1, 4.0), ((3, 2, 2), 0.3, 4.0),
                                                ((2, 2, 3), 0.05, 4.12), ((4, 3, 2), 0.2, 3.0)])
def test_cell_list_equals_brute(cells, jitter, rcut):
    s = W.diamond(*cells, jitter=jitter, seed=sum(cells))
    pos = s.pos.copy()
    pos[::4] += s.box * np.array([1, -1, 2])      # unwrapped coordinates
    o1, i1 = oracle.neighbors(pos, s.box, rcut, method="cell")
    o2, i2 = oracle.neighbors(pos, s.box, rcut, method="brute")
    assert np.array_equal(o1, o2) and np.array_equal(i1, i2)
    rows = brute.neighbors(pos, s.box, rcut)
    for i in range(s.n):
        assert np.array_equal(i1[o1[i]:o1[i + 1]], rows[i])


def test_neighbor_count_matches_lattice_shells():
    # perfect diamond: shells at a*sqrt(3)/4 (4), a/sqrt(2) (12); 4.0 A holds both
    s = W.diamond(3, 3, 3)
    off, idx = oracle.neighbors(s.pos, s.box, 4.0)
    assert np.all(np.diff(off) == 16)
    off, idx = oracle.neighbors(s.pos, s.box, 3.0)
    assert np.all(np.diff(off) == 4)


def test_counts():
    s = W.diamond(2, 2, 2, jitter=0.05, seed=3)
    off, idx = oracle.neighbors(s.pos, s.box, 4.0)
    S, P, T = oracle.counts(s.pos, s.types, s.box, W.si_table(), off, idx)
    assert S == len(idx) and P == 4 * s.n and T == 12 * s.n


def test_partial_range_sums_to_whole():
    s = jittered_cell(80)
    table = stress_table(1)
    off, idx = oracle.neighbors(s.pos, s.box, 4.0)
    E, F, Wv = oracle.compute(s.pos, s.types, s.box, table, off, idx)
    E1, F1, W1 = oracle.compute(s.pos, s.types, s.box, table, off, idx, 0, 23)
    E2, F2, W2 = oracle.compute(s.pos, s.types, s.box, table, off, idx, 23, s.n, threads=4)
    assert E1 + E2 == pytest.approx(E, rel=1e-13)
    assert np.abs(F1 + F2 - F).max() < 1e-11


def _trimer_energy_mp(pos, p):
    """Energy of a three-atom cluster from Eq. 1-3 with the literal switching
    function 1/2 - 1/2 sin(pi/2 (r - R)/D), in 50-digit arithmetic (mpmath),
    where its cancellation near R + D costs nothing."""
    import mpmath as mp
    R, D = mp.mpf(p["R"]), mp.mpf(p["D"])

    def fc(r):
        if r < R - D:
            return mp.mpf(1)
        if r < R + D:
            return mp.mpf("0.5") - mp.mpf("0.5") * mp.sin(mp.pi / 2 * (r - R) / D)
        return mp.mpf(0)

    def g(c):
        c2, d2 = mp.mpf(p["c"]) ** 2, mp.mpf(p["d"]) ** 2
        return mp.mpf(p["gamma"]) * (1 + c2 / d2 - c2 / (d2 + (mp.mpf(p["h"]) - c) ** 2))

    def dist(a, b):
        return mp.sqrt(sum((pos[b][x] - pos[a][x]) ** 2 for x in range(3)))

    E = mp.mpf(0)
    for i in range(3):
        for j in range(3):
            if j == i:
                continue
            rij = dist(i, j)
            zeta = mp.mpf(0)
            for k in range(3):
                if k in (i, j):
                    continue
                rik = dist(i, k)
                cos_t = sum((pos[j][x] - pos[i][x]) * (pos[k][x] - pos[i][x]) for x in range(3)) / (rij * rik)
                zeta += fc(rik) * g(cos_t)
            b = (1 + (mp.mpf(p["beta"]) * zeta) ** mp.mpf(p["eta"])) ** (-1 / (2 * mp.mpf(p["eta"])))
            fr = mp.mpf(p["A"]) * mp.exp(-mp.mpf(p["lambda1"]) * rij)
            fa = -mp.mpf(p["B"]) * mp.exp(-mp.mpf(p["lambda2"]) * rij)
            E += fc(rij) * (fr + b * fa) / 2
    return E


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8, 1e-10])
def test_third_atom_near_cutoff_against_50_digits(eps):
    """A bond at 2.35 A with a third atom eps inside R + D: f_C(r_ik) ~ eps^2
    is tiny, but dV/dzeta ~ zeta^(eta - 1) keeps the third atom's force
    finite (~ eps^(2 eta - 1)).  The oracle's forces must match the
    derivative of the 50-digit energy to 1e-10 of the largest force, which
    the literal 1/2 - 1/2 sin form misses by orders of magnitude below
    eps ~ 1e-7 A (cancellation).  (The third atom's force is not checked
    relative to itself: the FP64 rounding of r_ik alone moves it by
    ~0.6 * 3e-16 / eps relative.)"""
    import mpmath as mp
    mp.mp.dps = 50
    p = dict(W.SI)
    cut = p["R"] + p["D"]
    pos = [[0.0, 0.0, 0.0], [2.35, 0.0, 0.0], [0.3, cut - eps, 0.0]]
    # place k exactly: r_ik = cut - eps in FP64 (the oracle sees FP64 positions)
    y = math.sqrt((cut - eps) ** 2 - 0.09)
    pos[2][1] = y
    s = W.System(np.array(pos) + 10.0, np.zeros(3, np.int32), np.array([30.0, 30.0, 30.0]))
    off, idx = oracle.neighbors(s.pos, s.box, cut + 1.0)
    E, F, _ = oracle.compute(s.pos, s.types, s.box, W.si_table(), off, idx)
    mpos = [[mp.mpf(v) for v in row] for row in s.pos]
    Fref = np.zeros((3, 3))
    for a in range(3):
        for x in range(3):
            def e_of(t, a=a, x=x):
                q = [row[:] for row in mpos]
                q[a][x] = t
                return _trimer_energy_mp(q, p)
            Fref[a, x] = -float(mp.diff(e_of, mpos[a][x]))
    Eref = float(_trimer_energy_mp(mpos, p))
    assert abs(E - Eref) < 1e-12 * abs(Eref)
    fmax = np.abs(Fref).max()
    assert np.abs(F - Fref).max() < 1e-10 * fmax
    assert np.linalg.norm(Fref[2]) > 1e-5 * fmax   # the term really is there
