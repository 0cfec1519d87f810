"""GPU parity: neighbour lists bit-exact, energy / forces / virial within the
stated tolerances of the FP64 oracle, work counts exact, error paths.

All calls go through the C ABI of libtersoff.so (ctypes binding)."""
import numpy as np
import pytest

import oracle
from paper_1710_00882_amd import workloads as W

from gpu_helpers import assert_parity, gpu_eval, oracle_eval, say, to_dev, virial_tol

pytestmark = pytest.mark.gpu


def stress_table(m=1, lam3=1.3):
    return W.table_from_species([dict(W.SI, lambda3=lam3, m=m, R=2.55, D=0.35)])


def stress_two_species(lam3=0.9):
    s0 = dict(W.SI, lambda3=lam3, R=2.55, D=0.35)
    s1 = dict(W.species_variant(s0, 0.9, 1.04), lambda3=0.5 * lam3, h=-0.3, c=8.0e4, eta=0.7)
    return W.table_from_species([s0, s1])


CASES = {
    "si512": (lambda: W.si_512(), W.si_table),
    "si_3x3x2_hot": (lambda: W.diamond(3, 3, 2, jitter=0.25, seed=5), W.si_table),
    "lam3_m1": (lambda: W.diamond(3, 2, 3, jitter=0.2, seed=6), lambda: stress_table(1)),
    "lam3_m3": (lambda: W.diamond(2, 3, 3, jitter=0.2, seed=7), lambda: stress_table(3)),
    "two_species": (lambda: W.diamond(3, 3, 3, jitter=0.2, seed=8, ntypes=2), stress_two_species),
    "two_species_si": (lambda: W.diamond(4, 3, 3, jitter=0.15, seed=9, ntypes=2), W.two_species_table),
    "disordered_small": (lambda: W.disordered(3000, seed=10), W.two_species_table),
}


@pytest.mark.parametrize("case", list(CASES))
def test_neighbors_bit_exact(case):
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    say(f"[nbr] {case} n={s.n}")
    _, _, _, m = gpu_eval(s, table, "fp64")
    off, idx = m.neighbors()
    Eo, Fo, Vo, ooff, oidx = oracle_eval(s, table)
    assert np.array_equal(off, ooff)
    assert np.array_equal(idx, oidx)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "single"])
@pytest.mark.parametrize("case", list(CASES))
def test_compute_parity(case, precision):
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    say(f"[compute] {case} n={s.n} {precision}")
    E, F, V, m = gpu_eval(s, table, precision)
    m.check()
    Eo, Fo, Vo, off, idx = oracle_eval(s, table)
    assert_parity(E, F, V, Eo, Fo, Vo, s.n, precision, case)
    # work counts are integers: exact
    assert m.counts() == oracle.counts(s.pos, s.types, s.box, table, off, idx)


def test_unwrapped_positions_and_images():
    s = W.diamond(3, 3, 3, jitter=0.15, seed=12)
    table = stress_table(1)
    pos = s.pos.copy()
    pos[::3] += s.box
    pos[1::4] -= 3 * s.box
    s2 = W.System(pos, s.types, s.box)
    E, F, V, m = gpu_eval(s2, table, "fp64")
    off, idx = m.neighbors()
    Eo, Fo, Vo, ooff, oidx = oracle_eval(s2, table)
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert_parity(E, F, V, Eo, Fo, Vo, s.n, "fp64", "unwrapped")


@pytest.mark.parametrize("cells", [(2, 2, 2), (2, 2, 3), (2, 5, 2)])
def test_small_boxes_two_cells_per_axis(cells):
    # box of 10.86 A with a 4 A list radius gives two cells on that axis
    s = W.diamond(*cells, jitter=0.1, seed=sum(cells))
    table = W.si_table()
    E, F, V, m = gpu_eval(s, table, "fp64")
    off, idx = m.neighbors()
    Eo, Fo, Vo, ooff, oidx = oracle_eval(s, table)
    assert np.array_equal(off, ooff) and np.array_equal(idx, oidx)
    assert_parity(E, F, V, Eo, Fo, Vo, s.n, "fp64", f"box{cells}")


def test_perfect_diamond_closed_form():
    s = W.diamond(4, 4, 4)
    E, F, V, _ = gpu_eval(s, W.si_table(), "fp64")
    Eo, Fo, Vo, _, _ = oracle_eval(s, W.si_table())
    # closed form of the perfect lattice: E/atom = 2 V(r_nn, 3 g(-1/3)), F = 0
    assert abs(E / s.n - (-4.629593127666797)) < 1e-11
    assert abs(E - Eo) / s.n < 1e-12
    assert np.abs(F).max() < 1e-10            # forces vanish; a relative metric is undefined
    assert np.abs(V - Vo).max() < 1e-12 * s.n


def test_isolated_atoms_and_dimers():
    # atoms with no neighbour (zeta = 0, empty rows) next to a dimer
    pos = np.array([[1.0, 1.0, 1.0], [3.35, 1.0, 1.0], [10.0, 10.0, 10.0], [15.0, 2.0, 16.0]])
    s = W.System(pos, np.zeros(4, np.int32), np.array([20.0, 20.0, 20.0]))
    Eo, Fo, Vo, _, _ = oracle_eval(s, W.si_table())
    E, F, V, m = gpu_eval(s, W.si_table(), "fp64")
    assert_parity(E, F, V, Eo, Fo, Vo, s.n, "fp64", "dimer+isolated")
    assert np.all(F[2:] == 0.0)
    # a single bond: nothing averages, and the dimer force (0.56 eV/A) is the
    # difference of two 13 eV/A terms -- the stated bounds still hold
    for prec in ("mixed", "single"):
        E, F, V, m = gpu_eval(s, W.si_table(), prec)
        assert_parity(E, F, V, Eo, Fo, Vo, s.n, prec, "dimer+isolated")
        assert np.all(F[2:] == 0.0)


def _cluster(pos):
    pos = np.asarray(pos, dtype=np.float64) + 10.0
    return W.System(pos, np.zeros(len(pos), np.int32), np.array([24.0, 24.0, 24.0]))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_dimer_sweep(precision):
    """Dimers from 2.0 A to inside the switching zone (R - D = 2.7, R + D = 3.0
    A) in 0.05 A steps, each checked against the oracle.  Where the dimer
    force nears its zero crossing (about 2.3 A, where f_R' and f_A' cancel
    exactly) its relative error is undefined; there the bound is the same
    absolute error as at |F| = 0.5 eV/A."""
    ftol = {"mixed": 1e-5, "fp64": 1e-11}[precision]
    etol = {"mixed": 1e-6, "fp64": 1e-12}[precision]
    worst = (0.0, 0.0)
    for r in np.arange(2.0, 2.951, 0.05):
        s = _cluster([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        Eo, Fo, Vo, _, _ = oracle_eval(s, W.si_table())
        E, F, V, _ = gpu_eval(s, W.si_table(), precision)
        fmag = float(np.linalg.norm(Fo, axis=1).max())
        ferr = float(np.linalg.norm(F - Fo, axis=1).max()) / max(fmag, 0.5)
        eerr = abs(E - Eo) / s.n
        worst = (max(worst[0], ferr), max(worst[1], eerr))
        assert ferr <= ftol, f"r={r:.2f}: force error {ferr:.3e} (|F| = {fmag:.3e})"
        assert eerr <= etol, f"r={r:.2f}: energy/atom error {eerr:.3e}"
        assert float(np.abs(V - Vo).max()) <= virial_tol(Vo, s.n, precision)
    say(f"[parity] dimer sweep {precision}: worst force rel {worst[0]:.3e}, energy/atom {worst[1]:.3e}")


@pytest.mark.parametrize("precision", ["mixed", "single", "fp64"])
def test_trimers(precision):
    """Equilateral (side 2.35 A) and linear (spacing 2.35 A) trimers."""
    a = 2.35
    for label, pos in (("equilateral", [[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0]]),
                       ("linear", [[0, 0, 0], [a, 0, 0], [2 * a, 0, 0]]),
                       ("scalene", [[0, 0, 0], [2.3, 0, 0], [0.4, 2.2, 0.3]])):
        s = _cluster(pos)
        Eo, Fo, Vo, _, _ = oracle_eval(s, W.si_table())
        E, F, V, _ = gpu_eval(s, W.si_table(), precision)
        assert_parity(E, F, V, Eo, Fo, Vo, s.n, precision, label)


def test_recompute_path_many_triplets():
    # dense disordered packing: batches exceed the cached-triplet capacity
    s = W.disordered(2000, density=0.09, dmin=1.7, seed=13)
    table = W.two_species_table()
    for prec in ("fp64", "mixed", "single"):
        E, F, V, m = gpu_eval(s, table, prec)
        m.check()
        Eo, Fo, Vo, off, idx = oracle_eval(s, table)
        assert_parity(E, F, V, Eo, Fo, Vo, s.n, prec, "dense")


def test_repeated_compute_moved_positions():
    import torch
    from paper_1710_00882_amd import Tersoff
    s = W.diamond(5, 5, 5, jitter=0.1, seed=14)
    table = W.si_table()
    m = Tersoff(table)
    pos, types = to_dev(s)
    m.build_neighbors(pos, types, s.box)
    g = W.rng(99)
    p = s.pos.copy()
    off, idx = oracle.neighbors(s.pos, s.box, W.table_cutoff(table) + W.SKIN)
    for it in range(3):
        p = W.perturb(p, 0.01, g)
        out, F = m.compute(torch.tensor(p, device="cuda"), "fp64")
        torch.cuda.synchronize()
        m.check()
        Eo, Fo, Vo = oracle.compute(p, s.types, s.box, table, off, idx)
        o = out.cpu().numpy()
        assert_parity(o[0], F.cpu().numpy(), o[1:], Eo, Fo, Vo, s.n, "fp64", f"step{it}")


def test_batch_size_and_determinism():
    """The force sum has no atomics and a fixed order: two calls with the same
    batch size give bit-identical energy, virial and forces.  The batch size
    (centre atoms per wavefront, 1 = one centre atom per wavefront, the
    paper's J scheme) changes only the summation order: every size stays at
    parity with the oracle, with the same work counts."""
    import torch
    from paper_1710_00882_amd import Tersoff
    s = W.disordered(3000, seed=21)
    table = W.two_species_table()
    Eo, Fo, Vo, off, idx = oracle_eval(s, table)
    counts_o = oracle.counts(s.pos, s.types, s.box, table, off, idx)
    pos, types = to_dev(s)
    m = Tersoff(table)
    try:
        m.build_neighbors(pos, types, s.box)
        for prec in ("fp64", "mixed"):
            for B in (32, 1, 7, 64, 16):
                m.set_batch_atoms(B)
                say(f"[batch] {prec} B={B}")
                runs = []
                for _ in range(2):
                    out, f = m.compute(pos, prec)
                    torch.cuda.synchronize()
                    m.check()
                    runs.append((out.cpu().numpy().copy(), f.cpu().numpy().copy()))
                (o1, f1), (o2, f2) = runs
                assert np.array_equal(o1, o2) and np.array_equal(f1, f2), f"{prec} B={B}: calls differ"
                assert_parity(float(o1[0]), f1, o1[1:], Eo, Fo, Vo, s.n, prec, f"B={B}")
                assert m.counts() == counts_o
    finally:
        m.close()


# ---------------------------------------------------------------- errors

def test_error_paths():
    import torch
    from paper_1710_00882_amd import Tersoff, TersoffError
    s = W.diamond(2, 2, 2, jitter=0.05, seed=1)
    m = Tersoff(W.si_table())
    pos, types = to_dev(s)
    # compute before build
    with pytest.raises(TersoffError) as e:
        m.compute(pos)
    assert e.value.status == -9
    # box below 2 (cutoff + skin): 10.86 < 2 (3 + 2.5)
    with pytest.raises(TersoffError) as e:
        m.build_neighbors(pos, types, s.box, skin=2.5)
    assert e.value.status == -3
    # cutoff below R + D
    with pytest.raises(TersoffError) as e:
        m.build_neighbors(pos, types, s.box, cutoff=2.9)
    assert e.value.status == -1
    # type out of range
    bad = types.clone(); bad[3] = 1
    with pytest.raises(TersoffError) as e:
        m.build_neighbors(pos, bad, s.box)
    assert e.value.status == -1
    # non-finite position
    badp = pos.clone(); badp[5, 1] = float("nan")
    with pytest.raises(TersoffError) as e:
        m.build_neighbors(badp, types, s.box)
    assert e.value.status == -1
    # stale list: one atom moved by more than skin / 2
    m.build_neighbors(pos, types, s.box)
    moved = pos.clone(); moved[7, 0] += 0.6
    m.compute(moved)
    assert m.check_status() == -5
    assert m.check_status() == 0          # flags cleared by the check
    # invalid parameter tables
    bad_tab = W.si_table().copy(); bad_tab[0, 0, 0, 12] = 0.0
    with pytest.raises(TersoffError):
        Tersoff(bad_tab)


def test_atom_count_limits():
    """n = 0 and n = 2^24 + 1 are rejected before any device access (the
    pointers are never read); n = 1 (a lone atom) gives E = 0, F = 0."""
    import ctypes
    import torch
    from paper_1710_00882_amd import Tersoff
    m = Tersoff(W.si_table())
    box = np.array([20.0, 20.0, 20.0])
    bp = box.ctypes.data_as(ctypes.c_void_p)
    pos = torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64, device="cuda")
    types = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n in (0, (1 << 24) + 1):
        st = m._lib.tersoff_build_neighbors(m._h, pos.data_ptr(), types.data_ptr(), n, bp, 3.0, 1.0, None)
        assert st == -1, (n, st)
        assert "n must be in" in m._lib.tersoff_last_error(m._h).decode()
    m.build_neighbors(pos, types, box)
    for prec in ("fp64", "mixed", "single"):
        out, f = m.compute(pos, prec)
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == 0.0) and np.all(f.cpu().numpy() == 0.0)
    assert m.counts() == (0, 0, 0)
    m.close()


def test_overflow_is_reported_not_crashing():
    import torch
    from paper_1710_00882_amd import Tersoff
    # 80 atoms inside a 2.9 A ball: every atom has 79 in-range neighbours
    g = W.rng(5)
    v = g.normal(size=(80, 3))
    pos = 20.0 + v / np.linalg.norm(v, axis=1, keepdims=True) * g.uniform(0.0, 1.45, size=(80, 1))
    s = W.System(pos, np.zeros(80, np.int32), np.array([40.0, 40.0, 40.0]))
    m = Tersoff(W.si_table())
    p, t = to_dev(s)
    m.build_neighbors(p, t, s.box)
    m.compute(p, "mixed")
    torch.cuda.synchronize()
    assert m.check_status() == -4


@pytest.mark.parametrize("precision", ["mixed", "single", "fp64"])
def test_third_atom_at_cutoff_edge(precision):
    """A bond at 2.35 A and a third atom eps inside R + D: f_C(r_ik) ~ eps^2
    is tiny, yet dV/dzeta ~ zeta^(eta - 1) keeps the third atom's force at
    percents of the bond force (0.021 eV/A at eps = 1e-4 A).  A switching
    function evaluated as 1/2 - 1/2 sin rounds f_C to 0 in FP32 there and
    loses that force; the kernels take sin^2 of the distance to the cutoff."""
    cut = W.SI["R"] + W.SI["D"]
    for eps in (1e-3, 1e-4, 1e-5, 1e-6):
        y = float(np.sqrt((cut - eps) ** 2 - 0.09))
        s = _cluster([[0.0, 0.0, 0.0], [2.35, 0.0, 0.0], [0.3, y, 0.0]])
        Eo, Fo, Vo, _, _ = oracle_eval(s, W.si_table())
        E, F, V, _ = gpu_eval(s, W.si_table(), precision)
        assert_parity(E, F, V, Eo, Fo, Vo, s.n, precision, f"edge eps={eps:g}")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("case", ["si512", "two_species", "disordered_small"])
def test_atomic_scatter_matches_oracle_and_planes(case, precision):
    """The FP64 atomic scatter of the force terms (the comparison point of the
    atomic-free force planes) meets the same tolerances, and agrees with the
    planes to within summation order."""
    import torch
    from paper_1710_00882_amd import Tersoff
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    m = Tersoff(table)
    pos, types = to_dev(s)
    m.build_neighbors(pos, types, s.box)
    out_p, F_p = m.compute(pos, precision)
    m.set_force_sum("atomic")
    out_a, F_a = m.compute(pos, precision)
    torch.cuda.synchronize()
    m.check()
    o_p, o_a = out_p.cpu().numpy(), out_a.cpu().numpy()
    F_p, F_a = F_p.cpu().numpy(), F_a.cpu().numpy()
    Eo, Fo, Vo, _, _ = oracle_eval(s, table)
    assert_parity(o_a[0], F_a, o_a[1:], Eo, Fo, Vo, s.n, precision, f"{case} atomic")
    # the energy is not part of the scatter (equal up to the rounding of
    # the kernel instance's own instruction selection)
    assert abs(o_a[0] - o_p[0]) <= 1e-13 * abs(o_p[0])
    # mixed stores each pair's force term in the planes as FP32 (one rounding,
    # 2^-24 relative, per term of up to a dozen per atom); FP64 stores it exactly
    rel = 1e-6 if precision == "mixed" else 1e-12
    assert np.abs(F_a - F_p).max() <= rel * max(np.abs(F_p).max(), 1.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES) + ["dense"])
def test_triplet_mapping_matches_oracle(case, precision):
    """A lane per triplet (the comparison mapping) meets the oracle's
    tolerances with the work counts of the default mapping, also where a
    batch holds more triplets than the lanes keep (dense), and at one and at
    64 centre atoms per batch."""
    import torch
    from paper_1710_00882_amd import Tersoff
    if case == "dense":
        s, table = W.disordered(2000, density=0.09, dmin=1.7, seed=13), W.two_species_table()
    else:
        sysf, tabf = CASES[case]
        s, table = sysf(), tabf()
    Eo, Fo, Vo, off, idx = oracle_eval(s, table)
    counts_o = oracle.counts(s.pos, s.types, s.box, table, off, idx)
    m = Tersoff(table)
    try:
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box)
        m.set_mapping("triplet")
        for B in ((32, 1, 64) if case in ("si512", "dense") else (32,)):
            m.set_batch_atoms(B)
            say(f"[triplet] {case} n={s.n} {precision} B={B}")
            out, f = m.compute(pos, precision)
            torch.cuda.synchronize()
            m.check()
            o = out.cpu().numpy()
            assert_parity(float(o[0]), f.cpu().numpy(), o[1:], Eo, Fo, Vo, s.n, precision, f"{case} triplet B={B}")
            assert m.counts() == counts_o
    finally:
        m.close()


def test_triplet_mapping_rejects_single_and_atomic():
    from paper_1710_00882_amd import Tersoff, TersoffError
    s = W.diamond(2, 2, 2, jitter=0.05, seed=1)
    m = Tersoff(W.si_table())
    try:
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box)
        m.set_mapping("triplet")
        with pytest.raises(TersoffError) as e:
            m.compute(pos, "single")
        assert e.value.status == -1
        m.set_force_sum("atomic")
        with pytest.raises(TersoffError) as e:
            m.compute(pos, "mixed")
        assert e.value.status == -1
        m.set_force_sum("planes")
        m.set_mapping("pair")
        m.compute(pos, "single")
        m.check()
    finally:
        m.close()


def _eval_packing(m, pos, precision, mode):
    import torch
    m.set_packing(mode)
    out, f = m.compute(pos, precision)
    torch.cuda.synchronize()
    m.check()
    return out.cpu().numpy().copy(), f.cpu().numpy().copy(), m.counts()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "single"])
@pytest.mark.parametrize("case", list(CASES))
def test_fused_packing_matches_separate(case, precision):
    """Packing inside the compute kernel (the default) forms the same records
    and batches as the separate packing kernel, and the force gather adds the
    same planes in the same (row) order: forces agree bit for bit, energy and
    virial up to the order of the per-workgroup sums."""
    from paper_1710_00882_amd import Tersoff
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    m = Tersoff(table)
    try:
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box)
        say(f"[packing] {case} n={s.n} {precision}")
        o_f, f_f, c_f = _eval_packing(m, pos, precision, "fused")
        o_s, f_s, c_s = _eval_packing(m, pos, precision, "separate")
        assert c_f == c_s
        assert np.array_equal(f_f, f_s)
        assert np.allclose(o_f, o_s, rtol=1e-13, atol=1e-13 * abs(o_s[0]))
    finally:
        m.close()


@pytest.mark.parametrize("skin", [3.0, 3.5])
def test_long_rows_fused_and_fallback(skin):
    """Rows of 46 entries (skin 3.0: several 64-entry chunks per centre in
    the fused packing) and of 70 (skin 3.5: beyond the fused packing's
    64-entry rows, evaluated with the separate packing kernel) at parity."""
    import torch
    from paper_1710_00882_amd import Tersoff
    s, table = W.diamond(3, 3, 3, jitter=0.1, seed=31), W.si_table()
    Eo, Fo, Vo, off, idx = oracle_eval(s, table, skin=skin)
    m = Tersoff(table)
    try:
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box, skin=skin)
        for precision in ("fp64", "mixed"):
            for mode in ("fused", "separate"):
                say(f"[long rows] skin={skin} longest row {int(np.diff(off).max())} {precision} {mode}")
                o, F, _ = _eval_packing(m, pos, precision, mode)
                assert_parity(float(o[0]), F, o[1:], Eo, Fo, Vo, s.n, precision, f"skin {skin} {mode}")
    finally:
        m.close()


def test_long_rows_in_internal_numbering():
    """Rows of about 46 entries (skin 3.0) with the atoms in a random order, so
    that the build renumbers a list whose rows exceed the 32-entry register
    sort: the list handed back is the oracle's, and both packings are at
    parity with it (box of 5 cells per axis, so that the random order is
    found incoherent)."""
    from paper_1710_00882_amd import Tersoff
    skin = 3.0
    s0, table = W.diamond(6, 6, 6, jitter=0.1, seed=33), W.si_table()
    p = np.random.default_rng(9).permutation(s0.n)
    s = W.System(s0.pos[p].copy(), s0.types[p].copy(), s0.box.copy())
    Eo, Fo, Vo, off, idx = oracle_eval(s, table, skin=skin)
    assert int(np.diff(off).max()) > 32
    m = Tersoff(table)
    try:
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box, skin=skin)
        goff, gidx = m.neighbors()
        assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
        for precision in ("fp64", "mixed"):
            for mode in ("fused", "separate"):
                say(f"[long rows, random order] longest row {int(np.diff(off).max())} {precision} {mode}")
                o, F, _ = _eval_packing(m, pos, precision, mode)
                assert_parity(float(o[0]), F, o[1:], Eo, Fo, Vo, s.n, precision, f"random order {mode}")
    finally:
        m.close()


@pytest.mark.parametrize("natoms", [40, 80])
def test_overflow_reported_both_packings(natoms):
    """Atoms with more kept neighbours than a batch slot range holds are
    reported (E_OVERFLOW) without a fault: 40 atoms in a 2.9 A ball (rows of
    39: the fused packing drops the excess entries) and 80 (rows of 79: the
    separate packing kernel)."""
    import torch
    from paper_1710_00882_amd import Tersoff
    g = W.rng(7)
    v = g.normal(size=(natoms, 3))
    pos = 20.0 + v / np.linalg.norm(v, axis=1, keepdims=True) * g.uniform(0.0, 1.45, size=(natoms, 1))
    s = W.System(pos, np.zeros(natoms, np.int32), np.array([40.0, 40.0, 40.0]))
    m = Tersoff(W.si_table())
    try:
        p, t = to_dev(s)
        m.build_neighbors(p, t, s.box)
        for mode in ("fused", "separate"):
            m.set_packing(mode)
            m.compute(p, "mixed")
            torch.cuda.synchronize()
            assert m.check_status() == -4
    finally:
        m.close()


def test_stale_list_detected_in_internal_numbering():
    """With the atoms in a random order (evaluated in the library's cell-order
    numbering), moving one atom by more than skin / 2 since the build is
    reported as E_STALE, and a move below it is not."""
    import torch
    from paper_1710_00882_amd import Tersoff
    s = W.diamond(4, 4, 4, jitter=0.05, seed=21)
    p = np.random.default_rng(3).permutation(s.n)
    sp = W.System(s.pos[p].copy(), s.types[p].copy(), s.box.copy())
    m = Tersoff(W.si_table())
    try:
        pos, types = to_dev(sp)
        m.build_neighbors(pos, types, sp.box)   # skin 1.0: stale beyond 0.5
        for atom, dx, status in ((17, 0.45, 0), (17, 0.55, -5), (sp.n - 1, -0.6, -5)):
            moved = pos.clone()
            moved[atom, 1] += dx
            m.compute(moved)
            torch.cuda.synchronize()
            assert m.check_status() == status, (atom, dx)
    finally:
        m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["si512", "two_species", "disordered_small"])
def test_rebuild_is_bit_identical(case, precision):
    """Two builds from the same positions give the same energy, virial and
    forces bit for bit, also for an atom order the library renumbers (the
    within-cell order of the binning comes from atomics; the internal
    numbering sorts each cell's atoms by index)."""
    import torch
    from paper_1710_00882_amd import Tersoff
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    perm = np.random.default_rng(5).permutation(s.n)
    sp = W.System(s.pos[perm].copy(), s.types[perm].copy(), s.box.copy())
    m = Tersoff(table)
    try:
        pos, types = to_dev(sp)
        res = []
        for _ in range(2):
            m.build_neighbors(pos, types, sp.box)
            out, f = m.compute(pos, precision)
            torch.cuda.synchronize()
            m.check()
            res.append((out.cpu().numpy().copy(), f.cpu().numpy().copy()))
        assert np.array_equal(res[0][0], res[1][0])
        assert np.array_equal(res[0][1], res[1][1])
    finally:
        m.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["si512", "two_species"])
def test_atom_order_does_not_matter(case, precision):
    """The same configuration with its atoms in a random order (the library
    then renumbers the atoms in the build's cell order and writes the forces
    back at the caller's indices): the same energy and virial, and the
    permuted forces, to the stated tolerances; both orders at parity with the
    oracle."""
    from paper_1710_00882_amd import workloads as Wl
    sysf, tabf = CASES[case]
    s, table = sysf(), tabf()
    perm = np.random.default_rng(77).permutation(s.n)
    sp = Wl.System(s.pos[perm].copy(), s.types[perm].copy(), s.box.copy())
    Eo, Fo, Vo, _, _ = oracle_eval(s, table)
    E, F, V, m = gpu_eval(s, table, precision)
    m.close()
    Ep, Fp, Vp, mp = gpu_eval(sp, table, precision)
    mp.close()
    assert_parity(E, F, V, Eo, Fo, Vo, s.n, precision, f"{case} given order")
    assert_parity(Ep, Fp, Vp, Eo, Fo[perm], Vo, s.n, precision, f"{case} permuted")
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert abs(Ep - E) <= tol * abs(E)
    assert np.abs(Fp - F[perm]).max() <= tol * max(np.abs(F).max(), 1.0) * (1 if precision == "fp64" else 10)
