"""CPU check of the single-precision pre-test of the GPU neighbour search
(Section 2: the full list with skin must be exact, and the search keeps it
bit-exact by deciding borderline candidates with the FP64 predicate).

The kernel rejects a candidate when its FP32 distance, computed from
coordinates wrapped into the box and rounded to float, is at least
rc + delta, delta = 4e-7 (Lx + Ly + Lz) + 1e-5, and (on grids with at least
three cells per axis) accepts it without the FP64 test when that distance is
below rc - delta.  Its comment argues delta from rounding bounds; here the
same float32 operations are replayed with numpy (fma as an exact float64
product plus one rounding) on millions of pairs built to sit where the bound
is tight: at rc +- a few FP64 ulps, at the sure-accept and rejection radii
+- a few float ulps, at coordinates 0 and L - ulp, unwrapped by +-L and +-2L,
with a displacement component within ulps of L/2 in a box of exactly twice
the list radius, on large boxes (where the wrapped coordinates carry the
largest rounding) and on boxes of one, two and three cells per axis.  Every
pair the exact predicate accepts must pass the pre-test, and every pair the
pre-test accepts outright must pass the exact predicate."""
import numpy as np

f32 = np.float32


def fmaf(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def exact_in(xi, xj, L, rc):
    """The FP64 predicate of the oracle and of the search's second phase, up
    to the last rounding of r^2 (both bounds checked here leave a margin of
    thousands of FP64 ulps, so that rounding cannot decide an outcome)."""
    d = xj - xi
    s = np.rint(d / L)
    d = d - s * L                       # s L is exact for the small integers s
    r2 = d[:, 2] * d[:, 2] + (d[:, 1] * d[:, 1] + d[:, 0] * d[:, 0])
    return r2 < rc * rc


def pretest(xi, xj, L, rc):
    """(keep, sure, shifted) of the search's phase 1 for each pair."""
    nc = np.maximum(1, np.floor(L / (rc * (1.0 + 1e-10)))).astype(int)
    shifted = bool(np.all(nc >= 3))
    Lf = L.astype(f32)
    invLf = (1.0 / L).astype(f32)
    rcs = f32(rc)
    delta = f32(4e-7) * ((Lf[0] + Lf[1]) + Lf[2]) + f32(1e-5)
    lim = rcs + delta
    lim2 = lim * lim
    sure = max(rcs - delta, f32(0))
    sure2 = sure * sure
    fi = (xi - L * np.floor(xi / L)).astype(f32)
    fj = (xj - L * np.floor(xj / L)).astype(f32)
    if shifted:
        # the stencil cell's periodic image: the shift that makes the wrapped
        # difference the minimum image (the cell of an in-range neighbour is
        # adjacent, so the walk visits it with exactly this shift)
        k = np.rint((fj.astype(np.float64) - fi.astype(np.float64)) / L)
        s = (-k * Lf.astype(np.float64)).astype(f32)
        o = (fi - s).astype(f32)
        d = (fj - o).astype(f32)
    else:
        d = (fj - fi).astype(f32)
        q = np.rint((d * invLf).astype(f32)).astype(f32)
        d = fmaf(-q, np.broadcast_to(Lf, d.shape), d)
    r2 = fmaf(d[:, 2], d[:, 2], fmaf(d[:, 1], d[:, 1], (d[:, 0] * d[:, 0]).astype(f32)))
    return r2 < lim2, (r2 < sure2) & shifted, shifted, float(sure), float(lim)


def adversarial_pairs(L, rc, sure, lim, n, rng, edge_prob=0.5):
    """Pairs whose distance sits at rc, sure and lim within a few ulps, with
    centres at random or (each coordinate with probability edge_prob) at 0 or
    at L - ulp, both atoms unwrapped by up to +-2L."""
    radii = []
    for r0, ulp in ((rc, np.spacing(rc)), (sure, np.spacing(np.float32(sure)).astype(np.float64)),
                    (lim, np.spacing(np.float32(lim)).astype(np.float64))):
        k = rng.integers(-40, 41, n)
        radii.append(r0 + k * ulp)
    r = np.concatenate(radii)
    m = len(r)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    d = u * r[:, None]
    xi = rng.uniform(0, 1, (m, 3)) * L
    edge = rng.uniform(0, 1, (m, 3))
    xi = np.where(edge < edge_prob / 2, 0.0, xi)
    xi = np.where((edge >= edge_prob / 2) & (edge < edge_prob), np.nextafter(L, 0) * np.ones_like(xi), xi)
    xj = xi + d
    xi = xi + rng.integers(-2, 3, (m, 3)) * L
    xj = xj + rng.integers(-2, 3, (m, 3)) * L
    return xi, xj


def half_box_pairs(L, rc, n, rng):
    """x component L/2 +- a few ulps (both images almost equally near), the
    other components small enough that r stays near the list radius."""
    k = rng.integers(-8, 9, n)
    dx = L[0] / 2 + k * np.spacing(L[0] / 2)
    rest = np.sqrt(np.maximum(rc * rc - dx * dx, 0.0)) * rng.uniform(0.0, 1.2, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    d = np.stack([dx, rest * np.cos(ang), rest * np.sin(ang)], axis=1)
    xi = rng.uniform(0, 1, (n, 3)) * L
    return xi, xi + d


BOXES = {
    # rc = cutoff + skin of the silicon workloads (3.0 + 1.0)
    "si_2m_strained": np.array([434.48 * 1.0173, 434.48 * 0.9841, 217.24 * 1.0119]),
    "three_cells": np.array([12.0 + 1e-6, 12.5, 13.1]),
    "two_cells": np.array([10.862, 10.862, 10.862]),
    "one_cell_exact": np.array([8.0, 8.0, 8.0]),
    "mixed_axes": np.array([8.0, 12.4, 434.0]),
}


def test_pretest_never_rejects_and_never_wrongly_accepts():
    rng = np.random.default_rng(2024)
    rc = 4.0
    borderline = 0
    for name, L in BOXES.items():
        _, _, _, sure, lim = pretest(np.zeros((1, 3)), np.zeros((1, 3)), L, rc)
        xi, xj = adversarial_pairs(L, rc, sure, lim, 60000, rng)
        if name in ("one_cell_exact", "two_cells", "mixed_axes"):
            a, b = half_box_pairs(L, rc, 60000, rng)
            xi, xj = np.concatenate([xi, a]), np.concatenate([xj, b])
        ex = exact_in(xi, xj, L, rc)
        keep, sure_ok, shifted, _, _ = pretest(xi, xj, L, rc)
        assert not np.any(ex & ~keep), f"{name}: {int(np.sum(ex & ~keep))} in-range pairs rejected by the pre-test"
        assert not np.any(sure_ok & ~ex), f"{name}: {int(np.sum(sure_ok & ~ex))} pairs accepted outside the radius"
        borderline += int(np.sum(keep & ~sure_ok))
        # the cases really are borderline: both outcomes occur
        assert ex.any() and (~ex).any()
    assert borderline > 100000


def test_pretest_random_pairs_large_box():
    """Uniform pairs over the whole interaction shell of a large box."""
    rng = np.random.default_rng(7)
    rc = 4.0
    L = BOXES["si_2m_strained"]
    n = 400000
    r = rng.uniform(0.5, 4.5, n)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    xi = rng.uniform(0, 1, (n, 3)) * L
    xj = xi + u * r[:, None]
    ex = exact_in(xi, xj, L, rc)
    keep, sure_ok, shifted, sure, lim = pretest(xi, xj, L, rc)
    assert shifted
    assert np.all(keep[ex]) and not np.any(sure_ok & ~ex)
    # nearly every in-range pair is decided without the FP64 test
    assert np.mean(sure_ok[ex]) > 0.99
