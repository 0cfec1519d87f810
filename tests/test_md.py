"""GPU tests of the molecular-dynamics driver (velocity Verlet around the
evaluation): a few steps equal a host velocity-Verlet integration with the
oracle's forces, and a longer run conserves energy while rebuilding its list."""
import numpy as np
import pytest

from paper_1710_00882_amd import workloads as W

from gpu_helpers import oracle_eval, say

pytestmark = pytest.mark.gpu

CONV = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 / 1e14   # A/ps^2 per eV/(A amu)
MASS_SI = 28.0855


def _velocities(n, temperature, seed):
    g = W.rng(seed)
    kB = 8.617333262e-5
    v = g.normal(0.0, np.sqrt(kB * temperature * CONV / MASS_SI), size=(n, 3))
    return v - v.mean(axis=0)


def _ordered(s, order):
    """The system in lattice order, or with its atoms in a random order (the
    library then renumbers them in cell order at every build)."""
    if order == "lattice":
        return s
    p = np.random.default_rng(13).permutation(s.n)
    return W.System(s.pos[p].copy(), s.types[p].copy(), s.box.copy())


@pytest.mark.parametrize("order", ["lattice", "random"])
def test_steps_match_host_verlet_with_oracle_forces(order):
    import torch
    from paper_1710_00882_amd import Tersoff
    table = W.si_table()
    s = _ordered(W.si_512(), order)
    v0 = _velocities(s.n, 800.0, 7)
    dt, nsteps = 0.001, 4
    m = Tersoff(table)
    pos = torch.tensor(s.pos, device="cuda")
    vel = torch.tensor(v0, device="cuda")
    types = torch.tensor(s.types, device="cuda")
    res = m.md_run(pos, vel, types, s.box, [MASS_SI], dt, nsteps, "fp64", skin=W.SKIN)
    # host reference
    x, v = s.pos.copy(), v0.copy()
    sys_ = W.System(pos=x, types=s.types, box=s.box)
    _, F, _, _, _ = oracle_eval(sys_, table)
    for _ in range(nsteps):
        v += 0.5 * dt * CONV * F / MASS_SI
        x += dt * v
        sys_ = W.System(pos=x, types=s.types, box=s.box)
        E, F, _, _, _ = oracle_eval(sys_, table)
        v += 0.5 * dt * CONV * F / MASS_SI
    dx = np.abs(pos.cpu().numpy() - x).max()
    dv = np.abs(vel.cpu().numpy() - v).max()
    say(f"[md] {order}, {nsteps} steps: max|dx|={dx:.2e} A max|dv|={dv:.2e} A/ps dE={abs(res['epot'] - E):.2e} eV")
    assert dx < 1e-10 and dv < 1e-7
    assert abs(res["epot"] - E) / s.n < 1e-11
    ek = 0.5 * MASS_SI * (v ** 2).sum() / CONV
    assert abs(res["ekin"] - ek) / s.n < 1e-11


@pytest.mark.parametrize("order", ["lattice", "random"])
@pytest.mark.parametrize("precision,tol", [("fp64", 2e-4), ("mixed", 2e-4)])
def test_energy_conservation_with_rebuilds(precision, tol, order):
    import torch
    from paper_1710_00882_amd import Tersoff
    s = _ordered(W.si_512(), order)
    m = Tersoff(W.si_table())
    pos = torch.tensor(s.pos, device="cuda")
    vel = torch.tensor(_velocities(s.n, 1200.0, 11), device="cuda")
    types = torch.tensor(s.types, device="cuda")
    r0 = m.md_run(pos, vel, types, s.box, [MASS_SI], 0.0005, 0, precision, skin=0.3)
    e0 = r0["epot"] + r0["ekin"]
    r1 = m.md_run(pos, vel, types, s.box, [MASS_SI], 0.0005, 600, precision, skin=0.3)
    e1 = r1["epot"] + r1["ekin"]
    say(f"[md] {precision} {order}: E0={e0 / s.n:.6f} E1={e1 / s.n:.6f} eV/atom, T={r1['temperature']:.0f} K, "
        f"builds={r1['builds']}")
    assert r1["builds"] > 1
    assert abs(e1 - e0) / s.n < tol
