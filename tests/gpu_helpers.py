"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare with the stated error metrics.

Tolerances:
  forces: RMS relative error over all 3N components, <= 1e-11 (FP64 path),
          <= 1e-5 (mixed and single paths); and, so that one atom's error
          cannot hide in the average, the largest per-atom error relative to
          the largest force, max_i |F_i - F_ref,i| / max_i |F_ref,i|, within
          the same bound;
  energy: |E - E_ref| / N <= 1e-12 eV (FP64), <= 1e-6 eV (mixed), <= 5e-6 eV
          (single);
  virial: max_ab |W_ab - W_ref,ab| <= tol_E * max(N, max_ab |W_ref,ab| / 1 eV),
          tol_E the energy bound per atom (1e-12 eV FP64, 1e-6 eV mixed,
          5e-6 eV single): the energy bound per atom wherever |W| / N stays
          below 1 eV (every bulk workload), and the same number as a relative
          bound for small, strongly strained clusters, where one FP32-rounded
          term of |W| / N ~ 10 eV already carries ~1e-6 eV.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_1710_00882_amd import workloads as W

TOL = {
    "fp64": dict(force=1e-11, energy=1e-12),
    "mixed": dict(force=1e-5, energy=1e-6),
    # all-FP32 variant: each pair energy f_C (f_R + b f_A) / 2 is formed in
    # FP32, where f_R and f_A (~15 eV each at 2 A) nearly cancel, so a pair
    # carries a few 2^-24 * (|f_R| + |f_A|) ~ 1e-6 eV of rounding; the energy
    # bound is 5e-6 eV/atom, the force bound that of the mixed path
    "single": dict(force=1e-5, energy=5e-6),
}


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(system, device="cuda"):
    import torch
    pos = torch.tensor(system.pos, dtype=torch.float64, device=device)
    types = torch.tensor(system.types, dtype=torch.int32, device=device)
    return pos, types


def gpu_eval(system, table, precision, skin=W.SKIN, model=None):
    """(energy, forces (N,3), virial (6,), model) from the HIP path."""
    import torch
    from paper_1710_00882_amd import Tersoff
    m = model or Tersoff(table)
    pos, types = to_dev(system)
    m.build_neighbors(pos, types, system.box, skin=skin)
    out, f = m.compute(pos, precision)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return float(o[0]), f.cpu().numpy(), o[1:].copy(), m


def oracle_eval(system, table, skin=W.SKIN, threads=8):
    cut = W.table_cutoff(table)
    off, idx = oracle.neighbors(system.pos, system.box, cut + skin)
    E, F, V = oracle.compute(system.pos, system.types, system.box, table, off, idx, threads=threads)
    return E, F, V, off, idx


def errors(E, F, V, Eo, Fo, Vo, n):
    ferr = float(np.linalg.norm(F - Fo) / max(np.linalg.norm(Fo), 1e-300))
    eerr = abs(E - Eo) / n
    verr = float(np.abs(V - Vo).max())
    return ferr, eerr, verr


def max_atom_error(F, Fo):
    """max_i |F_i - F_ref,i| / max_i |F_ref,i| (0 when every force is 0)."""
    F = np.asarray(F).reshape(-1, 3)
    Fo = np.asarray(Fo).reshape(-1, 3)
    den = float(np.linalg.norm(Fo, axis=1).max()) if len(Fo) else 0.0
    num = float(np.linalg.norm(F - Fo, axis=1).max()) if len(Fo) else 0.0
    return num / den if den > 0 else num


def virial_tol(Vo, n, precision):
    return TOL[precision]["energy"] * max(n, float(np.abs(Vo).max()))


def assert_parity(E, F, V, Eo, Fo, Vo, n, precision, label=""):
    ferr, eerr, verr = errors(E, F, V, Eo, Fo, Vo, n)
    merr = max_atom_error(F, Fo)
    tol = TOL[precision]
    vtol = virial_tol(Vo, n, precision)
    say(f"[parity] {label} {precision}: force_rms_rel={ferr:.3e} max_atom_rel={merr:.3e} "
        f"energy/atom={eerr:.3e} virial/atom={verr / n:.3e} (tol {tol['energy']:.0e})")
    assert ferr <= tol["force"], f"force RMS rel {ferr:.3e} > {tol['force']}"
    assert merr <= tol["force"], f"largest per-atom force error {merr:.3e} of max|F| > {tol['force']}"
    assert eerr <= tol["energy"], f"energy/atom {eerr:.3e} > {tol['energy']}"
    assert verr <= vtol, f"virial error {verr:.3e} > {vtol:.3e}"
