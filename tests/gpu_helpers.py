"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare with the stated error metrics.

Tolerances:
  forces: RMS relative error over all 3N components, <= 1e-11 (FP64 path),
          <= 1e-5 (mixed and single paths);
  energy: |E - E_ref| / N <= 1e-12 eV (FP64), <= 1e-6 eV (mixed), <= 5e-6 eV
          (single);
  virial: max_ab |W_ab - W_ref,ab| <= max(rel * max_ab |W_ref,ab|, abs * N) with
          rel = the force tolerance (the virial is a sum of the same force
          terms times FP64 relative vectors, so it carries their relative
          error) and abs = the energy tolerance (floor for a near-zero virial).
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


def virial_tol(Vo, n, precision):
    t = TOL[precision]
    return max(t["force"] * float(np.abs(Vo).max()), t["energy"] * n)


def assert_parity(E, F, V, Eo, Fo, Vo, n, precision, label=""):
    ferr, eerr, verr = errors(E, F, V, Eo, Fo, Vo, n)
    tol = TOL[precision]
    vtol = virial_tol(Vo, n, precision)
    say(f"[parity] {label} {precision}: force_rms_rel={ferr:.3e} energy/atom={eerr:.3e} "
        f"virial_abs={verr:.3e} (tol {vtol:.2e})")
    assert ferr <= tol["force"], f"force RMS rel {ferr:.3e} > {tol['force']}"
    assert eerr <= tol["energy"], f"energy/atom {eerr:.3e} > {tol['energy']}"
    assert verr <= vtol, f"virial error {verr:.3e} > {vtol:.3e}"
