#!/usr/bin/env python
"""Tersoff E+F throughput on one MI355X; prints ONE JSON line.

A step is one evaluation of the whole path on the 2,048,000-atom silicon
workload (diamond Si 80x80x40 cells, N(0, 0.1 A) jitter, +-2% strain): the
positions of step k are those of step k-1 perturbed by N(0, 0.01 A); every
5th step rebuilds the neighbour list on the GPU (cell list, skin 1 A) before
the energy/force/virial kernel.  All position sets are resident in HBM before
the timed region starts.  The headline is the mixed-precision path; the
all-FP64 path is timed the same way and reported beside it.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Tersoff E+F atoms/s mixed vs FP64 @32k–2M Si (VALU roofline %); serve p50/p99"
UNIT = "atoms*evals/s"
REBUILD_EVERY = 5

# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
# Unpacked FP32 and FP64 issue at the same rate; packed FP32 (2x) is not used
# by this build.
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12      # 78.64
PEAK_FP32_PACKED_TFLOPS = 157.3

# Algorithmic flops of one evaluation, counted on the restructured
# Algorithm 1 (zeta and its gradients computed once): add/sub/mul/compare/
# rint = 1, fma = 2, sqrt/reciprocal/exp/log/log1p = 1 each.
FLOPS_PER_ENTRY = 21      # minimum-image displacement, r^2, skin test
FLOPS_PER_PAIR = 61       # r, u, f_R, f_A, b_ij (log form), energy, pair force, virial, dV/dzeta
FLOPS_PER_TRIPLET = 100   # cos, g, g', zeta term, both gradients, dV/dzeta * gradients, virial


def algorithmic_flops(S: int, P: int, T: int) -> float:
    return float(FLOPS_PER_ENTRY * S + FLOPS_PER_PAIR * P + FLOPS_PER_TRIPLET * T)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_positions(system, nsets, sigma=0.01, seed=1234):
    from paper_1710_00882_amd import workloads as W
    g = W.rng(seed)
    out = [system.pos]
    for _ in range(nsets - 1):
        out.append(W.perturb(out[-1], sigma, g))
    return out


def timed_run(model, pos_dev, types_dev, box, precision, nsteps, forces, out):
    import torch
    model.profile(True)
    model.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsteps):
        if k % REBUILD_EVERY == 0:
            model.build_neighbors(pos_dev[k], types_dev, box)
        model.compute(pos_dev[k], precision, forces=forces, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = model.profile_read()
    model.profile(False)
    model.check()
    return t1 - t0, prof


def measure_workload(system, table, steps, warmup, precisions, batch_atoms=None):
    import torch
    from paper_1710_00882_amd import Tersoff
    nsets = warmup + steps
    host_sets = make_positions(system, nsets)
    pos_dev = [torch.tensor(p, dtype=torch.float64, device="cuda") for p in host_sets]
    types_dev = torch.tensor(system.types, dtype=torch.int32, device="cuda")
    model = Tersoff(table)
    if batch_atoms:
        model.build_neighbors(pos_dev[0], types_dev, system.box)
        model.set_batch_atoms(batch_atoms)
    forces = torch.empty_like(pos_dev[0])
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    res = {}
    for prec in precisions:
        # warmup on the first `warmup` sets, then time on the rest
        for k in range(warmup):
            if k % REBUILD_EVERY == 0:
                model.build_neighbors(pos_dev[k], types_dev, system.box)
            model.compute(pos_dev[k], prec, forces=forces, out=out)
        torch.cuda.synchronize()
        dt, prof = timed_run(model, pos_dev[warmup:], types_dev, system.box, prec, steps, forces, out)
        S, P, T = model.counts()
        kernel_s = prof["kernel_ms"] / 1e3 / max(prof["kernels"], 1)
        flops = algorithmic_flops(S, P, T)
        res[prec] = dict(
            seconds=dt, value=system.n * steps / dt, ms_per_step=1e3 * dt / steps,
            kernel_ms=1e3 * kernel_s, build_ms=prof["build_ms"] / max(prof["builds"], 1),
            builds=prof["builds"], gather_ms=prof["gather_ms"] / max(prof["gathers"], 1),
            kernel_atoms_per_s=system.n / kernel_s, counts=dict(S=S, P=P, T=T),
            alg_flops_per_launch=flops, alg_tflops=flops / kernel_s / 1e12,
            energy_per_atom=float(out[0].item()) / system.n)
        log(f"[bench] {prec}: {res[prec]['value']:.4g} atoms*evals/s, {res[prec]['ms_per_step']:.3f} ms/step, "
            f"kernel {res[prec]['kernel_ms']:.3f} ms, gather {res[prec]['gather_ms']:.3f} ms, "
            f"build {res[prec]['build_ms']:.3f} ms, "
            f"{res[prec]['alg_tflops']:.2f} TFLOP/s alg")
    del pos_dev
    model.close()
    return res


def cpu_baseline(system, table, target_s=12.0):
    """The FP64 oracle on the host cores: full neighbour list, then the
    compute over a leading sample of centre atoms sized to ~target_s."""
    import oracle
    from paper_1710_00882_amd import workloads as W
    threads = min(os.cpu_count() or 1, 16)
    cut = W.table_cutoff(table) + W.SKIN
    t0 = time.perf_counter()
    off, idx = oracle.neighbors(system.pos, system.box, cut)
    t_nb = time.perf_counter() - t0
    m0 = min(system.n, 20000)
    t0 = time.perf_counter()
    oracle.compute(system.pos, system.types, system.box, table, off, idx, 0, m0, threads=threads)
    t_cal = time.perf_counter() - t0
    m = int(min(system.n, max(m0, m0 * target_s / max(t_cal, 1e-6))))
    t0 = time.perf_counter()
    oracle.compute(system.pos, system.types, system.box, table, off, idx, 0, m, threads=threads)
    t_c = time.perf_counter() - t0
    per_eval = t_c * system.n / m + t_nb / REBUILD_EVERY
    return dict(value=system.n / per_eval, unit=UNIT, cores=threads, kind="oracle",
                sample=(f"FP64 oracle, {threads} threads: compute over centre atoms [0, {m}) of the "
                        f"{system.n}-atom workload took {t_c:.2f} s, scaled to all atoms; plus the "
                        f"single-thread cell-list build ({t_nb:.2f} s) amortised over "
                        f"{REBUILD_EVERY} evaluations"))


def copy_probe(mib=256, reps=3):
    """A plain elementwise copy of known size: its FETCH_SIZE / WRITE_SIZE
    readings calibrate the HBM traffic counters."""
    import torch
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    log(f"[copy-probe] {reps} x elementwise copy of {mib} MiB read + {mib} MiB written")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-32k", action="store_true")
    ap.add_argument("--batch-atoms", type=int, default=0)
    ap.add_argument("--precision", choices=("both", "mixed", "fp64"), default="both",
                    help="profiling runs may time one precision only (no JSON line then)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 256 MiB device copy kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU runs are not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_00882_amd import workloads as W

    log("[bench] generating 2,048,000-atom Si workload")
    big = W.si_2m()
    table = W.si_table()
    if args.precision != "both":
        measure_workload(big, table, args.steps, args.warmup, (args.precision,), args.batch_atoms)
        return
    res = measure_workload(big, table, args.steps, args.warmup, ("mixed", "fp64"), args.batch_atoms)
    mixed, fp64 = res["mixed"], res["fp64"]

    extra_32k = None
    if not args.no_32k:
        small = W.si_32k()
        r32 = measure_workload(small, table, max(args.steps, 10), args.warmup, ("mixed", "fp64"),
                               args.batch_atoms)
        extra_32k = {p: dict(value=r32[p]["value"], kernel_ms=r32[p]["kernel_ms"],
                             kernel_atoms_per_s=r32[p]["kernel_atoms_per_s"]) for p in r32}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(big, table)
        log(f"[bench] cpu baseline {cpu['value']:.4g} atoms*evals/s on {cpu['cores']} threads")

    achieved = mixed["alg_tflops"]
    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "si_2m: diamond Si 80x80x40 cells, 2,048,000 atoms, jitter N(0,0.1 A), "
                        "strain +-2%, N(0,0.01 A) perturbation per step, GPU neighbour rebuild "
                        "every 5th step, skin 1 A, mixed precision",
            "atoms": big.n,
            "precision": "mixed",
            "rebuild_every": REBUILD_EVERY,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_ALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU_TFLOPS,
            "traffic": None,
            "kernel": "k_tersoff<float,single-type>",
            "kernel_ms": mixed["kernel_ms"],
            "alg_flops_per_launch": mixed["alg_flops_per_launch"],
            "frac_vs_packed_fp32_peak": achieved / PEAK_FP32_PACKED_TFLOPS,
        },
        "cpu_baseline": cpu,
        "fp64": {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                 "kernel_ms": fp64["kernel_ms"], "alg_tflops": fp64["alg_tflops"]},
        "mixed_vs_fp64_speedup": mixed["value"] / fp64["value"],
        "mixed_vs_fp64_kernel_speedup": fp64["kernel_ms"] / mixed["kernel_ms"],
        "build_ms": mixed["build_ms"],
        "gather_ms": mixed["gather_ms"],
        "counts_per_atom": {k: v / big.n for k, v in mixed["counts"].items()},
        "si_32k": extra_32k,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
