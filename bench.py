#!/usr/bin/env python
"""Tersoff E+F throughput on one MI355X; prints ONE JSON line.

A step is one evaluation of the whole path (packing, energy / force / virial
kernel, force gather; plus the GPU neighbour rebuild on every 5th step) on
the 2,048,000-atom silicon workload (diamond Si 80x80x40 cells, N(0, 0.1 A)
jitter, +-2% strain): the positions of step k are those of step k-1 perturbed
by N(0, 0.01 A).  All position sets are resident in HBM before the timed
region starts.  The headline is the mixed-precision path; the all-FP64 path
is timed the same way and reported beside it, with the 32,000-atom Si and
256,000-atom two-species disordered workloads, the batched serving loop over
4,096 small configurations, and the FP64 oracle on the host cores.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
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

# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
# = 78.64 TFLOP/s for unpacked FP32 and FP64 instructions; packed FP32 issues
# two per lane, the published FP32 vector peak of 157.3 TFLOP/s.  The roofline
# fraction is reported against that FP32 vector peak (the figure the target
# is stated against); the HIP sources are compiled without packed FP32, so
# the unpacked issue rate, half of it, is the ceiling this code can reach and
# is reported beside it.
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12      # 78.64
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic flops, counted on the restructured Algorithm 1 (zeta and its
# gradients formed once per triplet): add/sub/mul/compare/rint = 1, fma = 2,
# sqrt/reciprocal/exp/log/log1p/sin/cos = 1 each.
FLOPS_PER_ENTRY = 21      # packing: minimum-image displacement, r^2, radius test
FLOPS_PER_PAIR = 61       # r, u, f_C, f_R, f_A, b_ij (log form), energy, pair force, virial, dV/dzeta
FLOPS_PER_TRIPLET = 100   # cos, g, g', zeta term, both gradients, dV/dzeta * gradients

# Algorithmic (compulsory) HBM bytes of the packing kernel: per list entry
# the neighbour index (4); per atom its position and its position at the last
# build (24 + 24), row length and record count (4 + 4) and the first block of
# its kept-neighbour list (32), each read or written once; per kept record
# 16 B (mixed, single) or 32 B (FP64).
PACK_BYTES_PER_ENTRY = 4
PACK_BYTES_PER_ATOM = 88
RECORD_BYTES = {"mixed": 16, "single": 16, "fp64": 32}

# HBM traffic of the mixed compute kernel on the 2,048,000-atom workload from
# two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch),
# each scaled by the reading of a plain copy kernel of known size (FETCH_SIZE
# reads 0.5 of the bytes a copy moves, WRITE_SIZE 1.0).  Valid only for the
# compute source it was measured on (its SHA-256 prefix).
TRAFFIC_PROFILE = {
    "source": "f267cfdb3d72ebea",
    "fetch_kib": 140509.0, "fetch_factor": 2.0,
    "write_kib": 229662.8, "write_factor": 1.0,
    "bytes_per_launch": 140509.0 * 1024 * 2.0 + 229662.8 * 1024 * 1.0,
}
TRAFFIC_SOURCE = os.path.join(ROOT, "paper_1710_00882_amd", "csrc", "compute.hip")


def traffic_bytes():
    """The measured HBM bytes per launch of the compute kernel, or None when
    compute.hip has changed since the counters were taken."""
    if TRAFFIC_PROFILE and TRAFFIC_PROFILE["source"] == source_hash(TRAFFIC_SOURCE):
        return TRAFFIC_PROFILE["bytes_per_launch"]
    return None


def algorithmic_flops(P: int, T: int) -> float:
    return float(FLOPS_PER_PAIR * P + FLOPS_PER_TRIPLET * T)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def make_positions(system, nsets, sigma=0.01, seed=1234):
    from paper_1710_00882_amd import workloads as W
    g = W.rng(seed)
    out = [system.pos]
    for _ in range(nsets - 1):
        out.append(W.perturb(out[-1], sigma, g))
    return out


def timed_run(model, pos_dev, types_dev, box, precision, nsteps, forces, out, skin):
    import torch
    model.profile(True)
    model.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsteps):
        if k % REBUILD_EVERY == 0:
            model.build_neighbors(pos_dev[k], types_dev, box, skin=skin)
        model.compute(pos_dev[k], precision, forces=forces, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = model.profile_read()
    model.profile(False)
    model.check()
    return t1 - t0, prof


def measure_workload(system, table, steps, warmup, precisions, batch_atoms=None, sigma=0.01, force_sum="planes",
                     mapping="pair", packing="separate"):
    import torch
    from paper_1710_00882_amd import Tersoff
    from paper_1710_00882_amd import workloads as W
    nsets = warmup + steps
    host_sets = make_positions(system, nsets, sigma=sigma)
    pos_dev = [torch.tensor(p, dtype=torch.float64, device="cuda") for p in host_sets]
    types_dev = torch.tensor(system.types, dtype=torch.int32, device="cuda")
    model = Tersoff(table)
    model.set_force_sum(force_sum)
    model.set_mapping(mapping)
    model.set_packing(packing)
    if batch_atoms:
        model.build_neighbors(pos_dev[0], types_dev, system.box, skin=W.SKIN)
        model.set_batch_atoms(batch_atoms)
    forces = torch.empty_like(pos_dev[0])
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    res = {}
    for prec in precisions:
        for k in range(warmup):
            if k % REBUILD_EVERY == 0:
                model.build_neighbors(pos_dev[k], types_dev, system.box, skin=W.SKIN)
            model.compute(pos_dev[k], prec, forces=forces, out=out)
        torch.cuda.synchronize()
        dt, prof = timed_run(model, pos_dev[warmup:], types_dev, system.box, prec, steps, forces, out, W.SKIN)
        S, P, T = model.counts()
        main_s = prof["kernel_ms"] / 1e3 / max(prof["kernels"], 1)
        pack_s = prof["pack_ms"] / 1e3 / max(prof["packs"], 1)
        gather_s = prof["gather_ms"] / 1e3 / max(prof["gathers"], 1)
        # the fused packing (no packing kernel timed) counts the packing's
        # entry work in the compute kernel
        fused = prof["packs"] == 0
        flops = algorithmic_flops(P, T) + (FLOPS_PER_ENTRY * S if fused else 0)
        # kept records: the in-cutoff pairs (exact for one species; a lower
        # bound with several, whose packing radius is the largest cutoff)
        pack_bytes = PACK_BYTES_PER_ENTRY * S + PACK_BYTES_PER_ATOM * system.n + RECORD_BYTES[prec] * P
        res[prec] = dict(
            seconds=dt, value=system.n * steps / dt, ms_per_step=1e3 * dt / steps,
            main_ms=1e3 * main_s, pack_ms=1e3 * pack_s, gather_ms=1e3 * gather_s,
            build_ms=prof["build_ms"] / max(prof["builds"], 1), builds=prof["builds"],
            compute_ms=1e3 * (main_s + pack_s + gather_s),
            compute_atoms_per_s=system.n / (main_s + pack_s + gather_s),
            counts=dict(S=S, P=P, T=T), alg_flops_per_launch=flops, alg_tflops=flops / main_s / 1e12, fused=fused,
            pack_alg_bytes=pack_bytes, pack_gbs=pack_bytes / pack_s / 1e9 if pack_s > 0 else None,
            energy_per_atom=float(out[0].item()) / system.n)
        r = res[prec]
        log(f"[bench] n={system.n} {prec}: "
            f"{r['value']:.4g} atoms*evals/s, {r['ms_per_step']:.3f} ms/step | pack {r['pack_ms']:.3f} "
            f"main {r['main_ms']:.3f} gather {r['gather_ms']:.3f} build {r['build_ms']:.3f} ms | "
            f"main {r['alg_tflops']:.2f} TFLOP/s alg" + (" (packing fused)" if fused else
                                                          f", pack {r['pack_gbs']:.0f} GB/s alg"))
    del pos_dev
    model.close()
    return res


def ablate(system, table, args, default_res, sigma=0.01):
    """The three mappings of the triplet loop onto a wavefront, mixed
    precision: lane per neighbour of one centre atom (one atom per batch),
    lane per triplet, and the default lane per packed pair."""
    log(f"[bench] n={system.n}: one centre atom per wavefront (J-scheme ablation)")
    steps = max(args.steps, 10)
    r = measure_workload(system, table, steps, args.warmup, ("mixed",), batch_atoms=1, sigma=sigma)["mixed"]
    log(f"[bench] n={system.n}: a lane per triplet")
    t = measure_workload(system, table, steps, args.warmup, ("mixed",), sigma=sigma, mapping="triplet")["mixed"]
    return {"lane_per_pair_main_ms": default_res["main_ms"], "lane_per_j_main_ms": r["main_ms"],
            "lane_per_j_slowdown": r["main_ms"] / default_res["main_ms"],
            "lane_per_triplet_main_ms": t["main_ms"],
            "lane_per_triplet_slowdown": t["main_ms"] / default_res["main_ms"],
            "lane_per_pair_ms_per_step": default_res["ms_per_step"], "lane_per_j_ms_per_step": r["ms_per_step"],
            "lane_per_triplet_ms_per_step": t["ms_per_step"]}


def f1_comparison(system, table, args, default_res):
    """The atomic-free force sum (force planes + gather, the default) against
    an FP64 atomic scatter of the same force terms (Section 3's conflicting
    updates), mixed and FP64 on the 2M-atom workload: whole-step times and
    the kernels of each."""
    log(f"[bench] n={system.n}: FP64 atomic scatter of the force terms (f1 comparison)")
    r = measure_workload(system, table, args.steps, args.warmup, ("mixed", "fp64"), force_sum="atomic")
    out = {}
    for p in ("mixed", "fp64"):
        d, a = default_res[p], r[p]
        out[p] = {"planes_ms_per_step": d["ms_per_step"], "atomic_ms_per_step": a["ms_per_step"],
                  "planes_kernels_ms": {"pack": d["pack_ms"], "main": d["main_ms"], "gather": d["gather_ms"]},
                  "atomic_kernels_ms": {"zero+pack": a["pack_ms"], "main": a["main_ms"], "sums": a["gather_ms"]},
                  "atomic_vs_planes_step": a["ms_per_step"] / d["ms_per_step"]}
    return out


def packing_comparison(system, table, args, default_res):
    """The separate packing kernel (the default) against packing inside the
    compute kernel, mixed and FP64 on the 2M-atom workload."""
    log(f"[bench] n={system.n}: packing inside the compute kernel (comparison)")
    r = measure_workload(system, table, args.steps, args.warmup, ("mixed", "fp64"), packing="fused")
    out = {}
    for p in ("mixed", "fp64"):
        d, a = default_res[p], r[p]
        out[p] = {"separate_ms_per_step": d["ms_per_step"], "fused_ms_per_step": a["ms_per_step"],
                  "separate_kernels_ms": {"pack": d["pack_ms"], "main": d["main_ms"], "gather": d["gather_ms"]},
                  "fused_kernels_ms": {"main": a["main_ms"], "gather": a["gather_ms"]},
                  "fused_vs_separate_step": a["ms_per_step"] / d["ms_per_step"]}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, table, runs=5, sample_s=1.0):
    """The FP64 oracle on the host cores, as it stands: the cell-list build
    (single-threaded) over the whole workload, and the compute over a leading
    sample of centre atoms sized to ~sample_s per run, on all cores (at most
    16, the host share of one GPU) and on one thread; each the median of
    `runs` runs, the build amortised over the rebuild interval.  A compute
    call has a fixed cost (its per-thread force and virial arrays cover every
    atom) and a cost per centre atom: both are measured -- the call over 64
    centre atoms, then over the sample -- and the whole workload's time is the
    fixed cost plus the per-atom cost times its atoms."""
    import oracle
    from paper_1710_00882_amd import workloads as W
    threads = min(os.cpu_count() or 1, 16)
    cut = W.table_cutoff(table) + W.SKIN
    t_nb = []
    for _ in range(runs):
        t0 = time.perf_counter()
        off, idx = oracle.neighbors(system.pos, system.box, cut)
        t_nb.append(time.perf_counter() - t0)
    nb = float(np.median(t_nb))

    def timed(th, m):
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.compute(system.pos, system.types, system.box, table, off, idx, 0, m, threads=th)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def per_eval(th):
        fixed = timed(th, 64)
        m0 = min(system.n, 4000 * th)
        t0 = time.perf_counter()
        oracle.compute(system.pos, system.types, system.box, table, off, idx, 0, m0, threads=th)
        per = max(time.perf_counter() - t0 - fixed, 1e-9) / m0
        m = int(min(system.n, max(m0, sample_s / per)))
        per = max(timed(th, m) - fixed, 1e-9) / (m - 64)
        return fixed + per * system.n, m

    c_all, m_all = per_eval(threads)
    c_one, m_one = per_eval(1)
    per_eval_all = c_all + nb / REBUILD_EVERY
    per_eval_one = c_one + nb / REBUILD_EVERY
    return dict(value=system.n / per_eval_all, unit=UNIT, cores=threads, kind="oracle",
                sample=(f"FP64 oracle on {cpu_model()}: compute over centre atoms [0, {m_all}) on {threads} "
                        f"threads and [0, {m_one}) on 1 thread, and over 64 centre atoms (the call's fixed "
                        f"cost), each the median of {runs} runs, extrapolated to the {system.n}-atom "
                        f"workload; plus the single-thread cell-list build over all atoms (median {nb:.2f} s "
                        f"of {runs}) amortised over {REBUILD_EVERY} evaluations"),
                value_1_thread=system.n / per_eval_one, cpu_model=cpu_model(), runs=runs,
                compute_s_per_eval_all_cores=c_all, compute_s_per_eval_1_thread=c_one, build_s=nb)


# ---- serving ----------------------------------------------------------------

def _serve_run(model, systems, forces, offsets_ns, precision, lead_ns=300_000_000):
    """Submit every configuration with release time t0 + offset; wait for all.
    Returns (latencies ms, span s from first release to last ready)."""
    from paper_1710_00882_amd import clock_ns
    t0 = clock_ns() + lead_ns
    tickets = []
    for s, f, off in zip(systems, forces, offsets_ns):
        tickets.append(model.submit(s.pos, s.types, s.box, precision, forces=f, release_ns=t0 + int(off)))
    lat = np.zeros(len(tickets))
    ready = np.zeros(len(tickets))
    bsz = np.zeros(len(tickets))
    for q, t in enumerate(tickets):
        r = model.wait(t, 120000.0)
        if r["status"] != 0:
            raise RuntimeError(f"serving: configuration {q} failed with status {r['status']}")
        lat[q] = r["latency_ms"]
        ready[q] = offsets_ns[q] * 1e-6 + r["latency_ms"]
        bsz[q] = r["batch_systems"]
    span_s = (ready.max() - float(np.min(offsets_ns)) * 1e-6) * 1e-3
    return lat, span_s, bsz


def serve_bench(table, count=4096, seed=0, max_batch_atoms=262144, max_batch_systems=1024,
                baseline_count=256, repeat=3):
    import torch
    from paper_1710_00882_amd import Tersoff
    from paper_1710_00882_amd import workloads as W
    systems = W.serve_stream(count=count, seed=seed)
    natoms = sum(s.n for s in systems)
    forces = [np.full(s.pos.shape, 0.0) for s in systems]      # pages touched before timing
    model = Tersoff(table)
    model.serve_start(max_batch_atoms=max_batch_atoms, max_batch_systems=max_batch_systems, skin=W.SKIN)
    out = dict(workload=(f"{count} periodic diamond-Si cells, target sizes log-uniform in [64, 4096] atoms "
                         f"({natoms} atoms in all), strain U(+-3%), jitter N(0, 0.08 A); forces returned "
                         f"to host memory; capacity and Poisson runs submit the stream {repeat} times"),
               configs=count, atoms=natoms, max_batch_atoms=max_batch_atoms,
               max_batch_systems=max_batch_systems)
    # the open-loop runs submit the stream `repeat` times (each copy with its
    # own force buffers) so that start-up and drain take a small share
    long_sys = systems * repeat
    long_forces = forces + [np.full(s.pos.shape, 0.0) for _ in range(repeat - 1) for s in systems]
    nlong = len(long_sys)
    g = np.random.default_rng(seed + 1)
    zeros = np.zeros(nlong)
    for prec in ("mixed", "fp64"):
        _serve_run(model, systems, forces, zeros[:count], prec)        # warm-up: the whole stream once
        lat, span, bsz = _serve_run(model, long_sys, long_forces, zeros, prec)
        cap = nlong / span
        entry = dict(capacity_configs_per_s=cap, capacity_atoms_per_s=repeat * natoms / span,
                     saturated_p50_ms=float(np.percentile(lat, 50)),
                     saturated_p99_ms=float(np.percentile(lat, 99)),
                     mean_batch_systems=float(bsz.mean()))
        log(f"[serve] {prec}: capacity {cap:.4g} configs/s ({repeat * natoms / span:.4g} atoms/s), "
            f"mean batch {bsz.mean():.1f} configs")
        if prec == "mixed":
            loads = []
            for frac in (0.5, 0.75, 1.0, 1.25, 1.5):
                rate = frac * cap
                offs = np.cumsum(g.exponential(1.0 / rate, size=nlong)) * 1e9
                offs -= offs[0]
                lat, span, bsz = _serve_run(model, long_sys, long_forces, offs, prec)
                loads.append(dict(load=frac, offered_configs_per_s=rate,
                                  achieved_configs_per_s=nlong / span,
                                  p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                                  mean_batch_systems=float(bsz.mean())))
                log(f"[serve] load {frac:.2f}: offered {rate:.4g}/s achieved {nlong / span:.4g}/s "
                    f"p50 {loads[-1]['p50_ms']:.3f} ms p99 {loads[-1]['p99_ms']:.3f} ms "
                    f"(mean batch {bsz.mean():.1f})")
            entry["poisson"] = loads
        out[prec] = entry
    # device-resident requests: positions, types and forces already in HBM,
    # so a batch needs no host staging and no PCIe copies
    import types as pytypes
    dsys = [pytypes.SimpleNamespace(pos=torch.from_numpy(s.pos).cuda(), types=torch.from_numpy(s.types).cuda(),
                                    box=s.box) for s in systems]
    dforces = [torch.zeros_like(d.pos) for _ in range(repeat) for d in dsys]
    torch.cuda.synchronize()
    _serve_run(model, dsys, dforces[:count], zeros[:count], "mixed")      # warm-up
    lat, span, bsz = _serve_run(model, dsys * repeat, dforces, zeros, "mixed")
    out["mixed_device_resident"] = dict(
        capacity_configs_per_s=nlong / span, capacity_atoms_per_s=repeat * natoms / span,
        saturated_p50_ms=float(np.percentile(lat, 50)), saturated_p99_ms=float(np.percentile(lat, 99)),
        mean_batch_systems=float(bsz.mean()))
    log(f"[serve] mixed, device-resident requests: capacity {nlong / span:.4g} configs/s "
        f"({repeat * natoms / span:.4g} atoms/s), mean batch {bsz.mean():.1f} configs")
    del dsys, dforces
    out["stats"] = model.serve_stats()
    model.close()

    # baseline: one configuration at a time, FP64, build + compute each
    # (host arrays in, forces back to host), no batching and no graph
    m1 = Tersoff(table)
    lat1 = []
    sub = systems[:baseline_count]
    for s in sub[:8]:
        pos = torch.from_numpy(s.pos).cuda()
        m1.build_neighbors(pos, torch.from_numpy(s.types).cuda(), s.box, skin=W.SKIN)
        m1.compute(pos, "fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sub:
        t1 = time.perf_counter()
        pos = torch.from_numpy(s.pos).cuda()
        m1.build_neighbors(pos, torch.from_numpy(s.types).cuda(), s.box, skin=W.SKIN)
        o, f = m1.compute(pos, "fp64")
        f.cpu()
        o.cpu()
        lat1.append(time.perf_counter() - t1)
    dt = time.perf_counter() - t0
    m1.close()
    lat1 = np.array(lat1) * 1e3
    out["baseline_one_at_a_time_fp64"] = dict(
        configs=len(sub), configs_per_s=len(sub) / dt, p50_ms=float(np.percentile(lat1, 50)),
        p99_ms=float(np.percentile(lat1, 99)))
    out["capacity_vs_baseline_fp64"] = out["fp64"]["capacity_configs_per_s"] / (len(sub) / dt)
    out["capacity_vs_baseline_mixed"] = out["mixed"]["capacity_configs_per_s"] / (len(sub) / dt)
    log(f"[serve] baseline one-at-a-time FP64: {len(sub) / dt:.4g} configs/s, p50 "
        f"{out['baseline_one_at_a_time_fp64']['p50_ms']:.3f} ms")
    return out


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
    ap.add_argument("--no-256k", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the lane-per-j vs lane-per-pair comparison on the 32k and 256k workloads")
    ap.add_argument("--batch-atoms", type=int, default=0)
    ap.add_argument("--precision", choices=("both", "mixed", "fp64", "single"), default="both",
                    help="profiling runs may time one precision of one workload only (no JSON line)")
    ap.add_argument("--workload", choices=("si_2m", "disordered_256k"), default="si_2m",
                    help="with --precision: the workload of the profiling run")
    ap.add_argument("--serve-only", action="store_true", help="profiling: the serving benchmark only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 256 MiB device copy kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this benchmark runs on a single GPU)", file=sys.stderr)
        sys.exit(2)

    from paper_1710_00882_amd import workloads as W

    table = W.si_table()
    if args.serve_only:
        serve_bench(table)
        return
    if args.precision != "both" and args.workload == "disordered_256k":
        log("[bench] generating the 256,000-atom two-species disordered workload")
        measure_workload(W.disordered_256k(), W.two_species_table(), args.steps, args.warmup, (args.precision,),
                         args.batch_atoms, sigma=0.005)
        return
    log("[bench] generating the 2,048,000-atom Si workload")
    big = W.si_2m()
    if args.precision != "both":
        measure_workload(big, table, args.steps, args.warmup, (args.precision,), args.batch_atoms)
        return
    res = measure_workload(big, table, args.steps, args.warmup, ("mixed", "fp64", "single"), args.batch_atoms)
    mixed, fp64, single = res["mixed"], res["fp64"], res["single"]

    ablation = {}
    f1 = None if args.no_ablation else f1_comparison(big, table, args, res)
    packing = None if args.no_ablation else packing_comparison(big, table, args, res)
    extra_32k = None
    if not args.no_32k:
        small = W.si_32k()
        r32 = measure_workload(small, table, max(args.steps, 10), args.warmup, ("mixed", "fp64"),
                               args.batch_atoms)
        extra_32k = {p: dict(value=r32[p]["value"], ms_per_step=r32[p]["ms_per_step"],
                             compute_ms=r32[p]["compute_ms"], main_ms=r32[p]["main_ms"],
                             build_ms=r32[p]["build_ms"]) for p in r32}
        extra_32k["mixed_vs_fp64_speedup"] = r32["mixed"]["value"] / r32["fp64"]["value"]
        if not args.no_ablation:
            ablation["si_32k"] = ablate(small, table, args, r32["mixed"])

    extra_256k = None
    if not args.no_256k:
        log("[bench] generating the 256,000-atom two-species disordered workload")
        dis = W.disordered_256k()
        t2 = W.two_species_table()
        r256 = measure_workload(dis, t2, max(args.steps, 10), args.warmup, ("mixed", "fp64"), args.batch_atoms,
                                sigma=0.005)
        extra_256k = {p: dict(value=r256[p]["value"], ms_per_step=r256[p]["ms_per_step"],
                              compute_ms=r256[p]["compute_ms"], main_ms=r256[p]["main_ms"],
                              pack_ms=r256[p]["pack_ms"], build_ms=r256[p]["build_ms"],
                              alg_tflops=r256[p]["alg_tflops"],
                              counts_per_atom={k: v / dis.n for k, v in r256[p]["counts"].items()})
                      for p in r256}
        extra_256k["mixed_vs_fp64_speedup"] = r256["mixed"]["value"] / r256["fp64"]["value"]
        if not args.no_ablation:
            ablation["disordered_256k"] = ablate(dis, t2, args, r256["mixed"], sigma=0.005)

    serve = None
    if not args.no_serve:
        log("[bench] serving benchmark")
        serve = serve_bench(table)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(big, table)
        log(f"[bench] cpu baseline {cpu['value']:.4g} atoms*evals/s on {cpu['cores']} threads")

    achieved = mixed["alg_tflops"]
    traffic = traffic_bytes()
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
            "peak": PEAK_FP32_PACKED_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_PACKED_TFLOPS,
            "traffic": traffic,
            "kernel": "k_tersoff<float, one species, lambda3 = 0" + (", fused packing> (packing, " if mixed["fused"]
                                                                       else "> (") + "energy / force / virial)",
            "kernel_ms": mixed["main_ms"],
            "alg_flops_per_launch": mixed["alg_flops_per_launch"],
            "peak_note": "FP32 vector peak (packed issue); 78.64 TFLOP/s unpacked FP32 / FP64 issue",
            "frac_vs_unpacked_issue_peak": achieved / PEAK_ALU_TFLOPS,
        },
        "pack_roofline": None if mixed["fused"] else {
            "bound": "hbm", "kernel": "k_pack<float, single-type>", "kernel_ms": mixed["pack_ms"],
            "alg_bytes_per_launch": mixed["pack_alg_bytes"], "achieved": mixed["pack_gbs"],
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": mixed["pack_gbs"] / PEAK_HBM_GBS,
        },
        "cpu_baseline": cpu,
        "step_breakdown_ms": {"pack": mixed["pack_ms"], "main": mixed["main_ms"], "gather": mixed["gather_ms"],
                              "build": mixed["build_ms"], "build_every": REBUILD_EVERY},
        "fp64": {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"], "main_ms": fp64["main_ms"],
                 "pack_ms": fp64["pack_ms"], "gather_ms": fp64["gather_ms"], "alg_tflops": fp64["alg_tflops"]},
        "single": {"value": single["value"], "ms_per_step": single["ms_per_step"], "main_ms": single["main_ms"],
                   "pack_ms": single["pack_ms"], "alg_tflops": single["alg_tflops"],
                   "note": "all-FP32 variant (FP32 zeta->b power and per-pair force sums)"},
        "mixed_vs_fp64_speedup": mixed["value"] / fp64["value"],
        "mixed_vs_fp64_compute_speedup": fp64["compute_ms"] / mixed["compute_ms"],
        "counts_per_atom": {k: v / big.n for k, v in mixed["counts"].items()},
        "si_32k": extra_32k,
        "disordered_256k_two_species": extra_256k,
        "f3_ablation": dict(ablation, note=(
            "compute-kernel time per evaluation (mixed) with one centre atom per wavefront, its packed "
            "neighbours on the lanes (the paper's J scheme on a 64-lane wavefront), and with the triplets of "
            "each batch on the lanes (zeta and force terms summed by LDS atomics), against the default "
            "batches of centre atoms whose packed pairs fill the lanes (I and J together)")) if ablation else None,
        "serve": serve,
        "packing": dict(packing, note=(
            "default: a separate packing kernel writes records, kept lists and counts for the compute kernel "
            "to read; compared with each group of centre atoms packed inside the compute kernel (FP64 "
            "displacement, cutoff test, records queued in LDS, forces stored to the plane of the centre's "
            "position in the neighbour's row)")) if packing else None,
        "f1_force_sum": dict(f1, note=(
            "default: every force term of centre i on atom j summed by the lane of pair (i, j) into a force plane "
            "of j, planes added per atom in a fixed order (no atomics, bitwise reproducible); compared with the "
            "same terms added by FP64 atomics into zeroed forces (no planes, no gather)")) if f1 else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
