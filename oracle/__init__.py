"""FP64 CPU oracle for the Tersoff potential (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The GPU library never imports, links or calls it, and it never
imports the GPU library.

``tersoff_oracle.c`` is the plain C implementation of Eq. (1)-(3) (Section
2): the energy, and the forces as its gradient by the chain rule;
``brute.py`` is an independent numpy evaluation of
the energy with no neighbour list.  This module compiles the C file with gcc
(once, on first use, or from ``build()``) and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tersoff_oracle.c")
_LIB = os.path.join(_HERE, "libtersoff_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library (gcc, -O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                        "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_neighbors_brute.argtypes = [i64, P, P, f64, P, P, i64]
        lib.oracle_neighbors_brute.restype = i64
        lib.oracle_neighbors_cell.argtypes = [i64, P, P, f64, P, P, i64]
        lib.oracle_neighbors_cell.restype = i64
        lib.oracle_compute.argtypes = [i64, P, P, P, P, i32, P, P, i64, i64, i32, P, P, P]
        lib.oracle_compute.restype = ctypes.c_int
        lib.oracle_counts.argtypes = [i64, P, P, P, P, i32, P, P, i64, i64, P]
        lib.oracle_counts.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(pos, box):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    return pos, box


def neighbors(pos, box, rcut: float, method: str = "cell"):
    """Full neighbour list: (offsets int64[N+1], idx int32[S]), rows sorted.

    Every j != i with min-image r^2 < rcut^2."""
    lib = _load()
    pos, box = _prep(pos, box)
    n = pos.shape[0]
    fn = lib.oracle_neighbors_cell if method == "cell" else lib.oracle_neighbors_brute
    offsets = np.zeros(n + 1, dtype=np.int64)
    cap = max(16 * n, 1)
    while True:
        idx = np.zeros(cap, dtype=np.int32)
        total = fn(n, _p(pos), _p(box), float(rcut), _p(offsets), _p(idx), cap)
        if total <= cap:
            return offsets, idx[:total].copy()
        cap = int(total)


def table_array(table, ntypes: int | None = None):
    t = np.ascontiguousarray(table, dtype=np.float64)
    if ntypes is None:
        ntypes = int(round((t.size // 14) ** (1.0 / 3.0)))
    assert t.size == ntypes ** 3 * 14, "table must hold ntypes^3 entries of 14 values"
    return t.reshape(-1), ntypes


def compute(pos, types, box, table, offsets, idx, i0: int = 0, i1: int | None = None,
            threads: int = 1):
    """Energy (eV), forces (N x 3, eV/A) and virial (xx yy zz xy xz yz, eV).

    Contributions of centre atoms i in [i0, i1) only (default: all)."""
    lib = _load()
    pos, box = _prep(pos, box)
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    tab, nt = table_array(table)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    forces = np.zeros((n, 3))
    virial = np.zeros(6)
    energy = np.zeros(1)
    rc = lib.oracle_compute(n, _p(pos), _p(types), _p(box), _p(tab), nt, _p(offsets), _p(idx),
                            int(i0), int(n if i1 is None else i1), int(threads),
                            _p(energy), _p(forces), _p(virial))
    if rc != 0:
        raise ValueError(f"oracle_compute failed ({rc})")
    return float(energy[0]), forces, virial


def counts(pos, types, box, table, offsets, idx, i0: int = 0, i1: int | None = None):
    """(S, P, T): list entries, in-cutoff ordered pairs, ordered triplets."""
    lib = _load()
    pos, box = _prep(pos, box)
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    tab, nt = table_array(table)
    out = np.zeros(3, dtype=np.int64)
    lib.oracle_counts(n, _p(pos), _p(types), _p(box), _p(tab), nt,
                      _p(np.ascontiguousarray(offsets, dtype=np.int64)),
                      _p(np.ascontiguousarray(idx, dtype=np.int32)),
                      int(i0), int(n if i1 is None else i1), _p(out))
    return tuple(int(v) for v in out)


def evaluate(pos, types, box, table, skin: float = 1.0, threads: int = 1):
    """Neighbour list at cutoff + skin, then compute()."""
    tab = np.asarray(table).reshape(-1, 14)
    rcut = float(np.max(tab[:, 11] + tab[:, 12]))
    off, idx = neighbors(pos, box, rcut + skin)
    return compute(pos, types, box, table, off, idx, threads=threads)
