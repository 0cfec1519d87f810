"""Seeded synthetic inputs for the Tersoff evaluation: silicon lattices,
disordered two-species systems, a serving stream, and parameter tables.

This module holds input construction only.  It computes none of the
potential's arithmetic (no cutoff function, no bond order, no forces), so it
can feed both the GPU library and the independent CPU checker.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.  For every
structure the draw order is fixed: strain first, then jitter (row-major
N x 3), then species.

The benchmark of the paper (a carbon-nanotube stretching run, Section 5) is
not available; these silicon structures stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Field order of one parameter-table entry (14 float64 values).  The GPU
# library and the CPU checker both read tables in this layout.
PARAM_FIELDS = ("A", "B", "lambda1", "lambda2", "lambda3", "beta", "eta",
                "c", "d", "h", "gamma", "R", "D", "m")
NPARAM = len(PARAM_FIELDS)

# Tersoff Si parameters used by every silicon workload (eV, Angstrom).
# gamma = 1 and m = 1 (lambda3 = 0 makes m irrelevant for these inputs).
SI = dict(A=1830.8, B=471.18, lambda1=2.4799, lambda2=1.7322, lambda3=0.0,
          beta=1.1e-6, eta=0.78734, c=100390.0, d=16.217, h=-0.59825,
          gamma=1.0, R=2.85, D=0.15, m=1.0)

SI_LATTICE = 5.431          # diamond lattice constant (Angstrom)
SKIN = 1.0                  # neighbour-list skin (Angstrom)

# Conventional diamond cell basis (fractional coordinates).
DIAMOND_BASIS = np.array([
    [0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def entry(**kw) -> np.ndarray:
    """One table entry from keyword values (missing keys taken from SI)."""
    p = dict(SI)
    p.update(kw)
    return np.array([float(p[k]) for k in PARAM_FIELDS], dtype=np.float64)


def species_variant(base: dict, scale_AB: float, scale_RD: float) -> dict:
    p = dict(base)
    p["A"] *= scale_AB
    p["B"] *= scale_AB
    p["R"] *= scale_RD
    p["D"] *= scale_RD
    return p


def table_from_species(species: list[dict]) -> np.ndarray:
    """Parameter table of shape (nt, nt, nt, NPARAM), entry [ti, tj, tk].

    Entries whose three types are all equal take that species' values;
    every other entry takes the arithmetic mean of the species that occur in
    it (for two species: the mean of the two)."""
    nt = len(species)
    tab = np.zeros((nt, nt, nt, NPARAM))
    for ti in range(nt):
        for tj in range(nt):
            for tk in range(nt):
                used = sorted({ti, tj, tk})
                vals = {k: float(np.mean([species[s][k] for s in used])) for k in PARAM_FIELDS}
                tab[ti, tj, tk] = [vals[k] for k in PARAM_FIELDS]
    return tab


def si_table() -> np.ndarray:
    return table_from_species([SI])


def two_species_table() -> np.ndarray:
    """Species 0 = Si; species 1 = Si with A, B x0.9 and R, D x1.04."""
    return table_from_species([SI, species_variant(SI, 0.9, 1.04)])


def table_cutoff(table: np.ndarray) -> float:
    """Largest R + D in a table (the interaction range)."""
    t = np.asarray(table).reshape(-1, NPARAM)
    return float(np.max(t[:, PARAM_FIELDS.index("R")] + t[:, PARAM_FIELDS.index("D")]))


@dataclass
class System:
    pos: np.ndarray      # (N, 3) float64, Angstrom
    types: np.ndarray    # (N,) int32
    box: np.ndarray      # (3,) float64, periodic box lengths

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def diamond(nx: int, ny: int, nz: int, a: float = SI_LATTICE, jitter: float = 0.0,
            strain: float = 0.0, seed: int = 0, ntypes: int = 1) -> System:
    """Diamond-cubic lattice of nx*ny*nz conventional cells.

    Atom index = ((ix*ny + iy)*nz + iz)*8 + b.  ``strain`` > 0 draws a uniform
    axial strain in [-strain, strain] per axis (applied affinely before the
    jitter); ``jitter`` is the per-axis Gaussian sigma in Angstrom."""
    g = rng(seed)
    eps = g.uniform(-strain, strain, size=3) if strain > 0 else np.zeros(3)
    cells = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                                 indexing="ij"), axis=-1).reshape(-1, 1, 3)
    frac = (cells + DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    scale = a * (1.0 + eps)
    pos = frac * scale[None, :]
    box = np.array([nx, ny, nz], dtype=np.float64) * scale
    n = pos.shape[0]
    if jitter > 0:
        pos = pos + g.normal(0.0, jitter, size=(n, 3))
    if ntypes > 1:
        types = species_split(n, ntypes, g)
    else:
        types = np.zeros(n, dtype=np.int32)
    return System(np.ascontiguousarray(pos), types, box)


def species_split(n: int, ntypes: int, g: np.random.Generator) -> np.ndarray:
    """Exactly equal shares of each species, randomly placed (permutation)."""
    base = np.repeat(np.arange(ntypes, dtype=np.int32), -(-n // ntypes))[:n]
    return g.permutation(base).astype(np.int32)


def perturb(pos: np.ndarray, sigma: float, g: np.random.Generator) -> np.ndarray:
    return pos + g.normal(0.0, sigma, size=pos.shape)


def disordered(n: int, density: float = 0.05, dmin: float = 2.0, seed: int = 0,
               ntypes: int = 2, batch: int = 8192) -> System:
    """Random sequential addition of n points in a cubic periodic box at the
    given number density, rejecting any point closer than dmin (minimum
    image) to an accepted one.  Proposals are drawn in batches; inside a
    batch, a proposal conflicting with an earlier one of the same batch is
    dropped.  Species are assigned in exactly equal shares by permutation."""
    from scipy.spatial import cKDTree

    g = rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    acc = np.zeros((0, 3))
    while acc.shape[0] < n:
        cand = g.uniform(0.0, L, size=(batch, 3))
        if acc.shape[0]:
            tree = cKDTree(acc, boxsize=L)
            dist, _ = tree.query(cand, k=1, distance_upper_bound=dmin)
            cand = cand[~np.isfinite(dist) | (dist >= dmin)]
        if cand.shape[0] > 1:
            pairs = cKDTree(cand, boxsize=L).query_pairs(dmin, output_type="ndarray")
            keep = np.ones(cand.shape[0], dtype=bool)
            if pairs.size:
                pairs = np.sort(pairs, axis=1)
                order = np.lexsort((pairs[:, 1], pairs[:, 0]))
                for a, b in pairs[order]:
                    if keep[a]:
                        keep[b] = False
            cand = cand[keep]
        acc = np.concatenate([acc, cand[: n - acc.shape[0]]])
    # cKDTree needs coordinates in [0, L); keep them so.
    acc = np.minimum(acc, np.nextafter(L, 0.0))
    types = species_split(n, ntypes, g) if ntypes > 1 else np.zeros(n, np.int32)
    return System(np.ascontiguousarray(acc), types, np.array([L, L, L]))


def serve_stream(count: int = 4096, seed: int = 0, nmin: int = 64, nmax: int = 4096,
                 strain: float = 0.03, jitter: float = 0.08) -> list[System]:
    """Independent periodic diamond-Si cells with log-uniform target sizes.

    For a target size N: n = max(2, round((N/8)^(1/3))),
    m = max(2, round(N/(8 n^2))); the cell is n x n x m conventional cells."""
    g = rng(seed)
    targets = np.exp(g.uniform(math.log(nmin), math.log(nmax), size=count))
    seeds = g.integers(0, 2**63 - 1, size=count)
    out = []
    for N, s in zip(targets, seeds):
        nn = max(2, int(round((N / 8.0) ** (1.0 / 3.0))))
        mm = max(2, int(round(N / (8.0 * nn * nn))))
        out.append(diamond(nn, nn, mm, jitter=jitter, strain=strain, seed=int(s)))
    return out


# Named workloads (sizes of the benchmark configurations).
def si_512(seed: int = 1) -> System:
    return diamond(4, 4, 4, jitter=0.05, seed=seed)


def si_32k(seed: int = 2) -> System:
    return diamond(20, 20, 10, jitter=0.1, seed=seed)


def si_2m(seed: int = 3) -> System:
    return diamond(80, 80, 40, jitter=0.1, strain=0.02, seed=seed)


def disordered_256k(seed: int = 4) -> System:
    return disordered(256_000, density=0.05, dmin=2.0, seed=seed, ntypes=2)
