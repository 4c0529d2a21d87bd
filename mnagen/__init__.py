"""Seeded synthetic circuit matrices (modified nodal analysis) and value streams.

This module only assembles inputs: MNA stamps of resistors, capacitor companion
conductances, vias, pads, ideal voltage sources and transistor-like 4x4 stamps,
plus per-step value perturbations and right-hand sides.  It holds none of the
solver's arithmetic, so both the CPU oracle and the GPU library can be fed from
it without sharing any method code.

Every generator is deterministic in its seed.  Matrices come back in CSC form
(0-based, rows sorted inside each column, duplicates summed, explicit zeros
kept) as ``Circuit`` objects.

The workload classes follow the circuit families the paper evaluates: small
pre-layout circuits, post-layout RC meshes, mesh-plus-transistor circuits and
IBM-style power grids (Section VI).  None of the paper's benchmark matrices is
reproduced; these are stand-ins of the same shape and value spread.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Circuit", "assemble", "mesh_vsrc", "layered_rc", "mesh_transistor",
    "power_grid", "perturb", "restamp", "instance_values", "Stamping", "random_rhs", "step_rng",
    "random_pattern", "hand_pattern", "random_values", "serving_mix", "mix_circuit",
    "CONFIGS",
]


@dataclass
class Circuit:
    """A square sparse matrix in CSC form plus right-hand sides."""
    n: int
    colptr: np.ndarray          # int32 [n+1]
    rowind: np.ndarray          # int32 [nnz]
    values: np.ndarray          # float64 [nnz]
    rhs: np.ndarray             # float64 [nrhs, n]
    name: str = ""
    meta: dict = field(default_factory=dict)
    stamping: "Stamping | None" = None

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_scipy(self, values=None) -> sp.csc_matrix:
        v = self.values if values is None else values
        return sp.csc_matrix((v, self.rowind, self.colptr), shape=(self.n, self.n))


def assemble(n, rows, cols, vals) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Sum triplets into CSC (sorted rows, explicit zeros kept)."""
    m = sp.coo_matrix((np.asarray(vals, dtype=np.float64),
                       (np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64))),
                      shape=(n, n)).tocsc()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int32), m.indices.astype(np.int32),
            m.data.astype(np.float64))


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _grid_edges(nx, ny, offset=0):
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx) + offset
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)
    return np.concatenate([h, v])


class _Stamps:
    """Triplet accumulator for MNA stamps that remembers which element made each entry.

    Every resistor, via, pad, capacitor companion or transistor stamp is one
    element; ideal-source incidence entries are fixed elements (never scaled).
    build() returns the CSC matrix and a Stamping that re-assembles the matrix
    for any per-element scale factors.
    """

    def __init__(self):
        self.r, self.c, self.v, self.e = [], [], [], []
        self.nelem = 0
        self.fixed = []

    def _ids(self, m, fixed=False):
        ids = np.arange(self.nelem, self.nelem + m, dtype=np.int64)
        self.nelem += m
        if fixed:
            self.fixed.append(ids)
        return ids

    def conductance(self, a, b, g):
        a = np.asarray(a, np.int64); b = np.asarray(b, np.int64); g = np.asarray(g, np.float64)
        ids = self._ids(a.size)
        self.r += [a, b, a, b]; self.c += [a, b, b, a]; self.v += [g, g, -g, -g]; self.e += [ids] * 4

    def diag(self, a, g):
        a = np.asarray(a, np.int64)
        self.r.append(a); self.c.append(a); self.v.append(np.broadcast_to(np.asarray(g, np.float64), a.shape))
        self.e.append(self._ids(a.size))

    def entry(self, r, c, v, group=1, fixed=False):
        """Entries r, c, v; each run of `group` consecutive entries is one element."""
        r = np.asarray(r, np.int64); c = np.asarray(c, np.int64)
        self.r.append(r); self.c.append(c); self.v.append(np.broadcast_to(np.asarray(v, np.float64), r.shape))
        ids = self._ids(r.size // group, fixed)
        self.e.append(np.repeat(ids, group))

    def build(self, n):
        r = np.concatenate(self.r); c = np.concatenate(self.c)
        v = np.concatenate(self.v).astype(np.float64); e = np.concatenate(self.e)
        key = c * n + r                                     # column-major order = CSC order
        ukey, pos = np.unique(key, return_inverse=True)
        colptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(colptr, (ukey // n) + 1, 1)
        colptr = np.cumsum(colptr).astype(np.int32)
        rowind = (ukey % n).astype(np.int32)
        fixed = np.zeros(self.nelem, dtype=bool)
        for ids in self.fixed:
            fixed[ids] = True
        st = Stamping(pos.astype(np.int64), v, e, self.nelem, fixed, int(ukey.size))
        return colptr, rowind, st.values(), st


@dataclass
class Stamping:
    """Per-entry provenance of an assembled MNA matrix."""
    pos: np.ndarray        # nonzero index each triplet adds into
    val: np.ndarray        # triplet value
    elem: np.ndarray       # element id of each triplet
    nelem: int
    fixed: np.ndarray      # elements that are never scaled (ideal-source incidences)
    nnz: int

    def values(self, factors=None):
        w = self.val if factors is None else self.val * factors[self.elem]
        return np.bincount(self.pos, weights=w, minlength=self.nnz).astype(np.float64)

    def factors(self, rng, lo, hi):
        f = rng.uniform(lo, hi, self.nelem)
        f[self.fixed] = 1.0
        return f


def _transistor_stamps(st, rng, nx, ny, layers, count, sigma=1e-2, diag=0.05):
    """4x4 unsymmetric stamps on the 2x2 node square at a random site and layer."""
    x = rng.integers(0, nx - 1, count)
    y = rng.integers(0, ny - 1, count)
    lay = rng.integers(0, layers, count)
    base = lay * nx * ny + y * nx + x
    nodes = np.stack([base, base + 1, base + nx, base + nx + 1], 1)      # [count, 4]
    rr = np.repeat(nodes, 4, axis=1)                                     # row index of each of 16
    cc = np.tile(nodes, (1, 4))
    vals = rng.normal(0.0, sigma, (count, 16))
    vals[:, [0, 5, 10, 15]] += diag
    st.entry(rr.ravel(), cc.ravel(), vals.ravel(), group=16)


def random_rhs(rng, n, nrhs=1):
    return rng.uniform(-1.0, 1.0, (nrhs, n))


def mesh_vsrc(nx=32, ny=32, n_vsrc=4, seed=0, glo=1e-3, ghi=1e3, gmin=1e-12) -> Circuit:
    """2D resistor mesh with ideal voltage sources at the corners.

    Each source adds an MNA row/column k with A(p,k)=A(k,p)=1 and no (k,k)
    entry, so the matrix is unsymmetric in values and has zero diagonals.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1]))
    nn = nx * ny
    n = nn + n_vsrc
    st = _Stamps()
    e = _grid_edges(nx, ny)
    st.conductance(e[:, 0], e[:, 1], _loguniform(rng, glo, ghi, len(e)))
    st.diag(np.arange(nn), gmin)
    corners = [0, nx - 1, (ny - 1) * nx, ny * nx - 1]
    for s in range(n_vsrc):
        p = corners[s % 4] if s < 4 else int(rng.integers(0, nn))
        k = nn + s
        st.entry([p, k], [k, p], [1.0, 1.0], group=2, fixed=True)
    ap, ai, ax, stp = st.build(n)
    return Circuit(n, ap, ai, ax, random_rhs(rng, n), name=f"mesh_vsrc_{nx}x{ny}",
                   meta=dict(nx=nx, ny=ny, n_vsrc=n_vsrc, seed=seed), stamping=stp)


def layered_rc(nx=300, ny=300, layers=3, via_frac=0.01, stamp_frac=0.1, seed=0,
               glo=1e-3, ghi=1e3, cap=1e-3, gvia=10.0) -> Circuit:
    """Post-layout-like RC mesh: stacked 2D layers, vias, transistor stamps."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    nl = nx * ny
    n = nl * layers
    st = _Stamps()
    for l in range(layers):
        e = _grid_edges(nx, ny, l * nl)
        st.conductance(e[:, 0], e[:, 1], _loguniform(rng, glo, ghi, len(e)))
    st.diag(np.arange(n), cap)
    nvia = int(round(via_frac * nl))
    for l in range(layers - 1):
        sites = rng.choice(nl, nvia, replace=False)
        st.conductance(l * nl + sites, (l + 1) * nl + sites, np.full(nvia, gvia))
    _transistor_stamps(st, rng, nx, ny, layers, int(stamp_frac * n))
    ap, ai, ax, stp = st.build(n)
    return Circuit(n, ap, ai, ax, random_rhs(rng, n), name=f"layered_rc_{layers}x{nx}x{ny}",
                   meta=dict(nx=nx, ny=ny, layers=layers, seed=seed), stamping=stp)


def mesh_transistor(nx=141, ny=141, stamp_frac=0.1, seed=0, glo=1e-3, ghi=1e3,
                    cap=1e-3) -> Circuit:
    """Single-layer 2D mesh plus transistor-like stamps."""
    c = layered_rc(nx, ny, 1, 0.0, stamp_frac, seed=seed, glo=glo, ghi=ghi, cap=cap)
    c.name = f"mesh_transistor_{nx}x{ny}"
    return c


def power_grid(nx=1000, ny=1000, pad_frac=0.005, n_src=1000, nrhs=8, seed=0,
               glo=1e-3, ghi=1e3, gmin=1e-12, gpad=100.0, ilo=1e-3, ihi=1e-2) -> Circuit:
    """IBM-style power grid: resistive mesh, pads to ground, current loads."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    n = nx * ny
    st = _Stamps()
    e = _grid_edges(nx, ny)
    st.conductance(e[:, 0], e[:, 1], _loguniform(rng, glo, ghi, len(e)))
    st.diag(np.arange(n), gmin)
    npad = max(1, int(round(pad_frac * n)))
    st.diag(rng.choice(n, npad, replace=False), gpad)
    ap, ai, ax, stp = st.build(n)
    rhs = np.zeros((nrhs, n))
    for r in range(nrhs):
        nodes = rng.choice(n, min(n_src, n), replace=False)
        rhs[r, nodes] = rng.uniform(ilo, ihi, len(nodes))
    return Circuit(n, ap, ai, ax, rhs, name=f"power_grid_{nx}x{ny}",
                   meta=dict(nx=nx, ny=ny, seed=seed), stamping=stp)


def step_rng(seed, cfg, t):
    """Generator of NR step t of configuration cfg."""
    return np.random.default_rng(np.random.SeedSequence([seed, cfg, t]))


def restamp(c, seed, cfg, t, rel=0.05):
    """Per-step values of an NR iteration: every circuit element (resistor, via, pad,
    capacitor companion, transistor stamp) scaled by its own U[1-rel, 1+rel] factor
    and the matrix re-assembled, as a simulator re-stamps its devices (not cumulative;
    ideal-source incidences stay fixed)."""
    if c.stamping is None:          # no element provenance: every nonzero is its own element
        return perturb(c.values, seed, cfg, t, rel)
    f = c.stamping.factors(step_rng(seed, cfg, t), 1.0 - rel, 1.0 + rel)
    return c.stamping.values(f)


def perturb(values, seed, cfg, t, rel=0.05):
    """Stress recipe: every assembled nonzero times an independent U[1-rel, 1+rel].

    This breaks the element structure of the matrix (row sums no longer match the
    element conductances), which makes pivots flip far more often than in an NR run."""
    return values * step_rng(seed, cfg, t).uniform(1.0 - rel, 1.0 + rel, values.shape)


def instance_values(c, batch, sigma=0.3, seed=0):
    """Monte-Carlo corners: per-instance, per-element factor exp(sigma*N(0,1)), re-assembled."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3, batch]))
    out = np.empty((batch, c.nnz))
    for i in range(batch):
        f = np.exp(sigma * rng.standard_normal(c.stamping.nelem))
        f[c.stamping.fixed] = 1.0
        out[i] = c.stamping.values(f)
    return out


def random_values(rng, nnz, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, nnz)


def random_pattern(n, density, seed, diag=True, values=True):
    """Random unsymmetric sparse matrix (CSC); diag=True forces a full diagonal."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 100, n]))
    m = int(round(density * n * n))
    r = rng.integers(0, n, m); c = rng.integers(0, n, m)
    if diag:
        r = np.concatenate([r, np.arange(n)]); c = np.concatenate([c, np.arange(n)])
    v = rng.uniform(-1.0, 1.0, r.size)
    if diag:
        v[-n:] += np.where(rng.uniform(size=n) < 0.5, -4.0, 4.0)
    ap, ai, ax = assemble(n, r, c, v)
    return Circuit(n, ap, ai, ax, random_rhs(rng, n), name=f"random_{n}_{density}")


def hand_pattern(kind, n, seed=0):
    """Hand-made structures with known closed-form factor patterns."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 200, n]))
    r, c, v = [], [], []
    if kind == "diagonal":
        r = list(range(n)); c = list(range(n)); v = list(rng.uniform(1, 2, n))
    elif kind == "tridiagonal":          # diagonally dominant
        for i in range(n):
            r.append(i); c.append(i); v.append(4.0 + rng.uniform())
            if i + 1 < n:
                r += [i, i + 1]; c += [i + 1, i]; v += list(rng.uniform(-1, 1, 2))
    elif kind in ("arrow_last", "arrow_first"):
        hub = n - 1 if kind == "arrow_last" else 0
        for i in range(n):
            r.append(i); c.append(i); v.append(float(n) + rng.uniform())
            if i != hub:
                r += [i, hub]; c += [hub, i]; v += list(rng.uniform(-1, 1, 2))
    elif kind == "permutation":
        p = rng.permutation(n)
        while n > 1 and np.any(p == np.arange(n)):
            p = rng.permutation(n)
        r = list(p); c = list(range(n)); v = list(rng.uniform(1, 2, n))
    elif kind == "dense":
        rr, cc = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        r = rr.ravel(); c = cc.ravel(); v = rng.uniform(-1, 1, n * n) + 3.0 * (r == c)
    elif kind == "laplacian2d":          # n = side*side
        side = int(round(np.sqrt(n)))
        assert side * side == n
        st = _Stamps()
        e = _grid_edges(side, side)
        st.conductance(e[:, 0], e[:, 1], np.ones(len(e)))
        st.diag(np.arange(n), 0.5)
        ap, ai, ax, stp = st.build(n)
        return Circuit(n, ap, ai, ax, random_rhs(rng, n), name=f"laplacian2d_{side}", stamping=stp)
    else:
        raise ValueError(kind)
    ap, ai, ax = assemble(n, r, c, v)
    return Circuit(n, ap, ai, ax, random_rhs(rng, n), name=f"{kind}_{n}")


def serving_mix(n_requests, seed=0, nmin=1000, nmax=200_000):
    """Request sizes for the serving mix: n log-uniform in [nmin, nmax]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 5]))
    ns = np.exp(rng.uniform(np.log(nmin), np.log(nmax), n_requests))
    kinds = rng.integers(0, 3, n_requests)
    return [(int(k), int(v)) for k, v in zip(kinds, ns)]


def mix_circuit(kind, n, seed=0) -> Circuit:
    """A circuit of the serving mix with about n unknowns: kind 0 a mesh with
    ideal voltage sources, 1 a three-layer RC mesh, 2 a mesh with transistor
    stamps, 3 a power grid."""
    side = max(8, int(round(np.sqrt(n))))
    if kind == 0:
        return mesh_vsrc(side, side, 4, seed)
    if kind == 1:
        s3 = max(6, int(round(np.sqrt(n / 3.0))))
        return layered_rc(s3, s3, 3, seed=seed)
    if kind == 2:
        return mesh_transistor(side, side, seed=seed)
    return power_grid(side, side, n_src=max(10, n // 1000), nrhs=1, seed=seed)


# Configurations: name -> factory(seed) at full size, and a reduced size that the
# oracle finishes in seconds.
CONFIGS = {
    "mesh_vsrc_32": lambda seed=0: mesh_vsrc(32, 32, 4, seed),
    "layered_rc_3x300": lambda seed=0: layered_rc(300, 300, 3, seed=seed),
    "mesh_transistor_141": lambda seed=0: mesh_transistor(141, 141, seed=seed),
    "power_grid_1000": lambda seed=0: power_grid(1000, 1000, seed=seed),
    # reduced sizes
    "layered_rc_3x40": lambda seed=0: layered_rc(40, 40, 3, seed=seed),
    "mesh_transistor_60": lambda seed=0: mesh_transistor(60, 60, seed=seed),
    "power_grid_100": lambda seed=0: power_grid(100, 100, n_src=100, seed=seed),
}
