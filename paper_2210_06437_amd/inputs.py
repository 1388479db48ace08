"""Seeded synthetic workloads for the octree hydro step.

This module is shared by the tests (oracle side) and by ``bench.py`` (HIP
side).  It only *builds inputs*: leaf lists of a periodic octree of 8^3
sub-grids (Sec. IV-C of the paper) and initial states sampled at cell
centres.  It contains none of the solver's arithmetic (no reconstruction,
flux, update, time-step or ghost fill); the conversion from the sampled
primitive state (rho, v, p) to the stored conserved fields is part of the
input recipe.

The paper's production input (the V1309 merger files) is not available; these
workloads stand in for it with the shapes of the five benchmark cases:

1. one 8^3 sub-grid, periodic, smooth density + noise, uniform drift;
2. 16^3 = 4096 sub-grids, Sod tube along x with transverse noise;
3. uneven octree (levels 0-3) refined around two Gaussian blobs, 11 fields;
4. case 2 in FP32 storage;
5. 32^3 base grid with 4681 sub-grids refined once (65535 leaves), lognormal
   density and a Kolmogorov-spectrum solenoidal velocity, 11 fields.

Field order: rho, s_x, s_y, s_z, E, tau, rho_0..rho_4.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED0 = 2210064370
GAMMA = 5.0 / 3.0
SUB = 8


@dataclass
class Workload:
    name: str
    base: int
    leaf_coord: np.ndarray          # int32 [n][4]: level, ix, iy, iz
    U: np.ndarray                   # float64 [nf][n][8][8][8]
    cfl: float = 0.4
    steps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_coord.shape[0])

    @property
    def nf(self) -> int:
        return int(self.U.shape[0])

    @property
    def n_cells(self) -> int:
        return self.n_leaves * SUB ** 3


# --------------------------------------------------------------------------
# Octree leaf lists
# --------------------------------------------------------------------------

def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_order(coord: np.ndarray) -> np.ndarray:
    """Permutation sorting leaves along the Morton curve of their lower corner
    at the finest level present (parents of a region come before it)."""
    lmax = int(coord[:, 0].max()) if len(coord) else 0
    sh = (lmax - coord[:, 0]).astype(np.uint64)
    x = coord[:, 1].astype(np.uint64) << sh
    y = coord[:, 2].astype(np.uint64) << sh
    z = coord[:, 3].astype(np.uint64) << sh
    key = _part1by2(x) | (_part1by2(y) << np.uint64(1)) | (_part1by2(z) << np.uint64(2))
    return np.lexsort((coord[:, 0], key))


def uniform_leaves(base: int) -> np.ndarray:
    z, y, x = np.meshgrid(np.arange(base), np.arange(base), np.arange(base), indexing="ij")
    c = np.stack([np.zeros(base ** 3, np.int64), x.ravel(), y.ravel(), z.ravel()], 1)
    c = c[morton_order(c)]
    return np.ascontiguousarray(c, dtype=np.int32)


def cell_centres(coord: np.ndarray, base: int):
    """Cell-centre positions x, y, z with shape [n][8][8][8] (z, y, x order)."""
    lev = coord[:, 0].astype(np.float64)
    dx = 1.0 / (SUB * base * 2.0 ** lev)
    i = np.arange(SUB, dtype=np.float64) + 0.5
    x = (SUB * coord[:, 1, None] + i[None, :]) * dx[:, None]
    y = (SUB * coord[:, 2, None] + i[None, :]) * dx[:, None]
    z = (SUB * coord[:, 3, None] + i[None, :]) * dx[:, None]
    X = np.broadcast_to(x[:, None, None, :], (len(coord), SUB, SUB, SUB))
    Y = np.broadcast_to(y[:, None, :, None], (len(coord), SUB, SUB, SUB))
    Z = np.broadcast_to(z[:, :, None, None], (len(coord), SUB, SUB, SUB))
    return X, Y, Z


def _containing_level(leafset: set, level: int, x: int, y: int, z: int):
    for l in range(level, -1, -1):
        s = level - l
        if (l, x >> s, y >> s, z >> s) in leafset:
            return l
    return None


def balance_2to1(leaves: set, base: int) -> set:
    """Refine coarse leaves until every leaf's 26 neighbours are within one
    level ("properly nested", Sec. IV-C), periodic in all axes."""
    leaves = set(leaves)
    changed = True
    while changed:
        changed = False
        to_refine = set()
        for (L, x, y, z) in leaves:
            if L < 2:
                continue
            m = base << L
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if dx == dy == dz == 0:
                            continue
                        nx, ny, nz = (x + dx) % m, (y + dy) % m, (z + dz) % m
                        l = _containing_level(leaves, L, nx, ny, nz)
                        if l is not None and l < L - 1:
                            s = L - l
                            to_refine.add((l, nx >> s, ny >> s, nz >> s))
        for leaf in to_refine:
            L, x, y, z = leaf
            leaves.discard(leaf)
            for q in range(8):
                leaves.add((L + 1, 2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2)))
            changed = True
    return leaves


def refine_by(base: int, max_level: int, flag) -> np.ndarray:
    """Refine level by level: a leaf is split when flag(coord[1][4]) says so."""
    leaves = set(map(tuple, uniform_leaves(base).tolist()))
    for L in range(max_level):
        cur = np.array(sorted(l for l in leaves if l[0] == L), dtype=np.int64).reshape(-1, 4)
        if len(cur) == 0:
            break
        hit = flag(cur)
        for leaf in map(tuple, cur[hit].tolist()):
            leaves.discard(leaf)
            Lq, x, y, z = leaf
            for q in range(8):
                leaves.add((Lq + 1, 2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2)))
        leaves = balance_2to1(leaves, base)
    c = np.array(sorted(leaves), dtype=np.int64)
    c = c[morton_order(c)]
    return np.ascontiguousarray(c, dtype=np.int32)


# --------------------------------------------------------------------------
# Initial states
# --------------------------------------------------------------------------

def conserved(rho, vx, vy, vz, p, species=None, gamma=GAMMA):
    """Stored fields from a primitive state: s = rho v,
    E = p/(gamma-1) + rho |v|^2 / 2, tau = (p/(gamma-1))^(1/gamma)."""
    eint = p / (gamma - 1.0)
    E = eint + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    tau = eint ** (1.0 / gamma)
    fields = [rho, rho * vx, rho * vy, rho * vz, E, tau]
    if species is not None:
        fields += [rho * s for s in species]
    return np.ascontiguousarray(np.stack(fields, 0), dtype=np.float64)


def _dirichlet_species(rng, shape, k=5):
    g = rng.standard_exponential(size=(k,) + tuple(shape))
    return list(g / g.sum(0))


def config1(seed_offset: int = 1) -> Workload:
    """One periodic 8^3 sub-grid: rho = 1 + 0.1 sin sin sin + U(-1e-3, 1e-3),
    p = 1, v = 0.1 * (one seeded unit vector); one forward-Euler substep."""
    rng = np.random.default_rng(SEED0 + seed_offset)
    coord = uniform_leaves(1)
    X, Y, Z = cell_centres(coord, 1)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
    rho = rho + rng.uniform(-1e-3, 1e-3, size=rho.shape)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    v = 0.1 * n
    p = np.ones_like(rho)
    U = conserved(rho, v[0] + 0 * rho, v[1] + 0 * rho, v[2] + 0 * rho, p)
    return Workload("single 8^3 sub-grid, smooth density + noise, FP64, 6 fields", 1, coord, U,
                    cfl=0.4, steps=1, meta={"direction": n.tolist()})


def sod(base: int = 16, seed_offset: int = 2, noise: float = 1e-4, steps: int = 10) -> Workload:
    """Sod tube along x on a uniform level (rho, p = 1, 1 for x < 0.5 and
    0.125, 0.1 otherwise), v_x = 0, v_y and v_z uniform in +-noise."""
    rng = np.random.default_rng(SEED0 + seed_offset)
    coord = uniform_leaves(base)
    X, _, _ = cell_centres(coord, base)
    left = X < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    vy = rng.uniform(-noise, noise, size=rho.shape) if noise else np.zeros_like(rho)
    vz = rng.uniform(-noise, noise, size=rho.shape) if noise else np.zeros_like(rho)
    U = conserved(rho, np.zeros_like(rho), vy, vz, p)
    return Workload(f"Sod tube along x, {base}^3 sub-grids ({SUB * base}^3 cells), FP64, 6 fields",
                    base, coord, U, cfl=0.4, steps=steps)


def config2() -> Workload:
    return sod(16, 2, 1e-4, 10)


def blobs(base: int = 8, max_level: int = 3, seed_offset: int = 3, steps: int = 5,
          threshold: float = 0.05) -> Workload:
    """Two Gaussian density blobs (peak 1, background 1e-4, half-widths at
    half maximum 0.1 and 0.07, centres 0.4 apart) on an octree refined where
    any cell-centre density exceeds 0.05, p = rho^(5/3), circular-orbit
    velocities, 5 Dirichlet-distributed species."""
    rng = np.random.default_rng(SEED0 + seed_offset)
    cen = np.array([[0.3, 0.5, 0.5], [0.7, 0.5, 0.5]])
    rad = np.array([0.1, 0.07])
    ln2 = np.log(2.0)

    def blob_terms(X, Y, Z):
        out = []
        for c, r in zip(cen, rad):
            d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
            out.append(np.exp(-ln2 * d2 / (r * r)))
        return out

    def flag(cur):
        X, Y, Z = cell_centres(cur, base)
        g = blob_terms(X, Y, Z)
        rho = 1e-4 + g[0] + g[1]
        return (rho > threshold).reshape(len(cur), -1).any(1)

    coord = refine_by(base, max_level, flag)
    X, Y, Z = cell_centres(coord, base)
    g = blob_terms(X, Y, Z)
    rho = 1e-4 + g[0] + g[1]
    mass = np.pi ** 1.5 * (rad / np.sqrt(ln2)) ** 3
    xcm = (mass[:, None] * cen).sum(0) / mass.sum()
    omega = np.sqrt(mass.sum() / 0.4 ** 3)
    vx = np.zeros_like(rho)
    vy = np.zeros_like(rho)
    for k in range(2):
        w = g[k] / rho
        rx, ry = cen[k, 0] - xcm[0], cen[k, 1] - xcm[1]
        vx += w * (-omega * ry)
        vy += w * (omega * rx)
    p = rho ** GAMMA
    U = conserved(rho, vx, vy, np.zeros_like(rho), p, _dirichlet_species(rng, rho.shape))
    levels = np.bincount(coord[:, 0], minlength=max_level + 1).tolist()
    return Workload(f"uneven octree around two blobs, base {base}^3, levels 0-{max_level}, FP64, "
                    f"11 fields", base, coord, U, cfl=0.4, steps=steps,
                    meta={"leaves_per_level": levels})


def config3() -> Workload:
    return blobs(8, 3, 3, 5)


def config4() -> Workload:
    w = sod(16, 4, 1e-4, 100)
    w.name = "Sod tube, 16^3 sub-grids, FP32 storage, 6 fields"
    return w


def turbulence(base: int = 32, n_refine: int = 4681, seed_offset: int = 5,
               mach: float = 0.5) -> Workload:
    """Lognormal density rho = exp(0.1 g - 0.005) (g: unit white noise per
    cell), solenoidal Gaussian velocity with power spectrum k^(-11/3) for
    1 <= |k| <= N/2, rms Mach `mach` at p = 1; the n_refine sub-grids with
    the largest max |v| are refined once (cells inherit the parent value)."""
    rng = np.random.default_rng(SEED0 + seed_offset)
    N = SUB * base
    g = rng.standard_normal((N, N, N))
    rho_g = np.exp(0.1 * g - 0.005)
    del g
    k1 = np.fft.fftfreq(N, 1.0 / N)
    kr = np.fft.rfftfreq(N, 1.0 / N)
    KZ, KY, KX = np.meshgrid(k1, k1, kr, indexing="ij", sparse=True)
    K2 = KX * KX + KY * KY + KZ * KZ
    Kmag = np.sqrt(K2)
    amp = np.where((Kmag >= 1.0) & (Kmag <= N // 2), np.power(np.maximum(Kmag, 1.0), -11.0 / 6.0),
                   0.0)
    what = []
    for _ in range(3):
        re = rng.standard_normal(amp.shape)
        im = rng.standard_normal(amp.shape)
        what.append((re + 1j * im) * amp)
    del amp
    K2s = np.where(K2 == 0, 1.0, K2)
    kdotw = KX * what[0] + KY * what[1] + KZ * what[2]
    for i, Kc in enumerate((KX, KY, KZ)):
        what[i] = what[i] - Kc * kdotw / K2s
    del kdotw, K2s
    v = [np.fft.irfftn(w, s=(N, N, N), axes=(0, 1, 2)) for w in what]
    del what
    vrms = np.sqrt((v[0] ** 2 + v[1] ** 2 + v[2] ** 2).mean())
    scale = mach * np.sqrt(GAMMA) / vrms
    vg = [vi * scale for vi in v]
    del v
    # level-0 leaves and their max |v|
    c0 = uniform_leaves(base)

    def per_leaf(a, coord):
        # a[z, y, x] on the level-0 grid -> [n][8][8][8]
        ix, iy, iz = coord[:, 1], coord[:, 2], coord[:, 3]
        o = np.arange(SUB)
        zz = (SUB * iz[:, None] + o)[:, :, None, None]
        yy = (SUB * iy[:, None] + o)[:, None, :, None]
        xx = (SUB * ix[:, None] + o)[:, None, None, :]
        return a[zz, yy, xx]

    speed = np.sqrt(vg[0] ** 2 + vg[1] ** 2 + vg[2] ** 2)
    vmax = per_leaf(speed, c0).reshape(len(c0), -1).max(1)
    del speed
    order = np.lexsort((np.arange(len(c0)), -vmax))  # leaves are already in Morton order
    refine = np.zeros(len(c0), bool)
    refine[order[:n_refine]] = True
    kids = []
    for leaf in c0[refine]:
        for q in range(8):
            kids.append((1, 2 * leaf[1] + (q & 1), 2 * leaf[2] + ((q >> 1) & 1),
                         2 * leaf[3] + (q >> 2)))
    coord = np.concatenate([c0[~refine].astype(np.int64), np.array(kids, np.int64).reshape(-1, 4)])
    coord = np.ascontiguousarray(coord[morton_order(coord)], dtype=np.int32)
    # sample: a level-1 cell inherits the level-0 cell that contains it
    L = coord[:, 0].astype(np.int64)
    o = np.arange(SUB)
    gz = ((SUB * coord[:, 3, None].astype(np.int64) + o) >> L[:, None])[:, :, None, None]
    gy = ((SUB * coord[:, 2, None].astype(np.int64) + o) >> L[:, None])[:, None, :, None]
    gx = ((SUB * coord[:, 1, None].astype(np.int64) + o) >> L[:, None])[:, None, None, :]
    rho = rho_g[gz, gy, gx]
    vx, vy, vz = (vi[gz, gy, gx] for vi in vg)
    del rho_g, vg
    p = np.ones_like(rho)
    U = conserved(rho, vx, vy, vz, p, _dirichlet_species(rng, rho.shape))
    return Workload(f"Kolmogorov turbulence, base {base}^3 + {n_refine} refined sub-grids "
                    f"({len(coord)} leaves), 11 fields", base, coord, U, cfl=0.4, steps=1,
                    meta={"n_refined": int(n_refine)})


def config5() -> Workload:
    return turbulence(32, 4681, 5)


def cold_band(coord: np.ndarray, base: int, nf: int = 6, seed_offset: int = 6,
              p_cold: float = 1e-6) -> Workload:
    """Supersonic flow with a cold band: rho = 1 + 0.2 sin(2 pi x) sin(2 pi y)
    + U(+-1e-3), v = (2 + 0.3 sin(2 pi y), 0.5 sin(2 pi z), 0.1), p = p_cold for
    0.25 <= z < 0.75 (Mach ~ 1500 there: internal energy ~ 1e-6 of the total)
    and 0.5 elsewhere; any leaf list.  In the band the internal energy is far
    below 1e-3 of the total energy, where the dual-energy switch takes the
    pressure from the entropy tracer."""
    rng = np.random.default_rng(SEED0 + seed_offset)
    X, Y, Z = cell_centres(coord, base)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    rho = rho + rng.uniform(-1e-3, 1e-3, size=rho.shape)
    vx = 2.0 + 0.3 * np.sin(2 * np.pi * Y)
    vy = 0.5 * np.sin(2 * np.pi * Z)
    vz = np.full_like(rho, 0.1)
    p = np.where((Z >= 0.25) & (Z < 0.75), p_cold, 0.5)
    species = _dirichlet_species(rng, rho.shape)[: nf - 6] if nf > 6 else None
    return Workload("supersonic flow with a cold band (dual-energy switch)", base, coord,
                    conserved(rho, vx, vy, vz, p, species))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def uniform_state(base: int, nf: int = 6, rho=1.0, v=(0.3, -0.2, 0.1), p=1.0) -> Workload:
    coord = uniform_leaves(base)
    shape = (len(coord), SUB, SUB, SUB)
    r = np.full(shape, rho)
    species = [np.full(shape, 0.2)] * (nf - 6) if nf > 6 else None
    U = conserved(r, np.full(shape, v[0]), np.full(shape, v[1]), np.full(shape, v[2]),
                  np.full(shape, p), species)
    return Workload("uniform state", base, coord, U)


def random_smooth(coord: np.ndarray, base: int, nf: int = 6, seed: int = 0,
                  amp: float = 0.05) -> Workload:
    """Smooth periodic state with random Fourier modes plus small noise; any
    leaf list."""
    rng = np.random.default_rng(SEED0 + 100 + seed)
    X, Y, Z = cell_centres(coord, base)

    def field(a0, a):
        out = np.full(X.shape, a0)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            out = out + a * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return out + rng.uniform(-1e-3, 1e-3, size=X.shape) * a

    rho = field(1.0, amp)
    p = field(1.0, amp)
    vx, vy, vz = field(0.1, amp), field(-0.05, amp), field(0.02, amp)
    species = _dirichlet_species(rng, rho.shape) if nf > 6 else None
    if species is not None:
        species = species[: nf - 6]
    return Workload("random smooth", base, coord, conserved(rho, vx, vy, vz, p, species))
