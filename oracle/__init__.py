"""FP64 CPU oracle for the octree hydro step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never calls it; the two share no code.

The arithmetic lives in ``octohydro_oracle.c`` (plain C, binary64, no FMA
contraction).  This module only builds that file with gcc and marshals numpy
arrays through ctypes.  Each function names the part of the paper it follows:

* octree of 8^3 sub-grids, properly nested: Sec. IV-C;
* ghost fill by direct reads of neighbour memory: Sec. VI;
* PPM reconstruction ("reconstruct" kernel) and central fluxes ("flux"
  kernel): Sec. V-B-1, method of Kurganov & Tadmor cited in Sec. IV-C;
* one Runge-Kutta substep with global time-step size: Sec. V-B-1
  (compute_fluxes); three hydro substeps per step: Sec. I.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "octohydro_oracle.c")
_LIB = os.path.join(_HERE, "liboctohydro_oracle.so")

SAME_LEAF, SAME_REFINED, COARSER_LEAF = 0, 1, 2
MAX_NF = 16


def build() -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    cmd = [
        "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
        "-shared", "-std=c11", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _OGrid(ctypes.Structure):
    _fields_ = [
        ("n_leaves", ctypes.c_int32),
        ("nf", ctypes.c_int32),
        ("base", ctypes.c_int32),
        ("coord", ctypes.c_void_p),
        ("nbr", ctypes.c_void_p),
        ("kind", ctypes.c_void_p),
        ("children", ctypes.c_void_p),
        ("gamma", ctypes.c_double),
        ("eta1", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("recon", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.oracle_build_table.argtypes = [i32, i32, vp, vp, vp, vp, i32, ctypes.POINTER(i32)]
    lib.oracle_build_table.restype = ctypes.c_int
    lib.oracle_fill_ghosts.argtypes = [ctypes.POINTER(_OGrid), vp, vp]
    lib.oracle_fill_ghosts.restype = None
    lib.oracle_ppm_1d.argtypes = [vp, ctypes.c_int, vp, vp]
    lib.oracle_ppm_1d.restype = None
    lib.oracle_face_flux.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, f64, f64, vp]
    lib.oracle_face_flux.restype = ctypes.c_int
    lib.oracle_step.argtypes = [ctypes.POINTER(_OGrid), vp, vp, vp, f64, f64]
    lib.oracle_step.restype = ctypes.c_int64
    lib.oracle_step_subset.argtypes = [ctypes.POINTER(_OGrid), vp, vp, vp, f64, f64, vp, i32]
    lib.oracle_step_subset.restype = ctypes.c_int64
    lib.oracle_cfl_dt.argtypes = [ctypes.POINTER(_OGrid), vp, f64]
    lib.oracle_cfl_dt.restype = f64
    lib.oracle_totals.argtypes = [ctypes.POINTER(_OGrid), vp, vp]
    lib.oracle_totals.restype = None
    lib.oracle_rk3_step.argtypes = [ctypes.POINTER(_OGrid), vp, vp, vp, f64, f64,
                                    ctypes.POINTER(f64)]
    lib.oracle_rk3_step.restype = ctypes.c_int64
    lib.oracle_step_1d.argtypes = [i32, ctypes.c_int, vp, vp, vp, f64, f64, f64, f64]
    lib.oracle_step_1d.restype = ctypes.c_int64
    lib.oracle_step_record.argtypes = [ctypes.POINTER(_OGrid), vp, vp, vp, f64, f64, vp, i32, vp]
    lib.oracle_step_record.restype = ctypes.c_int64
    lib.oracle_reflux.argtypes = [ctypes.POINTER(_OGrid), vp, f64, f64, vp, vp, i32]
    lib.oracle_reflux.restype = None
    lib.oracle_rk3_step_reflux.argtypes = [ctypes.POINTER(_OGrid), vp, vp, vp, f64, f64,
                                           ctypes.POINTER(f64), ctypes.c_int]
    lib.oracle_rk3_step_reflux.restype = ctypes.c_int64
    lib.oracle_point_value.argtypes = [vp, vp, vp]
    lib.oracle_point_value.restype = f64
    lib.oracle_face_flux_3d.argtypes = [ctypes.POINTER(_OGrid), vp, ctypes.c_int, vp, vp]
    lib.oracle_face_flux_3d.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (for timing it)."""
    _load().oracle_set_num_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


class Table:
    """Neighbour table of a leaf list: 27 slots per leaf (slot 13 = self),
    slot = (dz+1)*9 + (dy+1)*3 + (dx+1); kind SAME_LEAF / SAME_REFINED /
    COARSER_LEAF; refined nodes numbered in order of first reference."""

    def __init__(self, leaf_coord, base):
        lib = _load()
        self.coord = np.ascontiguousarray(leaf_coord, dtype=np.int32)
        n = self.coord.shape[0]
        self.base = int(base)
        self.nbr = np.zeros((n, 27), np.int32)
        self.kind = np.zeros((n, 27), np.uint8)
        cap = 27 * n + 8
        kids = np.full((cap, 8), -1, np.int32)
        nn = ctypes.c_int32(0)
        st = lib.oracle_build_table(n, self.base, _ptr(self.coord), _ptr(self.nbr),
                                    _ptr(self.kind), _ptr(kids), cap, ctypes.byref(nn))
        if st != 0:
            raise ValueError(f"oracle_build_table failed with status {st}")
        self.children = np.ascontiguousarray(kids[: max(nn.value, 1)])
        self.n_nodes = nn.value

    @property
    def n_leaves(self):
        return self.coord.shape[0]


# Frame angular velocity used by every call (0: inertial frame).  Set with
# set_omega(); rotating-frame sources (Sec. IV-C) are on when it is non-zero.
_OMEGA = [0.0]


def set_omega(omega: float) -> None:
    _OMEGA[0] = float(omega)


# Reconstruction used by every call: 0 = PPM per axis with the flux at the
# face centre, 1 = full 3D reconstruction with the 9-point Simpson flux per
# face (Sec. V-B-1).  Set with set_recon().
_RECON = [0]
RECON_AXIS, RECON_3D = 0, 1


def set_recon(mode: int) -> None:
    if mode not in (RECON_AXIS, RECON_3D):
        raise ValueError(f"unknown reconstruction {mode}")
    _RECON[0] = int(mode)


def _grid(table: Table, nf: int, gamma: float, eta1: float) -> _OGrid:
    g = _OGrid()
    g.omega = _OMEGA[0]
    g.recon = _RECON[0]
    g.n_leaves = table.n_leaves
    g.nf = nf
    g.base = table.base
    g.coord = _ptr(table.coord)
    g.nbr = _ptr(table.nbr)
    g.kind = _ptr(table.kind)
    g.children = _ptr(table.children)
    g.gamma = gamma
    g.eta1 = eta1
    return g


GAMMA = 5.0 / 3.0
ETA1 = 1e-3


def fill_ghosts(table: Table, U, gamma=GAMMA, eta1=ETA1):
    """Ghosted tiles G[nf][n][14][14][14] from U[nf][n][8][8][8] (Sec. VI)."""
    U = _c64(U)
    nf = U.shape[0]
    G = np.empty((nf, table.n_leaves, 14, 14, 14), np.float64)
    _load().oracle_fill_ghosts(ctypes.byref(_grid(table, nf, gamma, eta1)), _ptr(U), _ptr(G))
    return G


def ppm_1d(q):
    """PPM face values (qL, qR) of each cell j in [2, n-2); NaN elsewhere."""
    q = _c64(q)
    n = q.shape[0]
    qL = np.full(n, np.nan)
    qR = np.full(n, np.nan)
    _load().oracle_ppm_1d(_ptr(q), n, _ptr(qL), _ptr(qR))
    return qL, qR


def point_value(tile, t, p):
    """3D reconstruction: value of a 14^3 tile (one field) at the point
    t + p/2 of tile cell t, p in {-1,0,1}^3 without 0."""
    tile = _c64(tile)
    lib = _load()
    tt = np.ascontiguousarray(t, np.int32)
    pp = np.ascontiguousarray(p, np.int32)
    return lib.oracle_point_value(_ptr(tile), _ptr(tt), _ptr(pp))


def face_flux_3d(tiles, d, tl, gamma=GAMMA, eta1=ETA1):
    """9-point Simpson flux (3D reconstruction) of the face normal to d
    between tile cells tl and tl + d of tiles[nf][14][14][14]; (H, n_bad)."""
    tiles = _c64(tiles)
    nf = tiles.shape[0]
    H = np.empty(nf, np.float64)
    tt = np.ascontiguousarray(tl, np.int32)
    tab = Table(np.zeros((1, 4), np.int32), 1)
    bad = _load().oracle_face_flux_3d(ctypes.byref(_grid(tab, nf, gamma, eta1)), _ptr(tiles),
                                      int(d), _ptr(tt), _ptr(H))
    return H, bad


def face_flux(d, UL, UR, gamma=GAMMA, eta1=ETA1):
    """Kurganov-Tadmor flux across a face normal to axis d; returns (H, n_bad)."""
    UL = _c64(UL)
    UR = _c64(UR)
    H = np.empty_like(UL)
    bad = _load().oracle_face_flux(int(d), UL.shape[0], _ptr(UL), _ptr(UR), gamma, eta1, _ptr(H))
    return H, bad


def step(table: Table, Uk, dt, beta=1.0, U0=None, gamma=GAMMA, eta1=ETA1):
    """One RK substep with t = Uk + dt*L(Uk): Uout = t without U0, else
    Uout = U0 + beta*(t - U0); returns (Uout, n_bad)."""
    Uk = _c64(Uk)
    U0 = None if U0 is None else _c64(U0)
    nf = Uk.shape[0]
    out = np.empty_like(Uk)
    bad = _load().oracle_step(ctypes.byref(_grid(table, nf, gamma, eta1)), _ptr(U0), _ptr(Uk),
                              _ptr(out), float(dt), float(beta))
    return out, bad


def step_subset(table: Table, Uk, dt, leaves, beta=1.0, U0=None, out=None, gamma=GAMMA,
                eta1=ETA1):
    """The substep of :func:`step` computed only for `leaves`; other leaves of
    `out` keep their values (NaN when `out` is not given)."""
    Uk = _c64(Uk)
    U0 = None if U0 is None else _c64(U0)
    leaves = np.ascontiguousarray(leaves, dtype=np.int32)
    if out is None:
        out = np.full_like(Uk, np.nan)
    bad = _load().oracle_step_subset(ctypes.byref(_grid(table, Uk.shape[0], gamma, eta1)),
                                     _ptr(U0), _ptr(Uk), _ptr(out), float(dt), float(beta),
                                     _ptr(leaves), len(leaves))
    return out, bad


def neighbours(table: Table, leaves):
    """Leaves whose cells the ghost fill of `leaves` reads, plus `leaves`."""
    out = set(int(x) for x in leaves)
    for n in leaves:
        for s in range(27):
            k, m = int(table.kind[n, s]), int(table.nbr[n, s])
            if k == SAME_REFINED:
                out.update(int(c) for c in table.children[m] if c >= 0)
            else:
                out.add(m)
    return np.array(sorted(out), dtype=np.int32)


def cfl_dt(table: Table, U, cfl, gamma=GAMMA, eta1=ETA1):
    U = _c64(U)
    return _load().oracle_cfl_dt(ctypes.byref(_grid(table, U.shape[0], gamma, eta1)), _ptr(U),
                                 float(cfl))


def totals(table: Table, U):
    U = _c64(U)
    out = np.empty(U.shape[0], np.float64)
    _load().oracle_totals(ctypes.byref(_grid(table, U.shape[0], GAMMA, ETA1)), _ptr(U), _ptr(out))
    return out


def rk3_step(table: Table, U, cfl=0.4, dt=0.0, gamma=GAMMA, eta1=ETA1, reflux=False):
    """One SSP-RK3 step (three substeps, Sec. I), optionally with the
    coarse-fine flux correction after each substep. Returns (U_next, dt, n_bad)."""
    U = _c64(U).copy()
    W1 = np.empty_like(U)
    W2 = np.empty_like(U)
    dto = ctypes.c_double(0.0)
    bad = _load().oracle_rk3_step_reflux(ctypes.byref(_grid(table, U.shape[0], gamma, eta1)),
                                         _ptr(U), _ptr(W1), _ptr(W2), float(cfl), float(dt),
                                         ctypes.byref(dto), int(bool(reflux)))
    return U, dto.value, bad


def step_record(table: Table, Uk, dt, beta=1.0, U0=None, leaves=None, out=None, face_flux=None,
                gamma=GAMMA, eta1=ETA1):
    """Substep that also records the fluxes through the six faces of every
    processed leaf into face_flux[n][3][2][64][nf] (allocated if None)."""
    Uk = _c64(Uk)
    U0 = None if U0 is None else _c64(U0)
    nf = Uk.shape[0]
    if out is None:
        out = np.full_like(Uk, np.nan)
    if face_flux is None:
        face_flux = np.full((table.n_leaves, 3, 2, 64, nf), np.nan)
    sub = None if leaves is None else np.ascontiguousarray(leaves, dtype=np.int32)
    bad = _load().oracle_step_record(ctypes.byref(_grid(table, nf, gamma, eta1)), _ptr(U0),
                                     _ptr(Uk), _ptr(out), float(dt), float(beta), _ptr(sub),
                                     0 if sub is None else len(sub), _ptr(face_flux))
    return out, face_flux, bad


def reflux(table: Table, Uout, dt, w, face_flux, leaves=None):
    """Coarse-fine flux correction of a substep's result (in place)."""
    sub = None if leaves is None else np.ascontiguousarray(leaves, dtype=np.int32)
    _load().oracle_reflux(ctypes.byref(_grid(table, Uout.shape[0], GAMMA, ETA1)), _ptr(Uout),
                          float(dt), float(w), _ptr(face_flux), _ptr(sub),
                          0 if sub is None else len(sub))
    return Uout


def step_1d(Uk, dt, beta=1.0, U0=None, gamma=GAMMA, eta1=ETA1):
    """1D periodic substep with the same reconstruction and flux; Uk[nf][n]."""
    Uk = _c64(Uk)
    U0 = None if U0 is None else _c64(U0)
    nf, n = Uk.shape
    if n % 8:
        raise ValueError("1D length must be a multiple of 8")
    out = np.empty_like(Uk)
    bad = _load().oracle_step_1d(n, nf, _ptr(U0), _ptr(Uk), _ptr(out), float(dt), float(beta),
                                 gamma, eta1)
    return out, bad


def rk3_step_1d(U, dt, gamma=GAMMA, eta1=ETA1):
    U = _c64(U)
    W1, _ = step_1d(U, dt, 1.0, None, gamma, eta1)
    W2, _ = step_1d(W1, dt, 0.25, U, gamma, eta1)
    out, _ = step_1d(W2, dt, 2.0 / 3.0, U, gamma, eta1)
    return out


def cfl_dt_1d(U, cfl, gamma=GAMMA):
    """CFL time step of a 1D state U[nf][n] (cell width 1/n), same EOS reading."""
    U = _c64(U)
    n = U.shape[1]
    # Reuse the 3D routine on a single-row view would change layout; the 1D
    # reading is small enough to evaluate through a degenerate one-leaf grid.
    rho, sx, sy, sz, E = U[0], U[1], U[2], U[3], U[4]
    rinv = 1.0 / rho
    ss = (sx * sx + sy * sy) + sz * sz
    ei = E - 0.5 * ss * rinv
    p = (gamma - 1.0) * ei
    c = np.sqrt(gamma * p * rinv)
    vmax = np.maximum(np.maximum(np.abs(sx * rinv), np.abs(sy * rinv)), np.abs(sz * rinv))
    return cfl * np.min((1.0 / n) / (vmax + c))
