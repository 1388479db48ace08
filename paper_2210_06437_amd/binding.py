"""Thin ctypes binding of liboctohydro.so (C-ABI in include/octohydro.h).

Argument marshalling only: every step of the hydro path runs in the HIP
library.  PyTorch provides device memory and streams.  If the library has not
been built, importing this module fails loudly -- there is no fallback.

Entry points keep the C names: hydro_build_table, hydro_fill_ghosts,
hydro_step, hydro_step_per_leaf, hydro_cfl_dt, hydro_totals, hydro_totals_noalloc,
hydro_rk3_step,
hydro_rk3_graph_create / hydro_graph_launch / hydro_graph_destroy,
hydro_check_status, hydro_last_error, hydro_version.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# OCTOHYDRO_LIB may name another build of the same library (e.g. a tuning
# variant); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("OCTOHYDRO_LIB") or os.path.join(_PKG, "liboctohydro.so")

HYDRO_OK, HYDRO_E_ARG, HYDRO_E_TABLE, HYDRO_E_UNPHYSICAL, HYDRO_E_HIP, HYDRO_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5)
HYDRO_F64, HYDRO_F32 = 0, 1
HYDRO_SAME_LEAF, HYDRO_SAME_REFINED, HYDRO_COARSER_LEAF = 0, 1, 2
HYDRO_FLAG_VALIDATE = 1
HYDRO_FLAG_NODES_READY = 2
HYDRO_FLAG_CFL_NEXT = 4
HYDRO_RECON_AXIS, HYDRO_RECON_3D = 0, 1
HYDRO_MAX_LEAVES = 1048575
HYDRO_STATUS_UNPHYSICAL, HYDRO_STATUS_TABLE = 1, 2

EXPORTS = [
    "hydro_build_table", "hydro_fill_ghosts", "hydro_step", "hydro_step_per_leaf",
    "hydro_cfl_dt", "hydro_totals", "hydro_rk3_step", "hydro_rk3_graph_create",
    "hydro_graph_launch", "hydro_graph_destroy", "hydro_check_status", "hydro_last_error",
    "hydro_version", "hydro_set_option", "hydro_get_option", "hydro_build_reflux",
    "hydro_totals_noalloc", "hydro_build_leaf_node",
]
HYDRO_OPT_WAVES_PER_SIMD, HYDRO_OPT_XCD_REMAP, HYDRO_OPT_WAVES_PER_LEAF = 1, 2, 3
HYDRO_OPT_CFL_EPILOGUE = 4
HYDRO_OPT_FUSED_RESTRICT = 5
HYDRO_OPT_3D_WORKGROUP = 6


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class hydro_grid(ctypes.Structure):
    _fields_ = [
        ("n_leaves", ctypes.c_int32),
        ("n_nodes", ctypes.c_int32),
        ("n_fields", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("base", ctypes.c_int32),
        ("reconstruction", ctypes.c_int32),
        ("leaf_coord_dev", ctypes.c_void_p),
        ("nbr_dev", ctypes.c_void_p),
        ("nbr_kind_dev", ctypes.c_void_p),
        ("children_dev", ctypes.c_void_p),
        ("status_dev", ctypes.c_void_p),
        ("gamma", ctypes.c_double),
        ("dual_energy_eta1", ctypes.c_double),
        ("n_slots", ctypes.c_int32),
        ("orient_begin", ctypes.c_int32 * 7),
        ("face_slot_dev", ctypes.c_void_p),
        ("fine_slot_dev", ctypes.c_void_p),
        ("slot_leaf_dev", ctypes.c_void_p),
        ("flux_reg_dev", ctypes.c_void_p),
        ("omega", ctypes.c_double),
        ("node_state_dev", ctypes.c_void_p),
        ("ghost_tile_dev", ctypes.c_void_p),
        ("cfl_epilogue", ctypes.c_int32),
        ("node_state2_dev", ctypes.c_void_p),
        ("leaf_node_dev", ctypes.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    G = ctypes.POINTER(hydro_grid)
    sig = {
        "hydro_build_table": ([i32, i32, vp, vp, vp, vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "hydro_fill_ghosts": ([G, vp, vp, vp], ctypes.c_int),
        "hydro_step": ([G, vp, vp, vp, vp, f64, u32, vp], ctypes.c_int),
        "hydro_step_per_leaf": ([G, vp, vp, vp, vp, f64, i32, vp], ctypes.c_int),
        "hydro_cfl_dt": ([G, vp, f64, vp, vp], ctypes.c_int),
        "hydro_totals": ([G, vp, vp, vp], ctypes.c_int),
        "hydro_totals_noalloc": ([G, vp, vp, vp], ctypes.c_int),
        "hydro_rk3_step": ([G, vp, vp, vp, vp, f64, vp, vp], ctypes.c_int),
        "hydro_rk3_graph_create": ([G, vp, vp, vp, vp, f64, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "hydro_graph_launch": ([vp, vp], ctypes.c_int),
        "hydro_graph_destroy": ([vp], ctypes.c_int),
        "hydro_check_status": ([G, vp], ctypes.c_int),
        "hydro_last_error": ([], ctypes.c_char_p),
        "hydro_version": ([], ctypes.c_int),
        "hydro_set_option": ([i32, i32, i32, i32], ctypes.c_int),
        "hydro_build_reflux": ([i32, vp, vp, vp, vp, vp, vp, i32, vp, ctypes.POINTER(i32)],
                               ctypes.c_int),
        "hydro_get_option": ([i32, i32, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "hydro_build_leaf_node": ([i32, i32, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()

# Launch options chosen by the autotuner (autotune.py), applied at import.
TUNING_PATH = os.path.join(_PKG, "tuning.json")


def apply_tuning(path: str = TUNING_PATH) -> int:
    """Apply recorded autotuner choices; returns how many entries were set."""
    import json
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for e in data.get("entries", []):
        _lib.hydro_set_option(int(e["dtype"]), int(e["n_fields"]), 1, int(e["waves_per_simd"]))
        _lib.hydro_set_option(int(e["dtype"]), int(e["n_fields"]), 2, int(e["xcd_remap"]))
        _lib.hydro_set_option(int(e["dtype"]), int(e["n_fields"]), 3,
                              int(e.get("waves_per_leaf", 1)))
        _lib.hydro_set_option(int(e["dtype"]), int(e["n_fields"]), 4,
                              int(e.get("cfl_epilogue", 1)))
        _lib.hydro_set_option(int(e["dtype"]), int(e["n_fields"]), 5,
                              int(e.get("fused_restrict", 1)))
        n += 1
    return n


apply_tuning()


def _check(rc: int):
    if rc != HYDRO_OK:
        raise HydroError(rc, _lib.hydro_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def hydro_version() -> int:
    return _lib.hydro_version()


def hydro_last_error() -> str:
    return _lib.hydro_last_error().decode()


def hydro_set_option(dtype: int, n_fields: int, option: int, value: int):
    _check(_lib.hydro_set_option(int(dtype), int(n_fields), int(option), int(value)))


def hydro_get_option(dtype: int, n_fields: int, option: int) -> int:
    v = ctypes.c_int32(0)
    _check(_lib.hydro_get_option(int(dtype), int(n_fields), int(option), ctypes.byref(v)))
    return v.value


def hydro_build_table(leaf_coord: np.ndarray, base: int):
    """Host neighbour table: returns (nbr [n][27] int32, kind [n][27] uint8,
    children [n_nodes][8] int32)."""
    coord = np.ascontiguousarray(leaf_coord, dtype=np.int32)
    n = coord.shape[0]
    nbr = np.zeros((n, 27), np.int32)
    kind = np.zeros((n, 27), np.uint8)
    cap = 27 * n + 8
    kids = np.full((cap, 8), -1, np.int32)
    nn = ctypes.c_int32(0)
    _check(_lib.hydro_build_table(n, int(base), coord.ctypes.data, nbr.ctypes.data,
                                  kind.ctypes.data, kids.ctypes.data, cap, ctypes.byref(nn)))
    return nbr, kind, np.ascontiguousarray(kids[: nn.value])


def hydro_build_leaf_node(n_leaves: int, children: np.ndarray):
    """node * 8 + octant of every child leaf of the children table, else -1."""
    kids = np.ascontiguousarray(children, dtype=np.int32).reshape(-1, 8)
    out = np.zeros(int(n_leaves), np.int32)
    _check(_lib.hydro_build_leaf_node(int(n_leaves), len(kids), kids.ctypes.data,
                                      out.ctypes.data))
    return out


def hydro_build_reflux(leaf_coord: np.ndarray, nbr: np.ndarray, kind: np.ndarray):
    """Host flux-register tables: (face_slot [n][6], fine_slot [n][6],
    slot_leaf [n_slots], orient_begin [7])."""
    coord = np.ascontiguousarray(leaf_coord, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    n = coord.shape[0]
    face_slot = np.zeros((n, 6), np.int32)
    fine_slot = np.zeros((n, 6), np.int32)
    slot_leaf = np.zeros(6 * n, np.int32)
    orient = np.zeros(7, np.int32)
    ns = ctypes.c_int32(0)
    _check(_lib.hydro_build_reflux(n, coord.ctypes.data, nbr.ctypes.data, kind.ctypes.data,
                                   face_slot.ctypes.data, fine_slot.ctypes.data,
                                   slot_leaf.ctypes.data, 6 * n, orient.ctypes.data,
                                   ctypes.byref(ns)))
    return face_slot, fine_slot, np.ascontiguousarray(slot_leaf[: ns.value]), orient


class Grid:
    """A leaf batch resident on the GPU: the table in device memory plus the
    hydro_grid struct that points at it.  reflux=True also builds the
    flux-register tables and scratch, which turns on the coarse-fine flux
    correction.  cfl_epilogue=True chains the RK3 steps' time steps (dt of
    2 doubles; see hydro_grid.cfl_epilogue).  fused_restrict=False keeps a
    restriction pass before every RK3 substep (see hydro_grid.node_state2_dev)."""

    def __init__(self, leaf_coord, base, n_fields, dtype=HYDRO_F64, gamma=5.0 / 3.0,
                 eta1=1e-3, device="cuda", reflux=False, omega=0.0,
                 reconstruction=HYDRO_RECON_AXIS, cfl_epilogue=False, fused_restrict=True):
        coord = np.ascontiguousarray(leaf_coord, dtype=np.int32)
        nbr, kind, kids = hydro_build_table(coord, base)
        self.host_nbr, self.host_kind, self.host_children = nbr, kind, kids
        dev = torch.device(device)
        self.coord = torch.from_numpy(coord).to(dev)
        self.nbr = torch.from_numpy(nbr).to(dev)
        self.kind = torch.from_numpy(kind).to(dev)
        self.children = torch.from_numpy(kids if len(kids) else np.full((1, 8), -1, np.int32)).to(dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.n_leaves = coord.shape[0]
        self.n_fields = int(n_fields)
        self.dtype = int(dtype)
        self.base = int(base)
        self.torch_dtype = torch.float64 if dtype == HYDRO_F64 else torch.float32
        self.c = hydro_grid(
            n_leaves=self.n_leaves, n_nodes=len(kids), n_fields=self.n_fields, dtype=self.dtype,
            base=self.base, reconstruction=int(reconstruction),
            leaf_coord_dev=self.coord.data_ptr(),
            nbr_dev=self.nbr.data_ptr(), nbr_kind_dev=self.kind.data_ptr(),
            children_dev=self.children.data_ptr(), status_dev=self.status.data_ptr(),
            gamma=float(gamma), dual_energy_eta1=float(eta1), omega=float(omega),
            cfl_epilogue=int(bool(cfl_epilogue)))
        # scratch of the reconstruction: materialised ghosted tiles (3D), or
        # the restricted copies of the refined blocks
        if reconstruction == HYDRO_RECON_3D:
            self.ghost_tiles = torch.empty((self.n_fields, self.n_leaves, 14, 14, 14),
                                           dtype=self.torch_dtype, device=dev)
            self.c.ghost_tile_dev = self.ghost_tiles.data_ptr()
        elif len(kids):
            self.node_state = torch.empty((self.n_fields, len(kids), 8, 8, 8),
                                          dtype=self.torch_dtype, device=dev)
            self.c.node_state_dev = self.node_state.data_ptr()
            if fused_restrict:
                # a second node buffer: RK3 substeps leave the node copies of
                # their outputs for the next substep
                self.node_state2 = torch.empty_like(self.node_state)
                self.leaf_node = torch.from_numpy(
                    hydro_build_leaf_node(self.n_leaves, kids)).to(dev)
                self.c.node_state2_dev = self.node_state2.data_ptr()
                self.c.leaf_node_dev = self.leaf_node.data_ptr()
        self.reflux = bool(reflux)
        if self.reflux:
            fs, fi, sl, ob = hydro_build_reflux(coord, nbr, kind)
            self.n_slots = len(sl)
            if self.n_slots:
                self.face_slot = torch.from_numpy(fs).to(dev)
                self.fine_slot = torch.from_numpy(fi).to(dev)
                self.slot_leaf = torch.from_numpy(sl).to(dev)
                self.flux_reg = torch.empty((self.n_slots, self.n_fields, 320),
                                            dtype=torch.float64, device=dev)
                self.c.n_slots = self.n_slots
                for i in range(7):
                    self.c.orient_begin[i] = int(ob[i])
                self.c.face_slot_dev = self.face_slot.data_ptr()
                self.c.fine_slot_dev = self.fine_slot.data_ptr()
                self.c.slot_leaf_dev = self.slot_leaf.data_ptr()
                self.c.flux_reg_dev = self.flux_reg.data_ptr()

    @property
    def state_shape(self):
        return (self.n_fields, self.n_leaves, 8, 8, 8)

    def empty_state(self):
        return torch.empty(self.state_shape, dtype=self.torch_dtype, device=self.coord.device)

    def check_state(self, t, name):
        if t is None:
            return
        if tuple(t.shape) != self.state_shape or t.dtype != self.torch_dtype or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {self.torch_dtype} CUDA tensor of "
                             f"shape {self.state_shape}, got {t.dtype} {tuple(t.shape)}")


def hydro_fill_ghosts(grid: Grid, U, G, stream=None):
    grid.check_state(U, "U")
    want = (grid.n_fields, grid.n_leaves, 14, 14, 14)
    if tuple(G.shape) != want or G.dtype != grid.torch_dtype or not G.is_contiguous():
        raise ValueError(f"G: expected {grid.torch_dtype} tensor of shape {want}")
    _check(_lib.hydro_fill_ghosts(ctypes.byref(grid.c), _ptr(U), _ptr(G), _stream(stream)))


def hydro_step(grid: Grid, U0, Uk, Uout, dt, beta=1.0, flags=0, stream=None):
    for t, n in ((U0, "U0"), (Uk, "Uk"), (Uout, "Uout")):
        grid.check_state(t, n)
    _check(_lib.hydro_step(ctypes.byref(grid.c), _ptr(U0), _ptr(Uk), _ptr(Uout), _ptr(dt),
                           float(beta), int(flags), _stream(stream)))


def hydro_step_per_leaf(grid: Grid, U0, Uk, Uout, dt, beta=1.0, n_streams=128, stream=None):
    for t, n in ((U0, "U0"), (Uk, "Uk"), (Uout, "Uout")):
        grid.check_state(t, n)
    _check(_lib.hydro_step_per_leaf(ctypes.byref(grid.c), _ptr(U0), _ptr(Uk), _ptr(Uout),
                                    _ptr(dt), float(beta), int(n_streams), _stream(stream)))


def hydro_cfl_dt(grid: Grid, U, cfl, dt, stream=None):
    grid.check_state(U, "U")
    _check(_lib.hydro_cfl_dt(ctypes.byref(grid.c), _ptr(U), float(cfl), _ptr(dt),
                             _stream(stream)))


def hydro_totals(grid: Grid, U, out, stream=None):
    grid.check_state(U, "U")
    _check(_lib.hydro_totals(ctypes.byref(grid.c), _ptr(U), _ptr(out), _stream(stream)))


def hydro_totals_noalloc(grid: Grid, U, out, stream=None):
    """hydro_totals without any device allocation (fixed library scratch)."""
    grid.check_state(U, "U")
    _check(_lib.hydro_totals_noalloc(ctypes.byref(grid.c), _ptr(U), _ptr(out), _stream(stream)))


def hydro_rk3_step(grid: Grid, Un, W1, W2, Unext, cfl, dt, stream=None):
    for t, n in ((Un, "Un"), (W1, "W1"), (W2, "W2"), (Unext, "Unext")):
        grid.check_state(t, n)
    _check(_lib.hydro_rk3_step(ctypes.byref(grid.c), _ptr(Un), _ptr(W1), _ptr(W2), _ptr(Unext),
                               float(cfl), _ptr(dt), _stream(stream)))


class Rk3Graph:
    """hydro_rk3_graph_create / hydro_graph_launch / hydro_graph_destroy."""

    def __init__(self, grid: Grid, Un, W1, W2, Unext, cfl, dt):
        for t, n in ((Un, "Un"), (W1, "W1"), (W2, "W2"), (Unext, "Unext")):
            grid.check_state(t, n)
        self._keep = (grid, Un, W1, W2, Unext, dt)
        h = ctypes.c_void_p(0)
        _check(_lib.hydro_rk3_graph_create(ctypes.byref(grid.c), _ptr(Un), _ptr(W1), _ptr(W2),
                                           _ptr(Unext), float(cfl), _ptr(dt), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(_lib.hydro_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            _check(_lib.hydro_graph_destroy(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hydro_check_status(grid: Grid, stream=None) -> int:
    """Synchronous; returns the status code (does not raise)."""
    return _lib.hydro_check_status(ctypes.byref(grid.c), _stream(stream))
