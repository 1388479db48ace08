"""The binary32-storage path (FP32-mixed) against the binary64 oracle.

FP32-mixed stores the state in binary32 and evaluates PPM, the EOS and the
Kurganov-Tadmor flux in binary32; the flux differences, the divergence, the
stage combination, the totals and the time step are binary64.  Its error is
a property to state, not a parity to meet: per field the relative L1 error
    L1_f = sum |u32 - u64| / sum |u64|
after a run, and the drift of the totals of mass and energy.  The bounds
asserted here are the values measured on MI355X times a margin of about 5
(the measured numbers are printed)."""
import numpy as np
import pytest

import oracle
from paper_2210_06437_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS = ["rho", "s_x", "s_y", "s_z", "E", "tau"]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2210_06437_amd import binding as hb
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, hb


def _l1(a, b):
    nf = b.shape[0]
    return np.abs(a - b).reshape(nf, -1).sum(1) / np.abs(b).reshape(nf, -1).sum(1)


def test_sod_4096_leaves_100_rk3_steps_fp32_mixed(env):
    """The Sod tube on 16^3 sub-grids (128^3 cells) in binary32 storage,
    100 RK3 steps at CFL 0.4.  Both sides advance with the oracle's time step
    of each step (computed by the oracle from its binary64 state), so the
    error is that of the arithmetic, not of a shifted time; the device's own
    time step from its binary32 state is compared with it on the way."""
    torch, hb = env
    w = inputs.config4()
    print(f"case config4: {w.n_leaves} leaves, {w.steps} RK3 steps", flush=True)
    grid = hb.Grid(w.leaf_coord, w.base, w.nf, hb.HYDRO_F32)
    T = oracle.Table(w.leaf_coord, w.base)
    U = torch.from_numpy(w.U).to("cuda").float().contiguous()
    W1, W2, Un = grid.empty_state(), grid.empty_state(), grid.empty_state()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = torch.zeros(w.nf, dtype=torch.float64, device="cuda")
    hb.hydro_totals(grid, U, t0)
    tot0_64 = oracle.totals(T, w.U)
    Uo = w.U
    worst_dt = 0.0
    for step in range(w.steps):
        hb.hydro_cfl_dt(grid, U, 0.4, dtg)
        Uo_next, dto, bad = oracle.rk3_step(T, Uo, 0.4)
        assert bad == 0
        worst_dt = max(worst_dt, abs(dtg.item() - dto) / dto)
        dt.fill_(dto)
        hb.hydro_rk3_step(grid, U, W1, W2, Un, 0.0, dt)
        U, Un = Un, U
        Uo = Uo_next
        if step % 20 == 19:
            print(f"  step {step + 1}", flush=True)
    assert hb.hydro_check_status(grid) == hb.HYDRO_OK
    got = U.double().cpu().numpy()
    l1 = _l1(got, Uo)
    tg = torch.zeros(w.nf, dtype=torch.float64, device="cuda")
    hb.hydro_totals(grid, U, tg)
    t0 = t0.cpu().numpy()
    tg = tg.cpu().numpy()
    tot_o = oracle.totals(T, Uo)
    drift = np.abs(tg - t0) / np.abs(t0)
    drift64 = np.abs(tot_o - tot0_64) / np.abs(tot0_64)
    print("FP32-mixed per-field L1 vs the FP64 oracle after 100 RK3 steps: " +
          ", ".join(f"{n} {x:.3e}" for n, x in zip(FIELDS, l1)))
    print(f"FP32-mixed total drift over 100 steps: mass {drift[0]:.3e}, energy {drift[4]:.3e} "
          f"(FP64 oracle: mass {drift64[0]:.3e}, energy {drift64[4]:.3e}); "
          f"largest relative difference of the device's own time step {worst_dt:.3e}")
    # measured on MI355X: rho 2.7e-7, s_x 6.3e-7, s_y 2.3e-2, s_z 2.3e-2,
    # E 3.5e-7, tau 2.7e-7; drift mass 9.9e-9, energy 1.3e-9; dt 1.4e-7.
    # s_y and s_z are the 1e-4 transverse noise: binary32 rounding of the
    # O(1) pressure in their fluxes is an absolute error of ~1e-7 per face,
    # a few per cent of fields that small after 300 substeps.
    assert np.all(np.isfinite(l1))
    assert np.all(l1[[0, 1, 4, 5]] < 3e-6), l1
    assert np.all(l1[[2, 3]] < 0.12), l1
    assert drift[0] < 5e-8 and drift[4] < 5e-8, drift
    assert worst_dt < 1e-6


@pytest.mark.parametrize("what", ["reflux", "rotation"])
def test_fp32_mixed_with_flux_correction_and_rotation(env, what):
    """binary32 storage on an uneven tree with the coarse-fine flux
    correction, and with the rotating frame's sources: two RK3 steps against
    the binary64 oracle with the same options."""
    torch, hb = env
    w = inputs.blobs(base=4, max_level=3)
    kw = {"reflux": True} if what == "reflux" else {"omega": 0.9}
    print(f"case amr-base4-levels0-3 fp32 {what}: {w.n_leaves} leaves", flush=True)
    grid = hb.Grid(w.leaf_coord, w.base, w.nf, hb.HYDRO_F32, **kw)
    T = oracle.Table(w.leaf_coord, w.base)
    U = torch.from_numpy(w.U).to("cuda").float().contiguous()
    W1, W2, Un = grid.empty_state(), grid.empty_state(), grid.empty_state()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    Uo = w.U
    if what == "rotation":
        oracle.set_omega(0.9)
    try:
        for _ in range(2):
            Uo, dto, bad = oracle.rk3_step(T, Uo, 0.4, reflux=(what == "reflux"))
            assert bad == 0
            dt.fill_(dto)
            hb.hydro_rk3_step(grid, U, W1, W2, Un, 0.0, dt)
            U, Un = Un, U
    finally:
        oracle.set_omega(0.0)
    assert hb.hydro_check_status(grid) == hb.HYDRO_OK
    l1 = _l1(U.double().cpu().numpy(), Uo)
    print(f"  FP32-mixed ({what}) per-field L1 after 2 RK3 steps:",
          " ".join(f"{x:.2e}" for x in l1))
    # measured on MI355X: at most 7.6e-7 (s_x, s_z), 3e-8 to 2e-7 elsewhere
    assert np.all(l1 < 4e-6), l1
