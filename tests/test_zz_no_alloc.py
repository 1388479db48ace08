"""The allocation-free totals (hydro_totals_noalloc) through the C-ABI:
the same bits as hydro_totals, on two calls in a row whose second input is
smaller than the first (the fixed scratch keeps the first call's partial
sums, which the second must not read)."""
import numpy as np
import pytest

import oracle
from paper_2210_06437_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_totals_equal_the_allocating_entry_point():
    import torch

    from paper_2210_06437_amd import binding as hb
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cases = [("amr-base4-levels0-3-nf11", inputs.blobs(base=4, max_level=3), hb.HYDRO_F64),
             ("sod-base2-nf6", inputs.sod(base=2), hb.HYDRO_F64),
             ("sod-base2-nf6-f32", inputs.sod(base=2), hb.HYDRO_F32)]
    for name, w, dtype in cases:
        print(f"case {name}: {w.n_leaves} leaves nf={w.nf} dtype={dtype}", flush=True)
        grid = hb.Grid(w.leaf_coord, w.base, w.nf, dtype)
        tdt = torch.float64 if dtype == hb.HYDRO_F64 else torch.float32
        U = torch.from_numpy(w.U).to("cuda").to(tdt).contiguous()
        a = torch.full((w.nf,), float("nan"), dtype=torch.float64, device="cuda")
        b = torch.full((w.nf,), float("nan"), dtype=torch.float64, device="cuda")
        hb.hydro_totals_noalloc(grid, U, a)
        hb.hydro_totals(grid, U, b)
        torch.cuda.synchronize()
        got, want = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(got, want), (name, got, want)
        T = oracle.Table(w.leaf_coord, w.base)
        Uo = U.double().cpu().numpy()
        ref = oracle.totals(T, Uo)
        scale = oracle.totals(T, np.abs(Uo))
        assert np.all(np.abs(got - ref) <= 1e-14 * scale), (name, got, ref)
