"""MI355X-native octree hydro step (PPM + Kurganov-Tadmor, SSP-RK3) on gfx950.

The compute path is the HIP library ``liboctohydro.so`` behind the C-ABI in
``include/octohydro.h``; :mod:`paper_2210_06437_amd.binding` is the thin
ctypes binding with the same entry-point names.  Inputs are built by
:mod:`paper_2210_06437_amd.inputs`.
"""
__all__ = ["binding", "inputs"]
