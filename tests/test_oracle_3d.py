"""Pins of the oracle's full three-dimensional reconstruction with the
9-point Simpson face flux (Sec. V-B-1: a full 3D reconstruction, face fluxes
integrated by quadrature).

The reconstruction gives each cell values at its 26 face, edge and corner
points from the axis PPM applied along the 13 lines of cells through it; the
face flux combines the Kurganov-Tadmor flux at the face's 9 points with the
tensor Simpson weights 1, 4, 16 over 36.  Pinned here: linear data is
reproduced exactly at every point (line directions and which end of the
parabola feeds which point), a linear transverse profile integrates to its
face-centre value (the weights), and the whole step keeps a uniform state,
conserves, is mirror symmetric and reduces to the 1D solver for
plane-symmetric data.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2210_06437_amd import inputs

TW = 14
OFFSETS = [p for p in itertools.product((-1, 0, 1), repeat=3) if p != (0, 0, 0)]


@pytest.fixture
def recon3d():
    oracle.set_recon(oracle.RECON_3D)
    yield
    oracle.set_recon(oracle.RECON_AXIS)


def _linear_tile(a, b, c, d0):
    # value at tile cell (x, y, z) = d0 + a x + b y + c z, stored [z][y][x]
    z, y, x = np.meshgrid(np.arange(TW), np.arange(TW), np.arange(TW), indexing="ij")
    return d0 + a * x + b * y + c * z


@pytest.mark.parametrize("coef", [(1.0, 0.0, 0.0), (0.25, -2.0, 0.5), (-3.0, 1.5, 4.0)])
def test_linear_data_is_exact_at_every_point(coef):
    a, b, c = coef
    tile = _linear_tile(a, b, c, 7.0)
    for t in ((5, 5, 5), (3, 10, 7), (2, 11, 4)):
        base = 7.0 + a * t[0] + b * t[1] + c * t[2]
        for p in OFFSETS:
            want = base + 0.5 * (a * p[0] + b * p[1] + c * p[2])
            assert oracle.point_value(tile, t, p) == want, (t, p)


def test_point_values_are_the_two_ends_of_one_line():
    # opposite points of a cell come from the same line: on data that the
    # limiter flattens along that line only, both ends equal the cell value
    rng = np.random.default_rng(5)
    tile = rng.random((TW, TW, TW))
    t = (6, 6, 6)
    for p in OFFSETS:
        e = np.array(p)
        # make cell t a local maximum along the line t + m e only
        tt = tile.copy()
        tt[t[2], t[1], t[0]] = 10.0
        assert oracle.point_value(tt, t, p) == 10.0
        assert oracle.point_value(tt, t, tuple(-e)) == 10.0


def _uniform_tiles(nf=6, rho=1.0, v=(0.3, 0.0, 0.0), p=1.0):
    U = inputs.conserved(np.array([rho]), np.array([v[0]]), np.array([v[1]]), np.array([v[2]]),
                         np.array([p]))
    tiles = np.empty((nf, TW, TW, TW))
    for f in range(min(nf, U.shape[0])):
        tiles[f] = U[f][0]
    return tiles


@pytest.mark.parametrize("d", [0, 1, 2])
def test_linear_species_integrates_to_the_face_centre_value(d):
    # uniform flow along d, a passive species linear in all coordinates: the
    # reconstruction is exact and continuous, so each point flux is rho_k v_d
    # at that point and Simpson's rule returns the face-centre value exactly
    v = [0.0, 0.0, 0.0]
    v[d] = 0.5
    tiles = np.empty((7, TW, TW, TW))
    tiles[:6] = _uniform_tiles(6, v=tuple(v))
    tiles[6] = _linear_tile(0.125, -0.25, 0.5, 4.0)
    tl = [6, 6, 6]
    H, bad = oracle.face_flux_3d(tiles, d, tl)
    assert bad == 0
    centre = [6.0, 6.0, 6.0]
    centre[d] += 0.5
    rk = 4.0 + 0.125 * centre[0] - 0.25 * centre[1] + 0.5 * centre[2]
    assert H[6] == rk * 0.5
    # and the core fields see a uniform state: the physical flux
    Hu, _ = oracle.face_flux(d, tiles[:6, 6, 6, 6], tiles[:6, 6, 6, 6])
    np.testing.assert_allclose(H[:6], Hu, rtol=1e-15, atol=1e-17)


def test_uniform_state_is_bit_identical(recon3d):
    for w in (inputs.uniform_state(2, nf=6), inputs.uniform_state(2, nf=11)):
        T = oracle.Table(w.leaf_coord, w.base)
        U = w.U
        for _ in range(2):
            U, dt, bad = oracle.rk3_step(T, U, 0.4)
            assert bad == 0 and dt > 0
        assert np.array_equal(U, w.U)


def test_uniform_state_is_bit_identical_on_an_uneven_octree(recon3d):
    w = inputs.blobs(base=2, max_level=2, threshold=0.5)
    u = inputs.uniform_state(1, nf=11)
    U = np.repeat(u.U[:, :1], w.n_leaves, axis=1)
    T = oracle.Table(w.leaf_coord, w.base)
    out, _, bad = oracle.rk3_step(T, U, 0.4)
    assert bad == 0 and np.array_equal(out, U)


def test_periodic_uniform_level_conserves_totals(recon3d):
    w = inputs.random_smooth(inputs.uniform_leaves(2), 2, nf=11, seed=1, amp=0.2)
    T = oracle.Table(w.leaf_coord, w.base)
    before = oracle.totals(T, w.U)
    U, _, bad = oracle.rk3_step(T, w.U, 0.4)
    assert bad == 0
    after = oracle.totals(T, U)
    scale = oracle.totals(T, np.abs(U))
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale


def _global(U, base):
    coord = inputs.uniform_leaves(base)
    nf = U.shape[0]
    N = 8 * base
    out = np.empty((nf, N, N, N))
    for i, (_, x, y, z) in enumerate(coord):
        out[:, 8 * z:8 * z + 8, 8 * y:8 * y + 8, 8 * x:8 * x + 8] = U[:, i]
    return out


def _leaves(Gl, base):
    coord = inputs.uniform_leaves(base)
    return np.stack([Gl[:, 8 * z:8 * z + 8, 8 * y:8 * y + 8, 8 * x:8 * x + 8]
                     for (_, x, y, z) in coord], 1)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_bit_exact(recon3d, axis):
    base = 2
    w = inputs.random_smooth(inputs.uniform_leaves(base), base, nf=7, seed=2, amp=0.1)
    T = oracle.Table(w.leaf_coord, w.base)
    Gl = _global(w.U, base)
    ax = 3 - axis
    M = np.flip(Gl, ax).copy()
    M[1 + axis] = -M[1 + axis]
    out, _ = oracle.step(T, w.U, 1e-3)
    outm, _ = oracle.step(T, _leaves(M, base), 1e-3)
    back = np.flip(_global(outm, base), ax).copy()
    back[1 + axis] = -back[1 + axis]
    assert np.array_equal(back, _global(out, base))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_symmetric_data_reduces_to_the_1d_solver(recon3d, axis):
    # all 9 points of a face normal to the axis see the 1D face states, the
    # transverse faces cancel exactly; the Simpson sum (36 H) / 36 returns H
    # to within a few ulp
    base = 2
    N = 8 * base
    x = (np.arange(N) + 0.5) / N
    rho1 = np.where(x < 0.5, 1.0, 0.125) + 0.01 * np.sin(2 * np.pi * x)
    p1 = np.where(x < 0.5, 1.0, 0.1)
    v1 = 0.2 * np.cos(2 * np.pi * x)
    z = np.zeros(N)
    U1 = inputs.conserved(rho1, v1, z, z, p1)
    dt = 1e-3
    ref, _ = oracle.step_1d(U1, dt)
    Gl = np.empty((6, N, N, N))
    shape = [1, 1, 1]
    shape[2 - axis] = N
    for f, src in enumerate(U1):
        Gl[f] = src.reshape(shape)
    mom = Gl[1].copy()
    Gl[1:4] = 0.0
    Gl[1 + axis] = mom
    w = inputs.uniform_state(base)
    T = oracle.Table(w.leaf_coord, w.base)
    out, _ = oracle.step(T, _leaves(Gl, base), dt)
    o = _global(out, base)
    for f in range(6):
        if f in (1, 2, 3) and f != 1 + axis:
            assert np.all(o[f] == 0.0)
            continue
        src_f = 1 if f == 1 + axis else f
        line = np.moveaxis(o[f], 2 - axis, 0).reshape(N, -1)
        assert np.all(line == line[:, :1])  # exactly plane symmetric
        np.testing.assert_allclose(line[:, 0], ref[src_f], rtol=1e-14, atol=1e-16)


def test_differs_from_the_face_centre_flux_on_3d_data(recon3d):
    # on a genuinely 3D state the 9-point flux is a different operator (on
    # plane-symmetric data the two agree, pinned above)
    w = inputs.random_smooth(inputs.uniform_leaves(2), 2, nf=6, seed=8, amp=0.2)
    T = oracle.Table(w.leaf_coord, w.base)
    a, bad = oracle.step(T, w.U, 1e-3)
    assert bad == 0 and np.all(np.isfinite(a))
    oracle.set_recon(oracle.RECON_AXIS)
    b, _ = oracle.step(T, w.U, 1e-3)
    oracle.set_recon(oracle.RECON_3D)
    assert np.abs(a - b).max() > 1e-9


def test_flux_correction_keeps_uneven_trees_conservative(recon3d):
    # the coarse-fine correction acts on the quadrature fluxes of the faces
    import math
    w = inputs.blobs(base=2, max_level=2, threshold=0.5)
    s = inputs.random_smooth(w.leaf_coord, w.base, nf=7, seed=3, amp=0.2)
    T = oracle.Table(w.leaf_coord, w.base)
    dv = (1.0 / (8.0 * w.base * 2.0 ** w.leaf_coord[:, 0])) ** 3

    def tot(U):
        return np.array([math.fsum((U[f] * dv[:, None, None, None]).ravel().tolist())
                         for f in range(U.shape[0])])
    before, scale = tot(s.U), tot(np.abs(s.U))
    out, _, bad = oracle.rk3_step(T, s.U, 0.4, reflux=True)
    assert bad == 0
    assert np.all(np.abs(tot(out) - before) <= 1e-13 * scale)
    out2, _, _ = oracle.rk3_step(T, s.U, 0.4, reflux=False)
    assert np.abs(tot(out2) - before).max() > 1e-9 * scale.max()


# -- the face quadrature's weights --------------------------------------------
#
# Tensor-product Simpson weights over the 3 x 3 face points, built here from
# the 1D rule (1, 4, 1)/6 and indexed [pv + 1][pu + 1].
SIMPSON_1D = np.array([1.0, 4.0, 1.0]) / 6.0
SIMPSON_2D = np.outer(SIMPSON_1D, SIMPSON_1D)
# Plausible wrong rules: each is normalised and symmetric in both axes.
WRONG_RULES = {
    "1d-simpson-along-u": np.outer([0.0, 1.0, 0.0], SIMPSON_1D),
    "corners-1-edges-4-centre-4-over-24": np.array([[1, 4, 1], [4, 4, 4], [1, 4, 1]]) / 24.0,
    "no-corners-edges-1-centre-2-over-6": np.array([[0, 1, 0], [1, 2, 1], [0, 1, 0]]) / 6.0,
    "midpoint": np.array([[0, 0, 0], [0, 1, 0], [0, 0, 0]], dtype=float),
    "trapezoid": np.outer([0.25, 0.5, 0.25], [0.25, 0.5, 0.25]),
}


def _face_axes(d):
    return (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))


def _point_fluxes(tiles, d, tl):
    """KT flux at each of the 9 face points [pv + 1][pu + 1][field], from the
    separately pinned point values (linear exactness, line ends) and the
    separately pinned point flux."""
    u, v = _face_axes(d)
    tr = list(tl)
    tr[d] += 1
    H = np.empty((3, 3, tiles.shape[0]))
    for pv in (-1, 0, 1):
        for pu in (-1, 0, 1):
            pl, pr = [0, 0, 0], [0, 0, 0]
            pl[d], pr[d] = 1, -1
            pl[u] = pr[u] = pu
            pl[v] = pr[v] = pv
            UL = np.array([oracle.point_value(tiles[f], tl, pl) for f in range(tiles.shape[0])])
            UR = np.array([oracle.point_value(tiles[f], tr, pr) for f in range(tiles.shape[0])])
            H[pv + 1, pu + 1], bad = oracle.face_flux(d, UL, UR)
            assert bad == 0
    return H


def _smooth_tiles(seed, nf=8):
    # a smooth, genuinely 3D state: every face point sees a different state
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(TW), np.arange(TW), np.arange(TW), indexing="ij")

    def fld(a0, a):
        k = rng.uniform(0.2, 0.6, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        return a0 + a * np.sin(k[0] * x + ph[0]) * np.cos(k[1] * y + ph[1]) * np.sin(
            k[2] * z + ph[2])
    rho = fld(1.0, 0.3)
    vx, vy, vz = fld(0.1, 0.4), fld(-0.2, 0.4), fld(0.05, 0.4)
    p = fld(1.0, 0.2)
    spec = [rho * fld(0.5, 0.3) for _ in range(nf - 6)]
    U = inputs.conserved(rho.ravel(), vx.ravel(), vy.ravel(), vz.ravel(), p.ravel(),
                         species=[s.ravel() for s in spec] if spec else None)
    return np.ascontiguousarray(U.reshape(nf, TW, TW, TW))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_face_flux_is_the_tensor_simpson_rule_of_the_point_fluxes(d):
    tiles = _smooth_tiles(40 + d)
    tl = [6, 5, 7]
    Hp = _point_fluxes(tiles, d, tl)
    H, bad = oracle.face_flux_3d(tiles, d, tl)
    assert bad == 0
    want = np.einsum("ab,abf->f", SIMPSON_2D, Hp)
    scale = np.abs(Hp).max(axis=(0, 1))
    assert np.all(np.abs(H - want) <= 4e-16 * scale), (H - want) / scale
    # the data tells the rules apart: every wrong rule misses by far more
    for name, W in WRONG_RULES.items():
        miss = np.abs(np.einsum("ab,abf->f", W, Hp) - H) / scale
        assert miss.max() > 1e-6, name


def _species_times_velocity_tiles(d, axis, a, b, s0, s1):
    # rho = 1 and p = 1 uniform; the normal momentum s_d = s0 + s1 t_axis and
    # a passive species a + b t_axis, both linear in the tile coordinate of
    # one transverse axis, so the reconstruction reproduces both exactly at
    # every face point and the species' point flux is the quadratic
    # (a + b t)(s0 + s1 t)
    z, y, x = np.meshgrid(np.arange(TW), np.arange(TW), np.arange(TW), indexing="ij")
    t = (x, y, z)[axis].astype(float)
    one = np.ones_like(t)
    v = [0.0 * one, 0.0 * one, 0.0 * one]
    v[d] = s0 + s1 * t
    U = inputs.conserved(one.ravel(), v[0].ravel(), v[1].ravel(), v[2].ravel(), one.ravel(),
                         species=[(a + b * t).ravel()])
    return np.ascontiguousarray(U.reshape(7, TW, TW, TW))


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("which", [0, 1])
def test_simpson_integrates_a_quadratic_transverse_flux_exactly(d, which):
    # Simpson's rule is exact for quadratics: the face mean of
    # (a + b t)(s0 + s1 t) over the cell-wide face [t_c - 1/2, t_c + 1/2] is
    # (a + b t_c)(s0 + s1 t_c) + b s1 / 12.  The midpoint rule misses the
    # b s1 / 12 term, a trapezoid rule doubles it.  All inputs are dyadic, so
    # the nine point fluxes are exact and only the final division rounds.
    axis = _face_axes(d)[which]
    a, b, s0, s1 = 4.0, 0.125, 0.5, 0.0625
    tiles = _species_times_velocity_tiles(d, axis, a, b, s0, s1)
    tl = [6, 5, 7]
    H, bad = oracle.face_flux_3d(tiles, d, tl)
    assert bad == 0
    tc = float(tl[axis])
    exact = (a + b * tc) * (s0 + s1 * tc) + b * s1 / 12.0
    assert abs(H[6] - exact) <= 2e-16 * exact, (H[6], exact)
    assert abs(b * s1 / 12.0) > 1e4 * 2e-16 * exact  # the quadratic term is resolved
