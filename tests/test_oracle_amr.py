"""Pins of the oracle's AMR neighbour operations (Sec. 3.4 items 3 and 4, refinement ratio 2):
restriction, coarse-to-fine ghost interpolation with the primitive fallback, boundary fluxes and
the coarse-fine flux correction, and a two-level cycle built from them (one coarse step, two fine
sub-steps with time-interpolated coarse ghosts, restriction, flux correction).

What fixes them: a uniform state passes the whole cycle bit for bit; linear coarse data is
interpolated exactly; the eight children of a coarse cell average back to it (restriction and
interpolation both); with the flux correction the cycle conserves D, M and Et exactly over the
composite grid (periodic box), without it it does not; every interpolated ghost is physical,
also where the conserved-variable interpolation is not and the primitive fallback is taken."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import oracle_driver as drv


def _wave(x, y, z):
    s = np.sin(2 * np.pi * (x + 0.5 * y))
    return (1.0 + 0.2 * s, 0.3 + 0.1 * np.cos(2 * np.pi * z) + 0 * x, 0.1 * s, 0.0 * x,
            1.0 + 0.3 * np.cos(2 * np.pi * y) + 0 * x)


def test_geometry_of_the_two_level_hierarchy():
    t = W.two_level(4, 1, 3)
    assert t["fine_neighbor"].shape == (64, 27) and t["faces"].shape == (24, 6)
    # every fine patch's parent is refined and lists it as the child at its octant
    row = {int(P): k for k, P in enumerate(t["parent_of"])}
    for f in range(64):
        assert t["refined"][t["parent"][f]]
        assert t["child"][row[int(t["parent"][f])], t["octant"][f]] == f


def test_restriction_is_the_average_and_conserves():
    t = W.two_level(4, 1, 3)
    rng = np.random.default_rng(7)
    fine = rng.uniform(0.5, 2.0, (64, 5, 8, 8, 8))
    coarse = np.zeros((64, 5, 8, 8, 8))
    O.restrict(coarse, t["parent_of"], t["child"], fine)
    tot_c = coarse[t["parent_of"]].sum(axis=(0, 2, 3, 4)) * t["dh_c"] ** 3
    tot_f = fine.sum(axis=(0, 2, 3, 4)) * t["dh_f"] ** 3
    assert np.allclose(tot_c, tot_f, rtol=1e-14, atol=0)
    # one coarse cell against its eight children by hand
    P, k = int(t["parent_of"][3]), 3
    ch = fine[t["child"][k, 7]]                       # octant 7 covers coarse cells (4..7)^3
    assert np.allclose(coarse[P, :, 5, 6, 4], ch[:, 2:4, 4:6, 0:2].mean(axis=(1, 2, 3)), rtol=1e-15)


def _coarse_padded_from_fn(t, fn):
    nc = t["nc"]
    cc = np.empty((nc ** 3, 5, 8, 8, 8))
    x, y, z = t["coarse_xyz"]
    for f in range(5):
        cc[:, f] = fn(f, x, y, z)
    return cc, O.fill_ghosts(cc, t["coarse_neighbor"], 3)


def test_linear_coarse_data_is_interpolated_exactly():
    # conserved variables linear in x, y, z inside the refined region and its 3-cell halo (the
    # periodic wrap is far away): the limited slopes equal the differences, so every
    # interpolated fine ghost equals the linear function at its centre
    t = W.two_level(4, 1, 3)
    a = np.array([1.0, 0.01, -0.02, 0.0, 2.0])
    b = np.array([[0.3, 0.1, -0.2], [0.05, 0.0, 0.01], [0.0, 0.02, 0.0], [0.0, 0.0, 0.0],
                  [0.4, -0.1, 0.2]])
    fn = lambda f, x, y, z: a[f] + b[f, 0] * x + b[f, 1] * y + b[f, 2] * z
    _, pad_c = _coarse_padded_from_fn(t, fn)
    fine = np.zeros((64, 5, 8, 8, 8))
    pad_f = O.fill_ghosts(fine, t["fine_neighbor"], 3)
    pad_f[:] = np.nan
    n, nfb = O.fill_ghosts_coarse(pad_f, t["fine_neighbor"], t["parent"], t["octant"], pad_c)
    assert nfb == 0 and n > 0
    dhf = t["dh_f"]
    nf = t["nf"]
    lo = 2 * 1
    idx = np.arange(14) - 3
    checked = 0
    for p in range(64):
        fz, rem = divmod(p, nf * nf)
        fy, fx = divmod(rem, nf)
        X = ((lo + fx) * 8 + idx + 0.5) * dhf
        Y = ((lo + fy) * 8 + idx + 0.5) * dhf
        Z = ((lo + fz) * 8 + idx + 0.5) * dhf
        got = pad_f[p]
        mask = np.isfinite(got[0])
        for f in range(5):
            ref = a[f] + b[f, 0] * X[None, None, :] + b[f, 1] * Y[None, :, None] + b[f, 2] * Z[:, None, None]
            assert np.allclose(got[f][mask], np.broadcast_to(ref, got[f].shape)[mask], rtol=1e-13, atol=1e-15)
        checked += mask.sum()
    # exactly the ghost cells whose slot is covered by level 0 were written
    assert checked == n


def test_interpolated_children_average_to_the_coarse_cell():
    t = W.two_level(4, 1, 3)
    rng = np.random.default_rng(3)
    w = lambda f, x, y, z: (1 + 0.5 * rng.random(x.shape) if f in (0, 4) else 0.2 * (rng.random(x.shape) - 0.5))
    cw = np.stack([w(f, *t["coarse_xyz"]) for f in range(5)], axis=1)
    P = cw.shape[0]
    cc = np.ascontiguousarray(O.prim2cons(cw.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1))
                              .reshape(5, P, 512).transpose(1, 0, 2)).reshape(P, 5, 8, 8, 8)
    pad_c = O.fill_ghosts(cc, t["coarse_neighbor"], 3)
    pad_f = O.fill_ghosts(np.zeros((64, 5, 8, 8, 8)), t["fine_neighbor"], 3)
    O.fill_ghosts_coarse(pad_f, t["fine_neighbor"], t["parent"], t["octant"], pad_c)
    # fine patch 0 sits at the lower corner of the fine block: its ghosts x in {-2, -1} (array
    # 1, 2), y and z inside, are complete 2x2x2 groups of children of coarse cells x = -1
    p = 0
    par = t["parent"][p]
    for cy in range(4):
        for cz in range(4):
            grp = pad_f[p][:, 3 + 2 * cz:5 + 2 * cz, 3 + 2 * cy:5 + 2 * cy, 1:3]
            ref = pad_c[par][:, 3 + cz, 3 + cy, 3 - 1]
            assert np.allclose(grp.mean(axis=(1, 2, 3)), ref, rtol=1e-13), (cy, cz)


def test_primitive_fallback_keeps_ghosts_physical():
    # a cold (Theta = 1e-6) flow whose four-velocity varies between 1 and 100: the physical
    # margin L ~ 3 Theta is tiny next to m^2, the conserved variables' limited slopes differ per
    # component, and the interpolated conserved state leaves the physical region in many cells;
    # the primitive interpolation is physical
    t = W.two_level(4, 1, 3)
    def fn(x, y, z):
        Ux = 10 ** (np.sin(6 * np.pi * x) + 1)
        Uy = 0.5 * 10 ** np.cos(4 * np.pi * y)
        rho = 1 + 0.9 * np.sin(10 * np.pi * z)
        return (rho, Ux, Uy, 0 * x, 1e-6 * rho)
    _, cc, _ = drv.amr_setup(4, 1, 3, fn)
    pad_c = O.fill_ghosts(cc, t["coarse_neighbor"], 3)
    pad_f = O.fill_ghosts(np.zeros((64, 5, 8, 8, 8)), t["fine_neighbor"], 3)
    mark = np.full(pad_f.shape, np.nan)
    pad_f[:] = mark
    n, nfb = O.fill_ghosts_coarse(pad_f, t["fine_neighbor"], t["parent"], t["octant"], pad_c)
    print("interpolated %d ghosts, %d by the primitive fallback" % (n, nfb))
    assert nfb > 0
    u = pad_f.transpose(1, 0, 2, 3, 4).reshape(5, -1)
    u = u[:, np.isfinite(u[0])]
    assert u.shape[1] == n
    assert all(O.is_physical(u[:, i]) for i in range(u.shape[1]))


def test_uniform_state_passes_the_cycle_bitwise():
    const = lambda x, y, z: (0.7 + 0 * x, 0.2 + 0 * x, -0.1 + 0 * x, 0.05 + 0 * x, 3.0 + 0 * x)
    t, cc, cf = drv.amr_setup(4, 1, 3, const)
    c1, f1, _, info = drv.amr_step(t, cc, cf)
    assert np.array_equal(c1, cc) and np.array_equal(f1, cf)
    assert info["skipped"] == 0


@pytest.mark.parametrize("integrator", [0, 1])
def test_flux_correction_makes_the_cycle_conservative(integrator):
    t, cc, cf = drv.amr_setup(4, 1, 3, _wave)
    tot0 = drv.amr_totals(t, cc, cf)
    c1, f1, dt, info = drv.amr_step(t, cc, cf, integrator=integrator)
    assert info["coarse_counts"][3] == 0 and all(c[3] == 0 for c in info["fine_counts"])
    tot1 = drv.amr_totals(t, c1, f1)
    scale = np.abs(cc).sum(axis=(0, 2, 3, 4)) * t["dh_c"] ** 3
    scale[1:4] = scale[1:4].max()                    # momentum components against |M|'s scale
    rel = np.abs(tot1 - tot0) / scale
    print("conservation with flux correction: %s" % rel)
    assert np.all(rel < 1e-14), rel
    # without the correction the composite sums change at the first order of the flux mismatch
    c2, f2, _, _ = drv.amr_step(t, cc, cf, correct=False, integrator=integrator)
    rel2 = np.abs(drv.amr_totals(t, c2, f2) - tot0) / scale
    print("without: %s" % rel2)
    assert rel2[0] > 1e-9 and rel2[4] > 1e-9, rel2
