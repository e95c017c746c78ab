"""Precision guard of the FP32-bulk step (Eq. 20), through the C ABI, and the error bound of a
step per patch that every FP32-bulk parity test uses.

Eq. 20 puts the error of recovering the pressure from conserved variables that carry a relative
rounding error eps at (1 + M^2) eps.  An FP32 bulk rounds the half-step face states and the
update increment to FP32, so its one-step error grows with kappa = 1 + M^2 of the patch's tile:
  * the jet's nozzle state (gamma = 10^3, Theta = 10^2) has kappa ~ 2e6 -- with the guard off the
    FP32 bulk moves the nozzle face pressure by about 1.5 % and the cold neighbour's reduced
    energy by as much; with the guard on (kappa_max = 1024) the patches whose tile reaches the
    nozzle are stepped in FP64;
  * a moving gas below the threshold stays in FP32, at kappa ~ 6, 62 and 550.

The bound per patch, (C_KAPPA kappa_tile + C_FLUX) u (tests/parity.py, step_bound):
  * C_KAPPA = 16: a face state's conserved variables carry about 4 roundings each (prim -> cons,
    the half-step correction); Eq. 20 turns that into about 4 kappa u in L, hence in Theta and
    p, and a flux inherits at most the pressure's relative error; doubled for the two face
    states of an interface, doubled again as margin;
  * C_FLUX = 32: each Riemann flux component comes out of about 8 dependent roundings (signal
    speeds, HLL averages, contact speed, star state), six flux differences enter a cell's
    increment, which is summed and rounded once more, and dt/dh |F| stays below the CFL
    number times |U|: about 6 x 8 x 0.5 + 2 = 26, rounded up.  The momentum's error is measured
    against the grid's largest |M|, which a pressure jump of the same size creates in one step.
The pressure recovered from the updated conserved variables carries Eq. 20's amplification of
their error once more: the squares of x = Et/D in L double it and D's own error doubles it
again, hence 4 (C_KAPPA kappa_tile + C_FLUX) u.  The same holds in FP64 with u_64 = 2^-53: where
that exceeds 1e-10 (kappa above about 6e4, the nozzle) two correct FP64 steps differ by that
much, so FP64 parity there is judged by max(1e-10, (C_KAPPA kappa_tile + C_FLUX) u_64)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import (U32, U64, kappa_prim, oracle_cons, patch_errors, soa, step_bound,
                           step_errors, tile_max)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KMAX = 1024.0


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _setup(g):
    cons = oracle_cons(g)
    dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad_o = O.fill_ghosts(cons, g.neighbor, 3)
    ref, _ = O.fluid_step(pad_o, dt_o, g.dh_lev)
    kap = tile_max(kappa_prim(soa(g.prim)).reshape(g.n_patch, 8, 8, 8), g.neighbor)
    return cons, dt_o, pad_o, ref, kap


@pytest.mark.parametrize("prec", [1, 2])
def test_jet_block_padded(S, prec):
    g = W.jet_block()
    cons, dt_o, pad_o, ref, kap = _setup(g)
    hot = kap > KMAX
    assert hot.any() and (~hot).any()
    pad, dt = _gpu(pad_o), _gpu(dt_o)
    out64 = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=0).cpu().numpy()
    off = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, kappa_max=0.0).cpu().numpy()
    st = S.new_stats(DEV)
    on = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, kappa_max=KMAX, stats=st).cpu().numpy()
    sd = S.stats_dict(st)
    e_off, e_on = patch_errors(off, ref), patch_errors(on, ref)
    print("prec %d: guard off max error %.3e; on: hot patches %.3e, others %.3e (bound %.3e); %s"
          % (prec, e_off.max(), e_on[hot].max(), e_on[~hot].max(),
             step_bound(kap[~hot]).max(), sd))
    fp64_bound = np.maximum(1e-10, step_bound(kap, U64))
    assert np.all(patch_errors(out64, ref) <= fp64_bound)
    assert sd["n_fp64_patch"] == hot.sum()
    assert e_off.max() > 1e-3                      # the FP32 bulk loses the nozzle's pressure
    assert np.all(e_on[hot] <= fp64_bound[hot])    # stepped in FP64
    assert patch_errors(on[hot], out64[hot]).max() <= 1e-13   # the FP64 kernel's results
    assert np.all(e_on[~hot] <= step_bound(kap[~hot]))


@pytest.mark.parametrize("U", [0.3, 1.0, 3.0])
@pytest.mark.parametrize("prec", [1, 2])
def test_moving_gas_error_follows_kappa(S, prec, U):
    g = W.moving_gas(U=U, theta=1e-2)
    cons, dt_o, pad_o, ref, kap = _setup(g)
    assert kap.max() < KMAX
    st = S.new_stats(DEV)
    out = S.srhd_fluid_step(_gpu(pad_o), _gpu(dt_o), g.dh_lev, prec=prec, kappa_max=KMAX,
                            stats=st).cpu().numpy()
    e = patch_errors(out, ref)
    ratio = e / (kap * U32)
    print("prec %d U %.1f: kappa %.1f..%.1f, max error %.3e, error / (kappa u32) max %.2f median %.2f"
          % (prec, U, kap.min(), kap.max(), e.max(), ratio.max(), np.median(ratio)))
    assert S.stats_dict(st)["n_fp64_patch"] == 0
    assert np.all(e <= step_bound(kap))
    # where the amplification shows: the pressure of the updated state (its L is Eq. 15's left-hand
    # side of conserved variables that carry the FP32 step's rounding), per patch
    P = g.n_patch
    pg = O.cons2prim(soa(out))[0][4].reshape(P, -1)
    pr = O.cons2prim(soa(ref))[0][4].reshape(P, -1)
    ep = np.max(np.abs(pg / pr - 1), axis=1)
    print("   pressure of the updated state: max error %.3e, error / (kappa u32) max %.2f"
          % (ep.max(), (ep / (kap * U32)).max()))
    assert np.all(ep <= 4 * step_bound(kap))


def test_jet_block_gather_chain(S):
    # two steps of the gather-layout chain (FP32 primitives between steps) with the guard; each
    # step is compared with the oracle's step of the GPU's own input state
    g = W.jet_block()
    cons, dt_o, pad_o, ref, kap = _setup(g)
    nb = _gpu(g.neighbor)
    c = _gpu(cons)
    prims, smax = S.srhd_grid_prims(c, prec=1)
    for step in range(2):
        cin = c.cpu().numpy()
        k_host = tile_max(kappa_prim(O.cons2prim(soa(cin))[0]).reshape(g.n_patch, 8, 8, 8),
                          g.neighbor)
        dt_h, _, _ = O.cfl_dt(cin, None, g.dh_lev, 0.5)
        ref, _ = O.fluid_step(O.fill_ghosts(cin, g.neighbor, 3), dt_h, g.dh_lev)
        st = S.new_stats(DEV)
        c, prims, smax = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, dt_lev=_gpu(dt_h), prec=1,
                                                stats=st, kappa_max=KMAX)
        out = c.cpu().numpy()
        hot = k_host > KMAX
        e = patch_errors(out, ref)
        sd = S.stats_dict(st)
        print("gather step %d: hot %d (device %d), errors hot %.3e others %.3e"
              % (step, hot.sum(), sd["n_fp64_patch"], e[hot].max(), e[~hot].max()))
        assert sd["n_fp64_patch"] == hot.sum() and hot.any()
        assert np.all(e[hot] <= np.maximum(1e-10, step_bound(k_host[hot], U64)))
        assert np.all(e[~hot] <= step_bound(k_host[~hot]))


def test_guard_arguments(S):
    g = W.moving_gas(U=0.3)
    pad = _gpu(O.fill_ghosts(oracle_cons(g), g.neighbor, 3))
    dt = _gpu(np.array([1e-3]))
    with pytest.raises(S.SrhdError):
        S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, kappa_max=0.5)
    with pytest.raises(S.SrhdError):
        S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, kappa_max=float("nan"))
    # the FP64 step ignores the guard
    a = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=0, kappa_max=KMAX)
    b = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=0, kappa_max=0.0)
    assert torch.equal(a, b)
