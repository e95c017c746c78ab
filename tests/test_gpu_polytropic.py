"""GPU parity with the polytropic EoS of Sec. 2.2 (srhd_eos kind SRHD_EOS_POLYTROPIC) against the
oracle under the same EoS, through the C ABI: the conversions (FP64 to round-off, FP32 within
its stated error), the CFL time step, one MUSCL-Hancock step of a shock tube and of the 64^3
blast (FP64 within 1e-10 for HLLC and HLLE, the FP32-bulk modes within their stated error, the
persistent schedule bit for bit), a multi-step run with limiter retries, and the refused
combinations."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import kappa_tile_padded, patch_errors, step_bound
from tests.parity import prim_errors, soa, step_errors, unsoa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GAMMAS = [4.0 / 3.0, 5.0 / 3.0]


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cons(grid, gamma):
    with O.eos(gamma):
        return unsoa(O.prim2cons(soa(grid.prim)), grid.n_patch)


@pytest.mark.parametrize("gamma", GAMMAS)
def test_conversions(S, gamma):
    prim = W.conversion_batch(200_000, seed=31)
    with O.eos(gamma):
        cons = O.prim2cons(prim)
        ref, st, _ = O.cons2prim(cons)
    c = S.srhd_prim2cons(_g(prim), gamma=gamma)
    w, sg, _ = S.srhd_cons2prim(_g(cons), status=True, gamma=gamma)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    scale = np.abs(cons).max(axis=0)
    ec = float(np.max(np.abs(c - cons) / np.maximum(np.abs(cons), 1e-300 + 1e-16 * scale)))
    ok = (st == O.ST_OK) & (sg.cpu().numpy() == 0)
    assert np.array_equal(sg.cpu().numpy() == 1, st == O.ST_UNPHYSICAL)
    e64 = prim_errors(w.cpu().numpy(), ref, ok)
    print("Gamma %.4f: prim2cons %.2e; cons2prim fp64 %s" % (gamma, ec, e64))
    assert ec <= 1e-13
    assert max(e64.values()) <= 1e-12, e64


@pytest.mark.parametrize("gamma", GAMMAS)
def test_cons2prim_fp32_error_is_stated(S, gamma):
    # as for the TM EoS: FP32 inputs, the FP64 oracle on the upcast inputs; per state the error is
    # bounded by the Eq. 20 amplification kappa ~ 1 + Mach^2 of the FP32 round-off of L (kappa from
    # the state, L being the EoS-free left-hand side of Eq. 15), plus a few u32 of Newton tolerance
    # and recovery: 16 u32 (kappa + 4), over the states FP32 can represent (kappa u32 < 1e-2)
    prim = W.conversion_batch(200_000, seed=23)
    with O.eos(gamma):
        cons32 = O.prim2cons(prim).astype(np.float32)
        cons64 = cons32.astype(np.float64)
        ref, st_ref, _ = O.cons2prim(cons64)
    w, st, _ = S.srhd_cons2prim(_g(cons32), status=True, gamma=gamma)
    w, st = w.cpu().numpy().astype(np.float64), st.cpu().numpy()
    ok = (st_ref == 0) & (st == 0)
    D, M2, Et = cons64[0], (cons64[1:4] ** 2).sum(axis=0), cons64[4]
    x = Et / D
    with np.errstate(over="ignore", divide="ignore"):
        kappa = (x * x + 2 * x + M2 / D ** 2) / np.maximum(O.L_batch(cons64), 1e-300)
    u32 = 2.0 ** -24
    with np.errstate(invalid="ignore", divide="ignore"):
        er = np.abs(w[0] / ref[0] - 1)
        ep = np.abs(w[4] / ref[4] - 1)
        eu = np.max(np.abs(w[1:4] - ref[1:4]), axis=0) / np.maximum(np.sqrt((ref[1:4] ** 2).sum(axis=0)), 1e-300)
    emax = np.maximum(np.maximum(er, ep), eu)
    rep = ok & (kappa * u32 < 1e-2)
    ratio = emax[rep] / (u32 * (kappa[rep] + 4))
    print("Gamma %.4f fp32: %d states with kappa u32 < 1e-2; error / (u32 (kappa + 4)): median %.3f, "
          "max %.3f" % (gamma, rep.sum(), np.median(ratio), ratio.max()))
    assert rep.sum() > 1000
    assert np.all(emax[rep] <= 16 * u32 * (kappa[rep] + 4))
    assert not np.any((st == 0) & (st_ref == O.ST_UNPHYSICAL))


@pytest.mark.parametrize("gamma", GAMMAS)
@pytest.mark.parametrize("riemann", [0, 1])
def test_one_step_fp64(S, gamma, riemann):
    for g in (W.riemann_1d(64, (1.0, 0.0, 0.0, 0.0, 1e3), (0.5, 0.3, 0.0, 0.0, 1e-6)),
              W.blast(64, seed=3)):
        cons = _cons(g, gamma)
        with O.eos(gamma):
            dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
            pad_o = O.fill_ghosts(cons, g.neighbor, 3)
            ref, cnt = O.fluid_step(pad_o, dt_o, g.dh_lev, solver=riemann)
        c = _g(cons)
        dt_g = S.srhd_cfl_dt(c, g.dh_lev, 0.5, gamma=gamma)
        pad = S.srhd_fill_ghosts(c, _g(g.neighbor), 3)
        st = S.new_stats(DEV)
        out = S.srhd_fluid_step(pad, _g(dt_o), g.dh_lev, riemann=riemann, stats=st, gamma=gamma)
        o2 = S.srhd_fluid_step(pad, _g(dt_o), g.dh_lev, riemann=riemann, gamma=gamma,
                               sched=S.Sched(300, 2, DEV))
        torch.cuda.synchronize()
        assert torch.equal(out, o2)
        assert abs(dt_g.cpu().numpy()[0] / dt_o[0] - 1) < 1e-13
        e = step_errors(out.cpu().numpy(), ref)
        sd = S.stats_dict(st)
        print("Gamma %.4f %s riemann %d: %s, stats %s, oracle %s" % (gamma, g.name, riemann, e, sd, cnt))
        assert max(e.values()) <= 1e-10, e
        assert sd["n_retry"] == cnt[3] and sd["n_unphysical"] == cnt[0]


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_bulk_error_is_stated(S, prec):
    gamma = 5.0 / 3.0
    g = W.blast(32, seed=3)
    cons = _cons(g, gamma)
    with O.eos(gamma):
        dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
        pad_o = O.fill_ghosts(cons, g.neighbor, 3)
        ref, _ = O.fluid_step(pad_o, dt_o, g.dh_lev)
    out = S.srhd_fluid_step(_g(pad_o), _g(dt_o), g.dh_lev, prec=prec, gamma=gamma)
    o2 = S.srhd_fluid_step(_g(pad_o), _g(dt_o), g.dh_lev, prec=prec, gamma=gamma,
                           sched=S.Sched(0, 1, DEV, occupancy=2))
    torch.cuda.synchronize()
    assert torch.equal(out, o2)
    e = step_errors(out.cpu().numpy(), ref)
    with O.eos(gamma):
        bound = step_bound(kappa_tile_padded(pad_o))
    ep = patch_errors(out.cpu().numpy(), ref)
    print("Gamma 5/3 prec %d: %s, largest error / bound %.3f" % (prec, e, (ep / bound).max()))
    assert np.all(ep <= bound), e


def test_multistep_blast_with_retries(S):
    gamma = 4.0 / 3.0
    g = W.blast(64, seed=3)
    co = _cons(g, gamma)
    cg = _g(co)
    nb = _g(g.neighbor)
    retries = 0
    for step in range(4):
        with O.eos(gamma):
            dt_o, _, _ = O.cfl_dt(co, None, g.dh_lev, 0.5)
            pad_o = O.fill_ghosts(co, g.neighbor, 3)
            co, cnt = O.fluid_step(pad_o, dt_o, g.dh_lev)
        dt_g = S.srhd_cfl_dt(cg, g.dh_lev, 0.5, gamma=gamma)
        pad = S.srhd_fill_ghosts(cg, nb, 3)
        st = S.new_stats(DEV)
        cg = S.srhd_fluid_step(pad, dt_g, g.dh_lev, stats=st, gamma=gamma)
        torch.cuda.synchronize()
        sd = S.stats_dict(st)
        assert abs(dt_g.cpu().item() / dt_o[0] - 1) < 1e-12
        assert sd["n_retry"] == cnt[3] and sd["n_unphysical"] == cnt[0], (step, sd, cnt)
        retries += cnt[3]
        e = step_errors(cg.cpu().numpy(), co)
        assert max(e.values()) <= 1e-10 * (step + 1), (step, e)
    print("Gamma 4/3 blast 64^3: %d patch retries over 4 steps" % retries)


def test_refused_combinations(S):
    g = W.blast(16, seed=3)
    cons = _cons(g, 5 / 3)
    pad = S.srhd_fill_ghosts(_g(cons), _g(g.neighbor), 3)
    dt = torch.full((1,), 1e-4, dtype=torch.float64, device=DEV)
    for kw in ({"integrator": S.VL}, {"energy": S.ENERGY_TOTAL}):
        with pytest.raises(S.SrhdError) as ei:
            S.srhd_fluid_step(pad, dt, g.dh_lev, gamma=5 / 3, **kw)
        assert ei.value.code == S.EUNSUPPORTED
    prims, smax = S.srhd_grid_prims(_g(cons))
    with pytest.raises(S.SrhdError) as ei:
        S.srhd_fluid_step_grid(_g(cons), prims, _g(g.neighbor), g.dh_lev, smax_in=smax,
                               gamma=5 / 3)
    assert ei.value.code == S.EUNSUPPORTED
    assert S.srhd_step_occupancy(0, gamma=5 / 3) >= 1
    assert S.srhd_step_occupancy(1, occupancy=2, gamma=5 / 3) >= 2
