"""GPU parity of the VL predictor-corrector step (srhd_fluid_step with integrator = VL) against
the oracle's VL step, through the C ABI: one FP64 step within 1e-10 (HLLC and HLLE) on a shock
tube and the 64^3 blast, multi-step runs with limiter retries on both sides, the persistent
schedule bit for bit, the FP32-bulk modes within their stated errors, and sampled patches of the
full-size 256^3 blast in the benchmark's launch configuration."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import kappa_tile_padded, patch_errors, step_bound
from tests.parity import oracle_cons, step_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _pair(S, g, cons, prec=0, riemann=0, sched=None):
    dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad_o = O.fill_ghosts(cons, g.neighbor, 3)
    ref, cnt = O.fluid_step(pad_o, dt_o, g.dh_lev, solver=riemann, integrator=1)
    pad = S.srhd_fill_ghosts(_gpu(cons), _gpu(g.neighbor), 3)
    st = S.new_stats(DEV)
    out = S.srhd_fluid_step(pad, _gpu(dt_o), g.dh_lev, riemann=riemann, prec=prec, stats=st,
                            integrator=S.VL, sched=sched)
    torch.cuda.synchronize()
    return ref, cnt, out, S.stats_dict(st), pad, dt_o


@pytest.mark.parametrize("riemann", [0, 1])
def test_shock_tube_one_step_fp64(S, riemann):
    g = W.riemann_1d(64, (1.0, 0.0, 0.0, 0.0, 1e3), (0.5, 0.3, 0.0, 0.0, 1e-6))
    ref, cnt, out, sd, _, _ = _pair(S, g, oracle_cons(g), riemann=riemann)
    e = step_errors(out.cpu().numpy(), ref)
    print("VL shock tube (riemann %d): %s, stats %s" % (riemann, e, sd))
    assert max(e.values()) <= 1e-10, e


@pytest.mark.parametrize("riemann", [0, 1])
def test_blast_one_step_fp64_and_schedules(S, riemann):
    g = W.blast(64, seed=3)
    cons = oracle_cons(g)
    ref, cnt, out, sd, pad, dt_o = _pair(S, g, cons, riemann=riemann)
    e = step_errors(out.cpu().numpy(), ref)
    print("VL blast 64^3 (riemann %d): %s, stats %s, oracle counts %s" % (riemann, e, sd, cnt))
    assert max(e.values()) <= 1e-10, e
    assert sd["n_unphysical"] == 0 and sd["n_retry"] == cnt[3]
    for sch in (S.Sched(7, 3, DEV), S.Sched(1024, 1, DEV)):
        o = S.srhd_fluid_step(pad, _gpu(dt_o), g.dh_lev, riemann=riemann, integrator=S.VL,
                              sched=sch)
        torch.cuda.synchronize()
        assert torch.equal(o, out), sch


def test_blast_multistep_fp64_with_retries(S):
    g = W.blast(64, seed=3)
    co = oracle_cons(g)
    cg = _gpu(co)
    nb = _gpu(g.neighbor)
    retries = 0
    for step in range(6):
        dt_o, _, _ = O.cfl_dt(co, None, g.dh_lev, 0.5)
        pad_o = O.fill_ghosts(co, g.neighbor, 3)
        co, cnt = O.fluid_step(pad_o, dt_o, g.dh_lev, integrator=1)
        dt_g = S.srhd_cfl_dt(cg, g.dh_lev, 0.5)
        pad = S.srhd_fill_ghosts(cg, nb, 3)
        st = S.new_stats(DEV)
        cg = S.srhd_fluid_step(pad, dt_g, g.dh_lev, stats=st, integrator=S.VL)
        torch.cuda.synchronize()
        assert abs(dt_g.cpu().item() / dt_o[0] - 1) < 1e-12
        sd = S.stats_dict(st)
        assert sd["n_unphysical"] == cnt[0] and sd["n_retry"] == cnt[3], (step, sd, cnt)
        retries += cnt[3]
        e = step_errors(cg.cpu().numpy(), co)
        assert max(e.values()) <= 1e-10 * (step + 1), (step, e)
    print("VL blast 64^3: %d patch retries over 6 steps" % retries)


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_bulk_error_is_stated(S, prec):
    for g in (W.riemann_1d(64, (1.0, 0.0, 0.0, 0.0, 1e3), (0.5, 0.3, 0.0, 0.0, 1e-6)),
              W.blast(32, seed=3)):
        cons = oracle_cons(g)
        ref, cnt, out, sd, pad, dt_o = _pair(S, g, cons, prec=prec)
        o2 = S.srhd_fluid_step(pad, _gpu(dt_o), g.dh_lev, prec=prec, integrator=S.VL,
                               sched=S.Sched(0, 1, DEV, occupancy=2))
        torch.cuda.synchronize()
        assert torch.equal(o2, out)
        e = step_errors(out.cpu().numpy(), ref)
        # per patch (C_KAPPA kappa_tile + C_FLUX) u32 (Eq. 20), kappa over the whole padded input
        bound = step_bound(kappa_tile_padded(pad.cpu().numpy(), whole=True))
        ep = patch_errors(out.cpu().numpy(), ref)
        print("VL prec %d %s: %s, largest error / bound %.3f" % (prec, g.name, e, (ep / bound).max()))
        assert np.all(ep <= bound), e


def test_occupancy_and_autotune(S):
    for prec in (0, 1, 2):
        assert S.srhd_step_occupancy(prec, integrator=S.VL) >= 1
    assert S.srhd_step_occupancy(1, occupancy=2, integrator=S.VL) >= 2
    g = W.blast(64, seed=3)
    cons = oracle_cons(g)
    pad = S.srhd_fill_ghosts(_gpu(cons), _gpu(g.neighbor), 3)
    dt = S.srhd_cfl_dt(_gpu(cons), g.dh_lev)
    sch, table = S.srhd_autotune_step(pad, dt, g.dh_lev, prec=1, reps=1, integrator=S.VL)
    ref = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, integrator=S.VL)
    out = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, integrator=S.VL, sched=sch)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert len(table) == 20
    print("VL mixed autotune: %s -> %s" % (table, sch))


def test_full_size_blast_sampled_patches(S):
    g = W.blast(256, seed=1003)
    cons = oracle_cons(g)
    c = _gpu(cons)
    dt_g = S.srhd_cfl_dt(c, g.dh_lev)
    pad = S.srhd_fill_ghosts(c, _gpu(g.neighbor))
    out = S.srhd_fluid_step(pad, dt_g, g.dh_lev, integrator=S.VL)
    torch.cuda.synchronize()
    dt = dt_g.cpu().numpy()
    lab = g.extra["labels"].reshape(g.n_patch, -1).any(axis=1)
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([np.nonzero(lab)[0], rng.choice(g.n_patch, 200, replace=False)]))
    pad_o = O.fill_ghosts(cons, g.neighbor[sample], 3)
    ref, cnt = O.fluid_step(pad_o, dt, g.dh_lev, integrator=1)
    e = step_errors(out.cpu().numpy()[sample], ref)
    print("VL 256^3 sampled (%d patches): %s" % (sample.size, e))
    assert max(e.values()) <= 1e-10, e


def test_zero_limiter_and_the_last_resort(S):
    # theta = 0 from the start: the Godunov step (no predictor) against the oracle
    g = W.blast(64, seed=3)
    cons = oracle_cons(g)
    dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad_o = O.fill_ghosts(cons, g.neighbor, 3)
    ref, cnt = O.fluid_step(pad_o, dt_o, g.dh_lev, theta=0.0, integrator=1)
    out = S.srhd_fluid_step(_gpu(pad_o), _gpu(dt_o), g.dh_lev, theta=0.0, integrator=S.VL)
    torch.cuda.synchronize()
    e = step_errors(out.cpu().numpy(), ref)
    assert max(e.values()) <= 1e-10, e
    # 12 steps of the 128^3 blast: every output cell is physical in FP64 and with an FP32 bulk
    # (predictor fallbacks and, as the last resort, the Godunov step)
    g = W.blast(128, seed=3, order="morton")
    c0 = _gpu(oracle_cons(g))
    nb = _gpu(g.neighbor)
    for prec in (0, 1):
        c = c0
        bad = 0
        for k in range(12):
            dt = S.srhd_cfl_dt(c, g.dh_lev)
            pad = S.srhd_fill_ghosts(c, nb)
            st = S.new_stats(DEV)
            c = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st, integrator=S.VL)
            sd = S.stats_dict(st)
            bad += sd["n_unphysical"]
        print("VL prec %d 128^3, 12 steps: %d unphysical output cells; last stats %s" % (prec, bad, sd))
        assert bad == 0 and bool(torch.isfinite(c).all()), prec
