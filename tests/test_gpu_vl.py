"""GPU parity of the VL predictor-corrector step (srhd_fluid_step and srhd_fluid_step_grid with
integrator = VL) against the oracle's VL step, through the C ABI: one FP64 step within 1e-10
(HLLC and HLLE) on a shock tube and the 64^3 blast, multi-step runs with limiter retries on both
sides, the persistent schedule bit for bit, the FP32-bulk modes within their stated errors, and
sampled patches of the full-size 256^3 blast; the gather layout bit for bit against the padded
one in every precision mode and schedule, its fused S_max, a five-step FP64 chain against the
oracle, and the 256^3 blast in the benchmark's launch configuration."""
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


# ------------------------------------------------------------------------------ gather layout
def _grid_vl(S, g, cons, prec, sched=None, dt=None, stats=None):
    c = _gpu(cons)
    nb = _gpu(g.neighbor)
    prims, smax = S.srhd_grid_prims(c, prec=prec)
    dt_used = torch.empty(len(g.dh_lev), dtype=torch.float64, device=DEV)
    out, po, so = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, dt_lev=dt,
                                         prec=prec, integrator=S.VL, sched=sched,
                                         dt_used=dt_used, stats=stats)
    return out, po, so, dt_used


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_grid_vl_equals_padded_vl_bitwise(S, prec):
    # The gather layout reads the primitives that srhd_grid_prims stored -- the inversion that
    # the padded kernel's phase A runs -- and U^n from the neighbours' interiors: for the same dt
    # the output is the padded step's, bit for bit, in every precision mode (outflow and periodic
    # blocks, patches in Morton order), under every schedule, and the primitives and S_max handed
    # to the next step equal a fresh srhd_grid_prims of the output.
    for g in (W.shock_tube_32(), W.blast(64, seed=3, order="morton")):
        cons = oracle_cons(g)
        c = _gpu(cons)
        nb = _gpu(g.neighbor)
        dt = S.srhd_cfl_dt(c, g.dh_lev)
        ref = S.srhd_fluid_step(S.srhd_fill_ghosts(c, nb, 3), dt, g.dh_lev, prec=prec,
                                integrator=S.VL)
        out, po, so, dt_used = _grid_vl(S, g, cons, prec, dt=dt)
        torch.cuda.synchronize()
        assert torch.equal(dt_used, dt), g.name
        assert torch.equal(out, ref), (g.name, prec)
        p2, s2 = S.srhd_grid_prims(out, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(p2, po) and torch.equal(s2, so), g.name
        scheds = [S.Sched(7, 3, DEV), S.Sched(1024, 1, DEV)]
        if prec != 0:
            scheds += [S.Sched(0, 1, DEV, occupancy=2), S.Sched(512, 2, DEV, occupancy=2)]
        for sch in scheds:
            o2, p3, s3, _ = _grid_vl(S, g, cons, prec, sched=sch, dt=dt)
            torch.cuda.synchronize()
            assert torch.equal(o2, out) and torch.equal(p3, po) and torch.equal(s3, so), (g.name, sch)
        # the fused CFL: in FP64 the S_max of srhd_grid_prims gives the CFL kernel's dt bit for bit
        if prec == 0:
            o3, _, _, dt3 = _grid_vl(S, g, cons, prec)
            torch.cuda.synchronize()
            assert torch.equal(dt3, dt) and torch.equal(o3, out), g.name


def test_grid_vl_chain_matches_oracle(S):
    # 64^3 blast in Morton order, 5 FP64 steps chained through the output's primitives and S_max
    # (one kernel per step): each state against the oracle's CFL + ghost fill + VL step from its
    # own state, with the oracle's limiter retries counted alike.
    g = W.blast(64, seed=3, order="morton")
    co = oracle_cons(g)
    c = _gpu(co)
    nb = _gpu(g.neighbor)
    prims, smax = S.srhd_grid_prims(c, prec=0)
    st = S.new_stats(DEV)
    retries = 0
    for k in range(5):
        c, prims, smax = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=0,
                                                integrator=S.VL, stats=st)
        dt_o, _, _ = O.cfl_dt(co, None, g.dh_lev, 0.5)
        co, cnt = O.fluid_step(O.fill_ghosts(co, g.neighbor, 3), dt_o, g.dh_lev, integrator=1)
        retries += cnt[3]
        e = step_errors(c.cpu().numpy(), co)
        assert max(e.values()) <= 1e-10 * (k + 1), (k, e)
    sd = S.stats_dict(st)
    print("VL grid chain 64^3: %d patch retries over 5 steps; stats %s" % (retries, sd))
    assert sd["n_retry"] == retries and sd["n_unphysical"] == 0


def test_grid_vl_full_size_blast(S):
    # the 256^3 blast in the benchmark's launch configuration (gather layout, fused CFL, the
    # persistent schedule and the one-workgroup-per-patch launch): FP64 against the oracle on
    # sampled patches, and both layouts bit for bit in FP64 and with the FP32 bulk
    g = W.blast(256, seed=1003, order="morton")
    cons = oracle_cons(g)
    c = _gpu(cons)
    nb = _gpu(g.neighbor)
    dt_g = S.srhd_cfl_dt(c, g.dh_lev)
    pad = S.srhd_fill_ghosts(c, nb, 3)
    for prec in (0, 1):
        ref = S.srhd_fluid_step(pad, dt_g, g.dh_lev, prec=prec, integrator=S.VL)
        for sch in (None, S.Sched(2 * 256, 1, DEV)):
            out, _, _, dt_used = _grid_vl(S, g, cons, prec, sched=sch)
            torch.cuda.synchronize()
            if prec == 0:
                assert torch.equal(dt_used, dt_g)
            else:
                assert abs(dt_used.item() / dt_g.item() - 1) < 1e-6
            o = _grid_vl(S, g, cons, prec, sched=sch, dt=dt_g)[0]
            torch.cuda.synchronize()
            assert torch.equal(o, ref), (prec, sch)
            del o
        if prec == 0:
            lab = g.extra["labels"].reshape(g.n_patch, -1).any(axis=1)
            rng = np.random.default_rng(1)
            sample = np.unique(np.concatenate([np.nonzero(lab)[0][:150],
                                               rng.choice(g.n_patch, 150, replace=False)]))
            r, _ = O.fluid_step(O.fill_ghosts(cons, g.neighbor[sample], 3), dt_g.cpu().numpy(),
                                g.dh_lev, integrator=1)
            e = step_errors(out.cpu().numpy()[sample], r)
            print("VL grid 256^3 sampled (%d patches): %s" % (sample.size, e))
            assert max(e.values()) <= 1e-10, e
        del ref, out
    del pad
