"""Launch schedules of the step: the persistent work-queue grid and the autotuner change where
patches run, never what they compute -- outputs and counters must equal the one-workgroup-per-patch
launch bit for bit, for grids smaller and larger than the patch count and for every chunk size."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.parity import oracle_cons

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


@pytest.fixture(scope="module")
def blast(S):
    # a state of the 128^3 blast (4,096 patches) at the first step that retries patches, so
    # the work per patch is uneven: advance with the one-workgroup-per-patch launch until then
    g = W.blast(128, seed=3, order="morton")
    c = torch.from_numpy(oracle_cons(g)).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    for k in range(12):
        dt = S.srhd_cfl_dt(c, g.dh_lev)
        pad = S.srhd_fill_ghosts(c, nb)
        st = S.new_stats(DEV)
        nxt = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, stats=st)
        if S.stats_dict(st)["n_retry"] > 0:
            print("blast 128^3: step %d retries %d patches" % (k, S.stats_dict(st)["n_retry"]))
            return g, c, nb, dt, pad
        c = nxt
    pytest.fail("no limiter retry within 12 steps of the 128^3 blast")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("groups,chunk", [(1, 1), (7, 3), (256, 1), (600, 64), (2048, 2)])
def test_persistent_padded_step_is_bitwise_identical(S, blast, prec, groups, chunk):
    g, c, nb, dt, pad = blast
    st0, st1 = S.new_stats(DEV), S.new_stats(DEV)
    ref = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st0)
    out = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st1,
                            sched=S.Sched(groups, chunk, DEV))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    a, b = S.stats_dict(st0), S.stats_dict(st1)
    assert a == b
    if prec == 1:
        assert a["n_retry"] > 0


@pytest.mark.parametrize("groups,chunk", [(5, 1), (512, 4)])
def test_persistent_grid_step_is_bitwise_identical(S, blast, groups, chunk):
    g, c, nb, dt, pad = blast
    for prec in (0, 1):
        prims, smax = S.srhd_grid_prims(c, prec=prec)
        d0 = torch.empty(1, dtype=torch.float64, device=DEV)
        d1 = torch.empty(1, dtype=torch.float64, device=DEV)
        r = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec, dt_used=d0)
        o = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec, dt_used=d1,
                                   sched=S.Sched(groups, chunk, DEV))
        torch.cuda.synchronize()
        for x, y in zip(r, o):
            assert torch.equal(x, y)
        assert torch.equal(d0, d1)


def test_queue_is_reset_between_calls(S, blast):
    # the same Sched (and queue) used for consecutive calls, the second on fewer patches
    g, c, nb, dt, pad = blast
    sch = S.Sched(300, 2, DEV)
    for n in (4096, 77):
        ref = S.srhd_fluid_step(pad[:n], dt, g.dh_lev)
        out = S.srhd_fluid_step(pad[:n], dt, g.dh_lev, sched=sch)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), n


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("gather", [False, True])
def test_two_workgroup_variant_is_bitwise_identical(S, blast, gather, prec):
    # the kernel compiled for two workgroups per CU (FP32 bulk, analytic guess)
    g, c, nb, dt, pad = blast
    o0 = S.srhd_step_occupancy(prec, S.GUESS_ANALYTIC, gather, 0)
    o2 = S.srhd_step_occupancy(prec, S.GUESS_ANALYTIC, gather, 2)
    print("workgroups per CU (gather=%s): natural %d, two-workgroup variant %d" % (gather, o0, o2))
    assert o2 >= 2
    for sch in (S.Sched(0, 1, DEV, occupancy=2), S.Sched(1024, 2, DEV, occupancy=2)):
        if gather:
            prims, smax = S.srhd_grid_prims(c, prec=prec)
            st0, st1 = S.new_stats(DEV), S.new_stats(DEV)
            r = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec, stats=st0)
            o = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec, stats=st1,
                                       sched=sch)
            torch.cuda.synchronize()
            for x, y in zip(r, o):
                assert torch.equal(x, y)
        else:
            st0, st1 = S.new_stats(DEV), S.new_stats(DEV)
            r = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st0)
            o = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st1, sched=sch)
            torch.cuda.synchronize()
            assert torch.equal(o, r)
        assert S.stats_dict(st0) == S.stats_dict(st1)


def test_autotuner_picks_a_measured_candidate(S, blast):
    g, c, nb, dt, pad = blast
    occ = S.srhd_step_occupancy(1, S.GUESS_ANALYTIC, False)
    assert 1 <= occ <= 8
    for prec, n in ((1, 20), (0, 10)):
        sch, table = S.srhd_autotune_step(pad, dt, g.dh_lev, prec=prec, reps=2)
        assert len(table) == n and table[0][:3] == (0, 1, 0)
        assert all(t[3] > 0 for t in table)
        best = min(table, key=lambda t: t[3])
        assert (sch.groups, sch.chunk, sch.occupancy) == best[:3]
        ref = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec)
        out = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, sched=sch)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        print("prec %d: autotune table %s -> %s" % (prec, table, sch))


def test_grid_autotuner(S, blast):
    g, c, nb, dt, pad = blast
    prims, smax = S.srhd_grid_prims(c, prec=1)
    sch, table = S.srhd_autotune_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=1, reps=2)
    assert len(table) == 20
    r = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=1)
    o = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=1, sched=sch)
    torch.cuda.synchronize()
    for x, y in zip(r, o):
        assert torch.equal(x, y)
    print("grid autotune table %s -> %s" % (table, sch))


@pytest.mark.parametrize("prec", [1, 2])
def test_learned_guess_under_every_schedule_is_bitwise_identical(S, blast, prec):
    # the trained, gated network: the register variants (which spill around its evaluation)
    # and the persistent grid leave outputs and counters unchanged
    from paper_2012_11130_amd import mlp_train
    mlp = mlp_train.load(device=DEV)
    assert mlp is not None
    g, c, nb, dt, pad = blast
    prims, smax = S.srhd_grid_prims(c, prec=prec, guess=mlp.guess())
    st0 = S.new_stats(DEV)
    ref = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec,
                                 guess=mlp.guess(), stats=st0)
    torch.cuda.synchronize()
    a = S.stats_dict(st0)
    assert a["n_mlp"] > 0
    for sch in (S.Sched(0, 1, DEV, occupancy=2), S.Sched(1024, 2, DEV, occupancy=2),
                S.Sched(512, 4, DEV)):
        st1 = S.new_stats(DEV)
        out = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=prec,
                                     guess=mlp.guess(), stats=st1, sched=sch)
        torch.cuda.synchronize()
        for x, y in zip(ref, out):
            assert torch.equal(x, y), sch
        assert S.stats_dict(st1) == a, sch
