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
    # the 64^3 blast (512 patches) retries patches, so the work per patch is uneven
    g = W.blast(64, seed=3, order="morton")
    c = torch.from_numpy(oracle_cons(g)).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    dt = S.srhd_cfl_dt(c, g.dh_lev)
    pad = S.srhd_fill_ghosts(c, nb)
    return g, c, nb, dt, pad


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
    assert a == b and a["n_retry"] > 0


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
    for n in (512, 77):
        ref = S.srhd_fluid_step(pad[:n], dt, g.dh_lev)
        out = S.srhd_fluid_step(pad[:n], dt, g.dh_lev, sched=sch)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), n


def test_autotuner_picks_a_measured_candidate(S, blast):
    g, c, nb, dt, pad = blast
    occ = S.srhd_step_occupancy(1, S.GUESS_ANALYTIC, False)
    assert 1 <= occ <= 8
    sch, table = S.srhd_autotune_step(pad, dt, g.dh_lev, prec=1, reps=2)
    assert len(table) == 10 and table[0][:2] == (0, 1)
    assert all(t[2] > 0 for t in table)
    best = min(table, key=lambda t: t[2])
    assert (sch.groups, sch.chunk) == best[:2]
    ref = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1)
    out = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=1, sched=sch)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    print("occupancy %d; autotune table %s -> %s" % (occ, table, sch))
