"""Edge cases of the step entry points on the GPU: empty patch lists, lists shorter than the
eight XCD ranges of the persistent schedule, and a single patch; for the MUSCL-Hancock and the VL
integrators."""
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
def tube(S):
    g = W.shock_tube_32()
    c = torch.from_numpy(oracle_cons(g)).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    dt = S.srhd_cfl_dt(c, g.dh_lev)
    pad = S.srhd_fill_ghosts(c, nb)
    return g, c, nb, dt, pad


def test_empty_patch_lists(S, tube):
    g, c, nb, dt, pad = tube
    out = S.srhd_fluid_step(pad[:0], dt, g.dh_lev)
    assert out.shape[0] == 0
    out = S.srhd_fluid_step(pad[:0], dt, g.dh_lev, sched=S.Sched(64, 2, DEV))
    assert out.shape[0] == 0
    for prec in (0, 1, 2):
        prims, smax = S.srhd_grid_prims(c[:0], prec=prec)
        cons_out, prims_out, smax_out = S.srhd_fluid_step_grid(c[:0], prims, nb[:0], g.dh_lev,
                                                               smax_in=smax, prec=prec)
        torch.cuda.synchronize()
        assert cons_out.shape[0] == 0 and int(smax.item()) == 0 and int(smax_out.item()) == 0


@pytest.mark.parametrize("n", [1, 3, 9])
@pytest.mark.parametrize("groups,chunk", [(64, 1), (7, 4), (1, 64)])
def test_short_lists_under_the_persistent_schedule(S, tube, n, groups, chunk):
    # fewer patches than XCD ranges: some ranges are empty and every workgroup must still leave
    g, c, nb, dt, pad = tube
    for prec in (0, 1):
        ref = S.srhd_fluid_step(pad[:n], dt, g.dh_lev, prec=prec)
        out = S.srhd_fluid_step(pad[:n], dt, g.dh_lev, prec=prec, sched=S.Sched(groups, chunk, DEV))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, prec)


def test_single_patch_matches_its_place_in_the_list(S, tube):
    # a patch stepped alone (its padded copy) equals the same patch stepped in the full list
    g, c, nb, dt, pad = tube
    full = S.srhd_fluid_step(pad, dt, g.dh_lev)
    for p in (0, 17, 63):
        one = S.srhd_fluid_step(pad[p:p + 1].clone(), dt, g.dh_lev)
        torch.cuda.synchronize()
        assert torch.equal(one[0], full[p]), p


def test_vl_empty_and_short_lists(S, tube):
    g, c, nb, dt, pad = tube
    out = S.srhd_fluid_step(pad[:0], dt, g.dh_lev, integrator=S.VL)
    assert out.shape[0] == 0
    for prec in (0, 1, 2):
        prims, smax = S.srhd_grid_prims(c[:0], prec=prec)
        co, po, so = S.srhd_fluid_step_grid(c[:0], prims, nb[:0], g.dh_lev, smax_in=smax, prec=prec,
                                            integrator=S.VL)
        torch.cuda.synchronize()
        assert co.shape[0] == 0 and int(so.item()) == 0
    # the first n patches, each its own periodic neighbour in every slot, under the persistent
    # schedule (fewer patches than XCD ranges): both layouts give the one-per-patch padded step
    for n in (1, 3, 9):
        nbn = torch.arange(n, dtype=torch.int32, device=DEV)[:, None].repeat(1, 27).contiguous()
        cn = c[:n].contiguous()
        padn = S.srhd_fill_ghosts(cn, nbn, 3)
        dtn = S.srhd_cfl_dt(cn, g.dh_lev)
        for prec in (0, 1):
            ref = S.srhd_fluid_step(padn, dtn, g.dh_lev, prec=prec, integrator=S.VL)
            prims, _ = S.srhd_grid_prims(cn, prec=prec)
            for groups, chunk in ((64, 1), (7, 4), (1, 64)):
                sch = S.Sched(groups, chunk, DEV)
                o1 = S.srhd_fluid_step(padn, dtn, g.dh_lev, prec=prec, integrator=S.VL, sched=sch)
                o2 = S.srhd_fluid_step_grid(cn, prims, nbn, g.dh_lev, dt_lev=dtn, prec=prec,
                                            integrator=S.VL, sched=sch)[0]
                torch.cuda.synchronize()
                assert bool(torch.isfinite(ref).all()), (n, prec)
                assert torch.equal(o1, ref) and torch.equal(o2, ref), (n, prec, groups, chunk)
