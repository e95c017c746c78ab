"""The learned-guess split, through the C ABI: the kernel without the network steps every patch
and lists the patches whose tile holds a cell with L above the network's gate; the learned kernel
steps those in a second launch.  On the 64^3 blast with the trained network (gate 0.1), one step
in both layouts and every precision mode: the listed patches are exactly those whose stencil
reads such a cell (host count), their results equal the single-launch learned step's bit for bit,
the other patches' equal it to the Newton tolerance, and the step matches the oracle within the
parity bounds (FP64 1e-10; FP32 bulk (C_KAPPA kappa_tile + C_FLUX) u32)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import (kappa_tile_padded, oracle_cons, patch_errors, soa, step_bound,
                          step_errors, tile_max)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


@pytest.fixture(scope="module")
def case(S):
    from paper_2012_11130_amd import mlp_train
    mlp = mlp_train.load(device=DEV)
    assert mlp is not None and mlp.gate > 0
    g = W.blast(64, seed=3, order="morton")
    cons = oracle_cons(g)
    dt, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad = O.fill_ghosts(cons, g.neighbor, 3)
    ref, _ = O.fluid_step(pad, dt, g.dh_lev)
    # host: the patches whose step reads a cell with L above the gate
    L = O.L_batch(soa(cons)).reshape(g.n_patch, 8, 8, 8)
    listed = tile_max(L, g.neighbor) > mlp.gate
    return g, cons, dt, pad, ref, mlp, listed


def _run(S, g, cons, dt, pad, prec, guess, layout, split, stats):
    P = g.n_patch
    defer = S.defer_workspace(P, DEV)
    dtg = torch.from_numpy(dt).to(DEV)
    if layout == "padded":
        out = S.srhd_fluid_step(torch.from_numpy(pad).to(DEV), dtg, g.dh_lev, prec=prec,
                                guess=guess, stats=stats, learned_split=split, defer=defer)
    else:
        c = torch.from_numpy(cons).to(DEV)
        prims, smax = S.srhd_grid_prims(c, prec=prec, guess=guess)
        out, _, _ = S.srhd_fluid_step_grid(c, prims, torch.from_numpy(g.neighbor).to(DEV),
                                           g.dh_lev, dt_lev=dtg, prec=prec, guess=guess,
                                           stats=stats, learned_split=split, defer=defer)
    torch.cuda.synchronize()
    d = defer.cpu().numpy()
    n = int(d[P + 2]) if split else 0
    return out.cpu().numpy(), np.sort(d[P + 4:P + 4 + n])


@pytest.mark.parametrize("layout", ["grid", "padded"])
@pytest.mark.parametrize("prec", [1, 0, 2])
def test_split_equals_single_launch(S, case, layout, prec):
    g, cons, dt, pad, ref, mlp, listed = case
    st1, st2 = S.new_stats(DEV), S.new_stats(DEV)
    one, _ = _run(S, g, cons, dt, pad, prec, mlp.guess(), layout, False, st1)
    two, idx = _run(S, g, cons, dt, pad, prec, mlp.guess(), layout, True, st2)
    s1, s2 = S.stats_dict(st1), S.stats_dict(st2)
    print("%s prec %d: listed %d patches (host %d); network lanes %d (single launch %d)"
          % (layout, prec, s2["n_learned_patch"], listed.sum(), s2["n_mlp"], s1["n_mlp"]))
    assert s2["n_learned_patch"] == listed.sum() == idx.size and 0 < idx.size < g.n_patch
    assert np.array_equal(idx, np.flatnonzero(listed))
    assert s2["n_mlp"] > 0 and s1["n_learned_patch"] == 0
    assert np.array_equal(two[idx], one[idx])
    e = patch_errors(two, one)
    assert e.max() <= (1e-12 if prec == 0 else step_bound(1.0)), e.max()
    eo = patch_errors(two, ref)
    if prec == 0:
        assert max(step_errors(two, ref).values()) <= 1e-10
    else:
        assert np.all(eo <= step_bound(kappa_tile_padded(pad)))
