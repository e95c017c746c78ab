"""The learned-guess split, through the C ABI: the kernel without the network steps every patch
and lists the patches whose tile holds a cell with L above the network's gate; the learned kernel
steps those in a second launch.  On the 64^3 blast with the trained network (gate 0.1), one step
in both layouts and every precision mode: the listed patches are exactly those whose stencil
reads such a cell (host count), their results equal the single-launch learned step's bit for bit,
the other patches' equal it to the Newton tolerance, and the step matches the oracle within the
parity bounds (FP64 1e-10; FP32 bulk (C_KAPPA kappa_tile + C_FLUX) u32).

With the gather layout's network masks (per patch, the regions -- the patch, its two lowest or
highest layers along each axis -- holding a cell with L > gate) the list is formed before the step
from the masks of each patch's 27 neighbours, and the learned kernel runs on the library's second
stream beside the kernel without the network: the masks that srhd_grid_prims and the step write
agree with the oracle's L of the same states, the listed patches are those the masks select, and
the same equalities and bounds hold."""
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


_SEL = (slice(0, 2), slice(0, 8), slice(6, 8))          # r = -1, 0, +1 along one axis


def _mask_rule(L, gate):
    """Per patch and region bit (rz + 1) 9 + (ry + 1) 3 + (rx + 1): (the oracle's L puts a cell of
    the region above the gate, no cell is above it but one lies within 1e-9 of the gate -- there
    the device's L and the oracle's may round to either side).  L is [P][z][y][x]."""
    P = L.shape[0]
    above = np.zeros((P, 27), bool)
    near = np.zeros((P, 27), bool)
    for rz in range(3):
        for ry in range(3):
            for rx in range(3):
                b = rz * 9 + ry * 3 + rx
                sub = L[:, _SEL[rz], _SEL[ry], _SEL[rx]].reshape(P, -1)
                above[:, b] = (sub > gate * (1 + 1e-9)).any(axis=1)
                near[:, b] = (np.abs(sub / gate - 1) <= 1e-9).any(axis=1)
    return above, near & ~above


def _masks_host(m, P):
    """[P][27] booleans of int32 device masks."""
    v = m.cpu().numpy().astype(np.int64)[:P]
    return ((v[:, None] >> np.arange(27)[None, :]) & 1).astype(bool)


def _listed_by_masks(mask, neighbor):
    """Patches whose tile reaches a set region: neighbour k (offset order of srhd_fill_ghosts)
    contributes its region next to the patch, bit 26 - k."""
    P = neighbor.shape[0]
    out = np.zeros(P, bool)
    for k in range(27):
        q = neighbor[:, k]
        ok = q >= 0
        out[ok] |= mask[q[ok], 26 - k]
    return out


@pytest.mark.parametrize("prec", [1, 0, 2])
def test_network_masks_concurrent_split(S, case, prec):
    g, cons, dt, pad, ref, mlp, listed = case
    P = g.n_patch
    guess = mlp.guess()
    c = torch.from_numpy(cons).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    dtg = torch.from_numpy(dt).to(DEV)
    mask = S.new_net_mask(P, DEV)
    prims, smax = S.srhd_grid_prims(c, prec=prec, guess=guess, net_mask=mask)
    torch.cuda.synchronize()
    have = _masks_host(mask, P)
    above, near = _mask_rule(O.L_batch(soa(cons)).reshape(P, 8, 8, 8), mlp.gate)
    assert np.array_equal(have[~near], above[~near]) and have.any()
    want = _listed_by_masks(have, g.neighbor.reshape(P, 27))
    st1, st2 = S.new_stats(DEV), S.new_stats(DEV)
    one, _, _ = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, dt_lev=dtg, prec=prec, guess=guess,
                                       stats=st1, learned_split=False)
    defer = S.defer_workspace(P, DEV)
    out_mask = S.new_net_mask(P, DEV)
    out_mask.fill_(-1)                         # every patch's mask is written by the step
    two, _, _ = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, dt_lev=dtg, prec=prec, guess=guess,
                                       stats=st2, learned_split=True, defer=defer, net_in=mask,
                                       net_out=out_mask)
    torch.cuda.synchronize()
    s2 = S.stats_dict(st2)
    d = defer.cpu().numpy()
    n = int(d[P + 2])
    idx = np.sort(d[P + 4:P + 4 + n])
    print("prec %d: patches with a set region %d, listed %d (host %d, tile rule %d); network "
          "lanes %d" % (prec, have.any(axis=1).sum(), n, want.sum(), listed.sum(), s2["n_mlp"]))
    assert s2["n_learned_patch"] == want.sum() == n and np.array_equal(idx, np.flatnonzero(want))
    assert np.all(want[listed])                # every tile the in-kernel rule lists
    one, two = one.cpu().numpy(), two.cpu().numpy()
    assert np.array_equal(two[idx], one[idx])
    e = patch_errors(two, one)
    assert e.max() <= (1e-12 if prec == 0 else step_bound(1.0)), e.max()
    if prec == 0:
        assert max(step_errors(two, ref).values()) <= 1e-10
    else:
        assert np.all(patch_errors(two, ref) <= step_bound(kappa_tile_padded(pad)))
    # the output's masks follow the oracle's L of the output state
    got = _masks_host(out_mask, P)
    above, near = _mask_rule(O.L_batch(soa(two)).reshape(P, 8, 8, 8), mlp.gate)
    assert np.array_equal(got[~near], above[~near])
    # a chain's second step from those masks gives the single launch's listed results again
    t = torch.from_numpy(two).to(DEV)
    prims2 = S.srhd_grid_prims(t, prec=prec, guess=guess)[0]
    a, _, _ = S.srhd_fluid_step_grid(t, prims2, nb, g.dh_lev, dt_lev=dtg, prec=prec, guess=guess,
                                     learned_split=False)
    b, _, _ = S.srhd_fluid_step_grid(t, prims2, nb, g.dh_lev, dt_lev=dtg, prec=prec, guess=guess,
                                     learned_split=True, net_in=out_mask)
    torch.cuda.synchronize()
    w2 = _listed_by_masks(got, g.neighbor.reshape(P, 27))
    assert np.array_equal(b.cpu().numpy()[w2], a.cpu().numpy()[w2])


def test_concurrent_split_on_a_caller_stream(S, case):
    # the learned pass forks off the caller's stream and joins back into it: a chain of steps
    # issued on a stream of the caller's, with no synchronisation between the steps, gives the
    # bits of the same chain on the default stream
    g, cons, dt, pad, ref, mlp, listed = case
    P = g.n_patch
    guess = mlp.guess()
    nb = torch.from_numpy(g.neighbor).to(DEV)

    def chain():
        c = torch.from_numpy(cons).to(DEV)
        m = S.new_net_mask(P, DEV)
        prims, smax = S.srhd_grid_prims(c, prec=1, guess=guess, net_mask=m)
        for _ in range(3):
            m2 = S.new_net_mask(P, DEV)
            c, prims, smax = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, prec=1,
                                                    guess=guess, net_in=m, net_out=m2)
            m = m2
        return c, m

    ref_c, ref_m = chain()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got_c, got_m = chain()
    s.synchronize()
    assert torch.equal(got_c, ref_c) and torch.equal(got_m, ref_m)
