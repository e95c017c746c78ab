"""The jet patch list at full size: 4e5 patches of 8^3 over 4 levels (5/10/25/60 %), ghost cells
from the analytic initial state, one step of every patch in one launch of the persistent
schedule.  Parity on 1,000 sampled patches (half of them straddling the nozzle edge) against the
oracle: FP64 within 1e-10 per field; the mixed step (FP32 bulk, FP64 inversion, the learned guess
when its weights exist) with the precision guard of Eq. 20: the patches whose tile reaches the
nozzle (kappa = 1 + M^2 ~ 2e6) are stepped in FP64 and agree within 1e-10, the others within
(C_KAPPA kappa_tile + C_FLUX) u_32 (tests/test_gpu_guard.py derives the constants).

Both sides start from the same bits: the two conserved states (ambient, nozzle) come from the
oracle's prim -> cons and every padded cell holds one of them, selected by the cell's label."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import U64, kappa_prim, patch_errors, stencil_mask, step_errors
from tests.parity import step_bound
from tests.test_gpu_guard import KMAX

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N_SAMPLE = 1000


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


@pytest.fixture(scope="module")
def jet(S):
    pl = W.jet_patch_list()
    states = O.prim2cons(W.jet_states().T.copy()).T.copy()          # [2][5]: ambient, nozzle
    lab = W.jet_labels_torch(pl, DEV)
    pad = W.assemble_labeled(lab, states)
    level = torch.from_numpy(pl["level"]).to(DEV)
    # sample: half random patches, half among those with both labels (the nozzle edge)
    mixed = ((lab.amax(dim=(1, 2, 3)) == 1) & (lab.amin(dim=(1, 2, 3)) == 0)).cpu().numpy()
    rng = np.random.default_rng(55)
    edge = np.flatnonzero(mixed)
    e = rng.choice(edge, min(edge.size, N_SAMPLE // 2), replace=False)
    r = rng.choice(np.setdiff1d(np.arange(pad.shape[0]), e), N_SAMPLE - e.size, replace=False)
    sample = np.sort(np.concatenate([e, r]))
    torch.cuda.synchronize()
    print("jet: %d patches, %d with nozzle-edge cells, %d sampled" % (pad.shape[0], edge.size, sample.size))
    return pl, states, lab, pad, level, sample


@pytest.fixture(scope="module")
def dt(S, jet):
    pl, states, lab, pad, level, sample = jet
    interior = pad[:, :, 3:11, 3:11, 3:11].contiguous()
    dt_g = S.srhd_cfl_dt(interior, pl["dh_lev"], 0.5)
    del interior
    # S_max over the whole list is that of the faster of the two states
    one = np.empty((1, 5, 512))
    one[0] = states[0][:, None]
    one[0, :, 0] = states[1]
    dt_o, _, _ = O.cfl_dt(one, None, pl["dh_lev"], 0.5)
    torch.cuda.synchronize()
    assert np.max(np.abs(dt_g.cpu().numpy() / dt_o - 1)) < 1e-12
    return dt_o


def _oracle(jet, dt_o):
    pl, states, lab, pad, level, sample = jet
    host = W.assemble_labeled(W.jet_labels(pl, patches=sample), states)
    assert torch.equal(pad[torch.from_numpy(sample).to(DEV)].cpu(), torch.from_numpy(host))
    ref, cnt = O.fluid_step(host, dt_o, pl["dh_lev"], level=pl["level"][sample])
    return ref, cnt


@pytest.fixture(scope="module")
def oracle_ref(jet, dt):
    return _oracle(jet, dt)


def test_labels_on_device_equal_host(jet):
    pl, states, lab, pad, level, sample = jet
    assert np.array_equal(lab[torch.from_numpy(sample).to(DEV)].cpu().numpy(),
                          W.jet_labels(pl, patches=sample))


def test_fp64_full_list_persistent_sampled_parity(S, jet, dt, oracle_ref):
    pl, states, lab, pad, level, sample = jet
    ref, cnt = oracle_ref
    dtg = torch.from_numpy(dt).to(DEV)
    occ = S.srhd_step_occupancy(0, S.GUESS_ANALYTIC, False)
    sch = S.Sched(2 * occ * torch.cuda.get_device_properties(0).multi_processor_count, 2, DEV)
    st = S.new_stats(DEV)
    out = S.srhd_fluid_step(pad, dtg, pl["dh_lev"], level=level, prec=0, stats=st, sched=sch)
    per_patch = S.srhd_fluid_step(pad, dtg, pl["dh_lev"], level=level, prec=0)
    torch.cuda.synchronize()
    assert torch.equal(out, per_patch)
    got = out[torch.from_numpy(sample).to(DEV)].cpu().numpy()
    e = step_errors(got, ref)
    sd = S.stats_dict(st)
    print("fp64 jet: errors %s, oracle counts %s, device stats %s" % (e, cnt, sd))
    assert max(e.values()) <= 1e-10, e
    assert sd["n_noconv"] == 0


def _tile_kappa(labels, states_prim):
    """kappa_tile of padded patches given their cell labels [p][14][14][14] (ghost 3)."""
    kap = kappa_prim(np.asarray(states_prim).T)          # per state
    m = stencil_mask()
    box = labels[:, 1:13, 1:13, 1:13].reshape(labels.shape[0], -1)[:, m.ravel()]
    return kap[box].max(axis=1)


def test_mixed_learned_full_list_autotuned(S, jet, dt, oracle_ref):
    pl, states, lab, pad, level, sample = jet
    ref, cnt = oracle_ref
    from paper_2012_11130_amd import mlp_train
    mlp = mlp_train.load(device=DEV)
    guess = mlp.guess() if mlp is not None else None
    dtg = torch.from_numpy(dt).to(DEV)
    sch, table = S.srhd_autotune_step(pad, dtg, pl["dh_lev"], level=level, prec=1, guess=guess,
                                      reps=1, kappa_max=KMAX)
    st = S.new_stats(DEV)
    out = S.srhd_fluid_step(pad, dtg, pl["dh_lev"], level=level, prec=1, stats=st, guess=guess,
                            sched=sch, kappa_max=KMAX)
    # patches whose step reads a nozzle cell, over the whole list (on the device)
    m = torch.from_numpy(stencil_mask().ravel()).to(DEV)
    n_hot = 0
    for s0 in range(0, lab.shape[0], 32768):
        box = lab[s0:s0 + 32768, 1:13, 1:13, 1:13].reshape(-1, 1728)[:, m]
        n_hot += int((box.amax(dim=1) > 0).sum().item())
    torch.cuda.synchronize()
    got = out[torch.from_numpy(sample).to(DEV)].cpu().numpy()
    e = step_errors(got, ref)
    sd = S.stats_dict(st)
    kap = _tile_kappa(W.jet_labels(pl, patches=sample), W.jet_states())
    hot = kap > KMAX
    ep = patch_errors(got, ref)
    print("mixed jet (%s guess): errors %s; hot patches %d (device %d), sampled hot %d max error "
          "%.3e, others %.3e (bound %.3e); schedule %s of %s; stats %s"
          % ("learned" if mlp is not None else "analytic", e, n_hot, sd["n_fp64_patch"], hot.sum(),
             ep[hot].max(), ep[~hot].max(), step_bound(kap[~hot]).max(), sch, table, sd))
    assert sd["n_fp64_patch"] == n_hot and hot.any()
    assert np.all(ep[hot] <= np.maximum(1e-10, step_bound(kap[hot], U64)))
    assert np.all(ep[~hot] <= step_bound(kap[~hot]))
    assert sd["n_noconv"] == 0


def test_mixed_without_guard_loses_the_nozzle_pressure(S, jet, dt, oracle_ref):
    # Eq. 20 with the FP32 unit roundoff: rounding the nozzle's face states to FP32 moves their
    # pressure by about 1.5 %, and the cold neighbours' reduced energy follows
    pl, states, lab, pad, level, sample = jet
    ref, cnt = oracle_ref
    out = S.srhd_fluid_step(pad, torch.from_numpy(dt).to(DEV), pl["dh_lev"], level=level, prec=1,
                            kappa_max=0.0)
    got = out[torch.from_numpy(sample).to(DEV)].cpu().numpy()
    e = step_errors(got, ref)
    print("mixed jet without the guard: %s" % e)
    assert e["Et"] > 1e-3
