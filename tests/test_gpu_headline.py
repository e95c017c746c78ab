"""Full-size parity of the benchmark's headline configuration: the 256^3 blast (32,768 patches in
Morton order) stepped by the gather-layout chain -- the next step's time step fused in, FP32
primitives handed from step to step -- in mixed precision with the trained learned guess
(paper_2012_11130_amd/mlp_guess.npz), its network masks handed from step to step (the learned
kernel on the library's second stream), and the precision guard, for four steps; and the same
chain in FP64.

Each step is compared with the oracle's step of the GPU's own input state (the step is
patch-local given its ghosts, Sec. 3.1): the oracle fills the ghosts of the GPU's current
interiors and steps 300+ sampled patches -- every patch whose step reads the source ellipsoid's
cells or the waves it has launched (where the state departs from the ambient gas) and 300 random
ones -- with the time step the GPU used.  Mixed: per patch within (C_KAPPA kappa_tile + C_FLUX)
u32 (Eq. 20 with the FP32 unit roundoff, tests/test_gpu_guard.py; kappa_tile over the cells the
patch's step reads); FP64:
within 1e-10 per field."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import kappa_tile_padded, oracle_cons, patch_errors, step_bound, step_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N_STEPS = 4


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


@pytest.fixture(scope="module")
def blast():
    g = W.blast(256, seed=1003, order="morton")
    return g, oracle_cons(g)


def _sample(cons, g, rng):
    """Patches whose state departs from the ambient gas (the source and the waves it launched),
    with their face neighbours, plus 300 random patches."""
    amb = cons[np.flatnonzero(g.extra["labels"].reshape(g.n_patch, -1).sum(axis=1) == 0)[0], :, 0, 0, 0]
    dev = np.abs(cons - amb[None, :, None, None, None]).reshape(g.n_patch, -1).max(axis=1) > 1e-12
    active = np.flatnonzero(dev)
    nb = g.neighbor[active][:, [4, 10, 12, 14, 16, 22]].ravel()
    near = np.union1d(active, nb[nb >= 0])
    return np.union1d(near, rng.choice(g.n_patch, 300, replace=False))


@pytest.mark.parametrize("prec", [1, 0])
def test_headline_chain_full_size(S, blast, prec):
    g, cons0 = blast
    guess = None
    if prec == 1:
        from paper_2012_11130_amd import mlp_train
        mlp = mlp_train.load(device=DEV)
        assert mlp is not None, "the trained weights of the learned guess are part of the package"
        guess = mlp.guess()
    c = torch.from_numpy(cons0).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    mask = S.new_net_mask(g.n_patch, DEV) if guess is not None else None
    prims, smax = S.srhd_grid_prims(c, prec=prec, guess=guess, net_mask=mask)
    rng = np.random.default_rng(7)
    dt_used = torch.empty(1, dtype=torch.float64, device=DEV)
    for step in range(N_STEPS):
        cin = c.cpu().numpy()
        st = S.new_stats(DEV)
        mask_out = S.new_net_mask(g.n_patch, DEV) if guess is not None else None
        c, prims, smax = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, smax_in=smax, c_cfl=0.5,
                                                prec=prec, guess=guess, stats=st, dt_used=dt_used,
                                                net_in=mask, net_out=mask_out)
        mask = mask_out
        out = c.cpu().numpy()
        dt = dt_used.cpu().numpy()
        sd = S.stats_dict(st)
        sample = _sample(cin, g, rng)
        pad_o = O.fill_ghosts(cin, g.neighbor[sample], 3)
        ref, cnt = O.fluid_step(pad_o, dt, g.dh_lev)
        got = out[sample]
        e = step_errors(got, ref)
        ep = patch_errors(got, ref)
        if prec == 1:
            kap = kappa_tile_padded(pad_o)
            bound = step_bound(kap)
            print("mixed+learned step %d: %d sampled patches, errors %s, largest error / bound "
                  "%.3f (kappa_tile up to %.3g); stats %s"
                  % (step, sample.size, e, (ep / bound).max(), kap.max(), sd))
            assert np.all(ep <= bound), (step, e)
            assert sd["n_mlp"] > 0
        else:
            print("fp64 step %d: %d sampled patches, errors %s; stats %s" % (step, sample.size, e, sd))
            assert max(e.values()) <= 1e-10, (step, e)
            assert sd["n_retry"] == cnt[3]
        assert sd["n_noconv"] == 0 and sd["n_unphysical"] == 0 and cnt[0] == 0
