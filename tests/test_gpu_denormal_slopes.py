"""GPU regression: primitives whose differences are denormal in FP32 (an undisturbed ambient gas
carrying the 1e-40-sized velocity residue that distant waves leave in FP64) must give zero
slopes, not NaN.  The FP32 harmonic-mean slope divides through the hardware reciprocal, which
flushes a denormal denominator; every output cell must stay finite and physical in the FP32-bulk
modes, for MUSCL-Hancock and VL, and agree with the oracle in FP64."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import oracle_cons, step_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _ambient_with_residue(n=32):
    g = W.blast(n, seed=3)
    g.prim[:, 0] = W.BLAST_AMBIENT[0]                 # the ambient everywhere: no source
    g.prim[:, 4] = W.BLAST_AMBIENT[4]
    x, y, z = W.patch_cell_centres(n // 8, n // 8, n // 8, 1.0 / n)
    # FP32 denormals (FLT_MIN = 1.2e-38): monotone runs in every direction, so the limiter's
    # monotone branch is taken with both one-sided differences denormal
    g.prim[:, 1] = 1e-41 * (2.0 + np.sin(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * y))
    g.prim[:, 2] = -3e-42 * (2.0 + np.cos(2 * np.pi * z))
    g.prim[:, 3] = 1e-43 * (1.0 + x)
    return g


@pytest.mark.parametrize("integrator", [0, 1])
def test_denormal_differences_give_finite_physical_steps(S, integrator):
    g = _ambient_with_residue()
    cons = oracle_cons(g)
    dt, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad_o = O.fill_ghosts(cons, g.neighbor, 3)
    ref, cnt = O.fluid_step(pad_o, dt, g.dh_lev, integrator=integrator)
    assert cnt[0] == 0
    pad = torch.from_numpy(pad_o).to(DEV)
    dtg = torch.from_numpy(dt).to(DEV)
    for prec in (0, 1, 2):
        st = S.new_stats(DEV)
        out = S.srhd_fluid_step(pad, dtg, g.dh_lev, prec=prec, stats=st, integrator=integrator)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        sd = S.stats_dict(st)
        e = step_errors(o, ref)
        print("integrator %d prec %d: %s, stats %s" % (integrator, prec, e, sd))
        assert np.isfinite(o).all(), (integrator, prec)
        assert sd["n_unphysical"] == 0 and sd["n_retry"] == 0, sd
        # D and Et are the ambient's to round-off in every mode; the momenta are denormal-sized
        # in FP32 and compare in absolute terms
        assert e["D"] <= (1e-10 if prec == 0 else 1e-6) and e["Et"] <= (1e-10 if prec == 0 else 1e-5), e
        assert np.max(np.abs(o[:, 1:4] - ref[:, 1:4])) <= 1e-35


@pytest.mark.parametrize("integrator", [0, 1])
def test_blast_trajectory_with_residue_stays_physical(S, integrator):
    # the FP64 trajectory of the 64^3 blast fills the ambient gas with such residues ahead of
    # the shell; every precision mode must step each of its states without unphysical output
    g = W.blast(64, seed=3, order="morton")
    c = torch.from_numpy(oracle_cons(g)).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    bad = {1: 0, 2: 0}
    for k in range(16):
        dt = S.srhd_cfl_dt(c, g.dh_lev)
        pad = S.srhd_fill_ghosts(c, nb)
        for prec in (1, 2):
            st = S.new_stats(DEV)
            o = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=prec, stats=st, integrator=integrator)
            bad[prec] += S.stats_dict(st)["n_unphysical"] + int((~torch.isfinite(o)).sum().item())
        c = S.srhd_fluid_step(pad, dt, g.dh_lev, prec=0, integrator=integrator)
    torch.cuda.synchronize()
    print("integrator %d: unphysical or non-finite output cells over 16 steps %s" % (integrator, bad))
    assert bad == {1: 0, 2: 0}
