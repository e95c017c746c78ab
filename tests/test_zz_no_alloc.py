"""srhd_fluid_step_static, the allocation-free variant of srhd_fluid_step for callers that cannot
allocate, through the C ABI: its output equals srhd_fluid_step's bit for bit on two calls in a
row -- the jet block with the precision guard listing its nozzle patches (the guard's list in
the static array) on a persistent schedule (the queue counters there too), then a smaller input
(the first 27 of those patches) -- and sizes beyond the static array are refused."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.parity import oracle_cons

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _case(n=None):
    g = W.jet_block()
    cons = oracle_cons(g)
    dt, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    pad = O.fill_ghosts(cons, g.neighbor, 3)
    if n is not None:
        pad = pad[:n]
    return (torch.from_numpy(np.ascontiguousarray(pad)).to(DEV), torch.from_numpy(dt).to(DEV),
            g.dh_lev)


@pytest.mark.parametrize("prec", [1, 0])
def test_static_equals_step_twice(S, prec):
    for n in (None, 27):
        pad, dt, dh = _case(n)
        sch = S.Sched(512, 2, DEV)
        st_a, st_b = S.new_stats(DEV), S.new_stats(DEV)
        a = S.srhd_fluid_step(pad, dt, dh, prec=prec, sched=sch, stats=st_a)
        b = S.srhd_fluid_step_static(pad, dt, dh, prec=prec, groups=512, chunk=2, stats=st_b)
        torch.cuda.synchronize()
        sa, sb = S.stats_dict(st_a), S.stats_dict(st_b)
        print("prec %d, %d patches: %s" % (prec, pad.shape[0], sb))
        assert torch.equal(a, b)
        assert sa == sb
        if prec == 1:
            assert sb["n_fp64_patch"] > 0          # the guard's list was used


def test_static_one_patch_per_workgroup(S):
    pad, dt, dh = _case(40)
    a = S.srhd_fluid_step(pad, dt, dh, prec=1)
    b = S.srhd_fluid_step_static(pad, dt, dh, prec=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_static_refuses_oversized_and_buffers(S):
    pad, dt, dh = _case(8)
    d = S._patches(pad, dh, None, 3)
    d.n_patch = S.STATIC_MAX_PATCH + 1          # refused before any launch or read
    prm = S._params(1.5, S.HLLC, 1, 4, None, None)
    out = torch.empty((8, 5, 8, 8, 8), dtype=torch.float64, device=DEV)
    rc = S._lib.srhd_fluid_step_static(S.ctypes.byref(d), out.data_ptr(), dt.data_ptr(),
                                       S.ctypes.byref(prm), None, None)
    assert rc == -1 and b"static" in S._lib.srhd_last_error()
    d.n_patch = 8
    q = torch.zeros(8, dtype=torch.int64, device=DEV)
    prm.sched = S.srhd_sched(64, 1, 0, q.data_ptr())
    rc = S._lib.srhd_fluid_step_static(S.ctypes.byref(d), out.data_ptr(), dt.data_ptr(),
                                       S.ctypes.byref(prm), None, None)
    assert rc == -1 and b"queue" in S._lib.srhd_last_error()
