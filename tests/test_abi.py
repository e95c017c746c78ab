"""The C ABI: the shared library loads on the CPU and exports every function that
include/srhd.h declares; host-side argument checks reject bad calls before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srhd.h")
LIB = os.path.join(ROOT, "paper_2012_11130_amd", "libsrhd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(srhd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2012_11130_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_argument_errors_are_reported_without_a_gpu(lib):
    lib.srhd_prim2cons.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.srhd_last_error.restype = ctypes.c_char_p
    assert lib.srhd_prim2cons(7, 10, None, None, None, None) == -1
    assert b"dtype" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, -1, None, None, None, None) == -1
    assert lib.srhd_prim2cons(0, 10, None, None, None, None) == -1
    assert b"NULL" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, 0, None, None, None, None) == 0       # empty batch is a no-op
    # overlapping arrays are rejected before any launch (host addresses are never touched)
    buf = ctypes.create_string_buffer(800)
    a = ctypes.addressof(buf)
    assert lib.srhd_prim2cons(0, 10, a, a + 8, None, None) == -1
    assert b"overlap" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, 1, a + 1, a + 400, None, None) == -1      # misaligned
    lib.srhd_abi_version.restype = ctypes.c_int
    assert lib.srhd_abi_version() == 8


def test_step_descriptor_checks(lib):
    from paper_2012_11130_amd import srhd as S  # noqa: F401  (struct definitions only)
    d = S.srhd_patches()
    d.n_patch = 4
    d.ghost = 1
    d.dtype = 0
    d.n_level = 1
    d.dh[0] = 0.1
    prm = S.srhd_step_params()
    prm.theta = 1.5
    prm.max_retry = 4
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -1 and b"ghost" in S._lib.srhd_last_error()
    d.ghost = 3
    prm.theta = 5.0
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -1 and b"theta" in S._lib.srhd_last_error()
    prm.theta = 1.5
    d.dtype = 1
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -3


def test_schedule_checks(lib):
    # every call below fails its host-side checks before any launch (host buffers stand in for
    # device arrays and are never touched)
    from paper_2012_11130_amd import srhd as S
    pad = ctypes.create_string_buffer(4 * 5 * 14 ** 3 * 8 + 64)
    out = ctypes.create_string_buffer(4 * 5 * 512 * 8 + 64)
    dt = ctypes.create_string_buffer(64)
    al = lambda b: (ctypes.addressof(b) + 63) // 64 * 64
    d = S.srhd_patches()
    d.n_patch, d.ghost, d.dtype, d.n_level = 4, 3, 0, 1
    d.dh[0] = 0.1
    d.padded = al(pad)
    prm = S.srhd_step_params()
    prm.theta, prm.max_retry = 1.5, 4
    call = lambda: S._lib.srhd_fluid_step(ctypes.byref(d), al(out), al(dt), ctypes.byref(prm),
                                          None, None)
    prm.sched = S.srhd_sched(-1, 1, 0, None)
    assert call() == -1 and b"groups" in S._lib.srhd_last_error()
    prm.sched = S.srhd_sched(512, 1, 0, None)
    assert call() == -1 and b"queue" in S._lib.srhd_last_error()
    q = ctypes.create_string_buffer(128)
    prm.sched = S.srhd_sched(512, 0, 0, al(q))
    assert call() == -1 and b"chunk" in S._lib.srhd_last_error()
    prm.sched = S.srhd_sched(512, 65, 0, al(q))
    assert call() == -1 and b"chunk" in S._lib.srhd_last_error()
    n = ctypes.c_int(0)
    prm.sched = S.srhd_sched(0, 1, 0, None)
    rc = S._lib.srhd_autotune_step(ctypes.byref(d), al(out), al(dt), ctypes.byref(prm), 2, None,
                                   0, ctypes.byref(n), None)
    assert rc == -1 and b"queue" in S._lib.srhd_last_error()
    prm.sched = S.srhd_sched(0, 1, 0, al(q))
    rc = S._lib.srhd_autotune_step(ctypes.byref(d), al(out), al(dt), ctypes.byref(prm), 0, None,
                                   0, ctypes.byref(n), None)
    assert rc == -1 and b"reps" in S._lib.srhd_last_error()
    # the two-workgroup variant exists for mixed precision only
    prm.sched = S.srhd_sched(0, 1, 2, None)
    assert call() == -3 and b"occupancy" in S._lib.srhd_last_error()
    prm.sched = S.srhd_sched(0, 1, 3, None)
    assert call() == -1 and b"occupancy" in S._lib.srhd_last_error()
    def occ(prec, kind, gather, occupancy, energy=0, integrator=0):
        q = S.srhd_step_params()
        q.prec, q.guess, q.energy, q.integrator = prec, S.srhd_guess(kind, None, 0), energy, integrator
        q.sched = S.srhd_sched(0, 1, occupancy, None)
        return S._lib.srhd_step_occupancy(ctypes.byref(q), gather)
    assert S._lib.srhd_step_occupancy(None, 0) == -1
    assert occ(5, 0, 0, 0) == -1
    assert occ(0, 7, 0, 0) == -1
    assert occ(1, 0, 0, 1) == -1
    assert occ(0, 0, 0, 2) == -3
    assert occ(0, 1, 0, 2) == -3
    # the original (total-energy) scheme: padded layout, FP64 or FP32, analytic guess
    prm.sched = S.srhd_sched(0, 1, 0, None)
    prm.energy = 2
    assert call() == -1 and b"energy" in S._lib.srhd_last_error()
    prm.energy = 1
    prm.prec = 1
    assert call() == -3 and b"total-energy" in S._lib.srhd_last_error()
    prm.prec = 0
    prm.guess = S.srhd_guess(1, None, 0)
    assert call() == -1                      # learned guess without weights: rejected first
    prm.guess = S.srhd_guess(0, None, 0)
    prm.energy = 0
    assert occ(0, 0, 0, 0, energy=2) == -1
    assert occ(1, 0, 0, 0, energy=1) == -3
    assert occ(0, 1, 0, 0, energy=1) == -3
    assert occ(0, 0, 1, 0, energy=1) == -3 and b"padded" in S._lib.srhd_last_error()
    # the VL integrator: analytic guess, reduced energy; ghost >= 3 in the padded layout
    prm.integrator = 2
    assert call() == -1 and b"integrator" in S._lib.srhd_last_error()
    prm.integrator = 1
    prm.energy = 1
    assert call() == -3 and b"VL" in S._lib.srhd_last_error()
    prm.energy = 0
    d.ghost = 2
    assert call() == -1 and b"ghost" in S._lib.srhd_last_error()
    d.ghost = 3
    prm.integrator = 0
    assert occ(0, 0, 1, 0, energy=1, integrator=1) == -3 and b"VL" in S._lib.srhd_last_error()
    assert occ(2, 1, 0, 0, integrator=1) == -3
    assert occ(2, 1, 1, 0, integrator=1) == -3
    # the polytropic EoS: 1 < gamma <= 2; padded MUSCL-Hancock, reduced energy, analytic guess
    prm.eos = S.srhd_eos(1, 2.5)
    assert call() == -1 and b"gamma" in S._lib.srhd_last_error()
    prm.eos = S.srhd_eos(7, 1.5)
    assert call() == -1 and b"EoS" in S._lib.srhd_last_error()
    prm.eos = S.srhd_eos(1, 5.0 / 3.0)
    prm.integrator = 1
    assert call() == -3 and b"polytropic" in S._lib.srhd_last_error()
    prm.integrator = 0
    prm.eos = S.srhd_eos(0, 0.0)
    # the precision guard: kappa_max 0 or >= 1; an FP32 bulk needs an aligned workspace that
    # overlaps no other array of the call
    prm.prec = 1
    for bad_k in (0.5, -1.0, float("nan")):
        prm.kappa_max = bad_k
        assert call() == -1 and b"kappa_max" in S._lib.srhd_last_error()
    prm.kappa_max = 1024.0
    prm.defer = None
    assert call() == -1 and b"defer" in S._lib.srhd_last_error()
    ws = ctypes.create_string_buffer(8 * 8 + 64)
    prm.defer = al(ws) + 4
    assert call() == -1 and b"defer" in S._lib.srhd_last_error()
    prm.defer = al(out)
    assert call() == -1 and b"overlaps" in S._lib.srhd_last_error()
    prm.defer = None
    prm.kappa_max = 0.0
    prm.learned_split = 2
    assert call() == -1 and b"learned_split" in S._lib.srhd_last_error()
    prm.learned_split = 0
    prm.prec = 0
    # the allocation-free step: at most SRHD_STATIC_MAX_PATCH patches, no caller work buffers
    d.n_patch = S.STATIC_MAX_PATCH + 1
    rc = S._lib.srhd_fluid_step_static(ctypes.byref(d), al(out), al(dt), ctypes.byref(prm), None,
                                       None)
    assert rc == -1 and b"static" in S._lib.srhd_last_error()
    d.n_patch = 4
    prm.defer = al(ws)
    rc = S._lib.srhd_fluid_step_static(ctypes.byref(d), al(out), al(dt), ctypes.byref(prm), None,
                                       None)
    assert rc == -1 and b"defer" in S._lib.srhd_last_error()
    prm.defer = None
    q = S.srhd_step_params()
    q.eos = S.srhd_eos(1, 4.0 / 3.0)
    assert S._lib.srhd_step_occupancy(ctypes.byref(q), 1) == -3
    bad = S.srhd_eos(1, 1.0)
    assert S._lib.srhd_prim2cons(0, 10, None, None, ctypes.byref(bad), None) == -1
    assert S._lib.srhd_cfl_dt(0, 0, None, 1, (ctypes.c_double * 1)(0.1), 0.5, None, None,
                              ctypes.byref(bad), None) == -1


def test_network_mask_checks(lib):
    # host buffers stand in for device arrays: every call fails its checks before any launch
    from paper_2012_11130_amd import srhd as S
    P = 4
    buf = lambda n: ctypes.create_string_buffer(n + 64)
    al = lambda b: (ctypes.addressof(b) + 63) // 64 * 64
    cons, prims, cout, pout = buf(P * 2560 * 8), buf(P * 2560 * 4), buf(P * 2560 * 8), buf(P * 2560 * 4)
    nb, sm, masks = buf(P * 27 * 4), buf(16), buf(64)
    g = S.srhd_guess(0, None, 0)
    # srhd_grid_prims: misaligned or overlapping network masks
    assert S._lib.srhd_grid_prims(1, P, al(cons), al(prims), al(sm), al(masks) + 2, ctypes.byref(g),
                                  None) == -1
    assert b"misaligned" in S._lib.srhd_last_error()
    assert S._lib.srhd_grid_prims(1, P, al(cons), al(prims), al(sm), al(prims), ctypes.byref(g),
                                  None) == -1
    assert b"net_mask" in S._lib.srhd_last_error()
    gr = S.srhd_grid()
    gr.n_patch, gr.cons, gr.prims, gr.neighbor, gr.n_level = P, al(cons), al(prims), al(nb), 1
    gr.dh[0] = 0.1
    prm = S.srhd_step_params()
    prm.theta, prm.max_retry, prm.prec = 1.5, 4, 1
    call = lambda net_out: S._lib.srhd_fluid_step_grid(ctypes.byref(gr), al(sm), 0.5, None, al(cout),
                                                       al(pout), al(sm) + 8, net_out, None,
                                                       ctypes.byref(prm), None, None)
    assert call(al(masks) + 2) == -1 and b"misaligned" in S._lib.srhd_last_error()
    assert call(al(cout)) == -1 and b"net_out" in S._lib.srhd_last_error()
    gr.net_mask = al(masks)
    assert call(al(masks) + 8) == -1 and b"net_out" in S._lib.srhd_last_error()
    gr.net_mask = al(masks) + 2
    assert call(None) == -1 and b"misaligned" in S._lib.srhd_last_error()
    # the VL integrator in the gather layout: the reduced energy and the analytic guess only, no
    # boundary fluxes (rejected before any launch)
    gr.net_mask = None
    prm.integrator, prm.energy = 1, 1
    assert call(None) == -3 and b"VL" in S._lib.srhd_last_error()
    prm.energy = 0
    prm.flux_out = al(cout)
    assert call(None) == -3 and b"boundary fluxes" in S._lib.srhd_last_error()
    prm.flux_out = None
    prm.guess = S.srhd_guess(1, None, 0)
    assert call(None) == -1                  # a learned guess without weights: rejected first
    wb = buf(4352 * 2 + 129 * 4 + 8 * 4)
    mlp = S.srhd_mlp(al(wb), al(wb) + 8704, al(wb) + 8704 + 516, 0, 0.1)
    prm.guess = S.srhd_guess(1, ctypes.pointer(mlp), 0)
    assert call(None) == -3 and b"VL" in S._lib.srhd_last_error()
    prm.guess = S.srhd_guess(0, None, 0)
    prm.integrator = 0
