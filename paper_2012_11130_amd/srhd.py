"""Thin ctypes binding of libsrhd (include/srhd.h) for PyTorch device tensors.

Argument marshalling only: every computation runs in the HIP kernels of libsrhd.so.  Tensors
must live on the GPU; the current torch stream is passed to the library.  Importing this module
fails loudly if the library has not been built (``python -m paper_2012_11130_amd.build``).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrhd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libsrhd.so is missing: build it with `python -m paper_2012_11130_amd.build` "
                      "(there is no fallback implementation)")

_lib = ctypes.CDLL(LIB_PATH)

F64, F32 = 0, 1
OK, EINVAL, EHIP, EUNSUPPORTED = 0, -1, -2, -3
ST_OK, ST_UNPHYSICAL, ST_FALLBACK, ST_NOCONV = 0, 1, 2, 3
GUESS_ANALYTIC, GUESS_MLP = 0, 1
FEAT_CONS, FEAT_L = 0, 1
HLLC, HLLE = 0, 1
PREC_FP64, PREC_MIXED, PREC_FP32 = 0, 1, 2
ENERGY_REDUCED, ENERGY_TOTAL = 0, 1
MHM, VL = 0, 1
MAX_LEVEL = 8

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


class srhd_mlp(ctypes.Structure):
    _fields_ = [("w_bf16", _vp), ("bias", _vp), ("norm", _vp), ("features", _int),
                ("gate_L", ctypes.c_double)]


class srhd_guess(ctypes.Structure):
    _fields_ = [("kind", _int), ("mlp", ctypes.POINTER(srhd_mlp)), ("max_iter", _int)]


class srhd_patches(ctypes.Structure):
    _fields_ = [("n_patch", _i64), ("ghost", _int), ("dtype", _int), ("padded", _vp),
                ("level", _vp), ("n_level", _int), ("dh", ctypes.c_double * MAX_LEVEL)]


class srhd_grid(ctypes.Structure):
    _fields_ = [("n_patch", _i64), ("cons", _vp), ("prims", _vp), ("neighbor", _vp),
                ("level", _vp), ("n_level", _int), ("dh", ctypes.c_double * MAX_LEVEL),
                ("net_mask", _vp)]


class srhd_eos(ctypes.Structure):
    _fields_ = [("kind", _int), ("gamma", ctypes.c_double)]


EOS_TM, EOS_POLYTROPIC = 0, 1


def _eos(gamma):
    """srhd_eos for the TM EoS (gamma None) or the polytropic EoS with this Gamma."""
    return srhd_eos(EOS_TM, 0.0) if gamma is None else srhd_eos(EOS_POLYTROPIC, float(gamma))


class srhd_sched(ctypes.Structure):
    _fields_ = [("groups", _int), ("chunk", _int), ("occupancy", _int), ("queue", _vp)]


class srhd_step_params(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("riemann", _int), ("prec", _int),
                ("max_retry", _int), ("guess", srhd_guess), ("sched", srhd_sched),
                ("energy", _int), ("integrator", _int), ("eos", srhd_eos), ("flux_out", _vp),
                ("kappa_max", ctypes.c_double), ("learned_split", _int), ("defer", _vp)]


# precision guard of the FP32-bulk steps: patches holding a cell with 1 + M^2 above this are
# stepped in FP64 (0 turns it off)
KAPPA_MAX_DEFAULT = 1024.0


class srhd_tune_entry(ctypes.Structure):
    _fields_ = [("groups", _int), ("chunk", _int), ("occupancy", _int), ("ms", ctypes.c_float)]


QUEUE_WORDS = 8


class srhd_step_stats(ctypes.Structure):
    _fields_ = [("n_unphysical", ctypes.c_uint64), ("n_fallback", ctypes.c_uint64),
                ("n_noconv", ctypes.c_uint64), ("newton_iters", ctypes.c_uint64),
                ("n_inversions", ctypes.c_uint64), ("n_retry", ctypes.c_uint64),
                ("n_mlp", ctypes.c_uint64), ("n_pred_fallback", ctypes.c_uint64),
                ("n_fp64_patch", ctypes.c_uint64), ("n_learned_patch", ctypes.c_uint64)]


STATS_FIELDS = ("n_unphysical", "n_fallback", "n_noconv", "newton_iters", "n_inversions",
                "n_retry", "n_mlp", "n_pred_fallback", "n_fp64_patch", "n_learned_patch")
STATS_WORDS = len(STATS_FIELDS)

_sig = {
    "srhd_prim2cons": [_int, _i64, _vp, _vp, ctypes.POINTER(srhd_eos), _vp],
    "srhd_cons2prim": [_int, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(srhd_guess),
                       ctypes.POINTER(srhd_eos), _vp],
    "srhd_fill_ghosts": [_int, _i64, _int, _i64, _vp, _vp, _vp, _vp],
    "srhd_cfl_dt": [_int, _i64, _vp, _int, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                    _vp, _vp, ctypes.POINTER(srhd_eos), _vp],
    "srhd_stats_reset": [_vp, _vp],
    "srhd_fluid_step": [ctypes.POINTER(srhd_patches), _vp, _vp,
                        ctypes.POINTER(srhd_step_params), _vp, _vp],
    "srhd_fluid_step_static": [ctypes.POINTER(srhd_patches), _vp, _vp,
                               ctypes.POINTER(srhd_step_params), _vp, _vp],
    "srhd_grid_prims": [_int, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(srhd_guess), _vp],
    "srhd_mlp_features": [_int, _int, _i64, _vp, _vp, _vp, _vp, _vp],
    "srhd_mlp_forward": [ctypes.POINTER(srhd_mlp), _i64, _vp, _vp, _vp],
    "srhd_mlp_grad": [ctypes.POINTER(srhd_mlp), _i64, _vp, _vp, _vp, _vp, _vp, _vp],
    "srhd_mlp_adam": [_vp, _vp, _vp, _vp, _int, ctypes.c_float, _vp, _vp, _vp],
    "srhd_fluid_step_grid": [ctypes.POINTER(srhd_grid), _vp, ctypes.c_double, _vp, _vp, _vp,
                             _vp, _vp, _vp, ctypes.POINTER(srhd_step_params), _vp, _vp],
    "srhd_step_occupancy": [ctypes.POINTER(srhd_step_params), _int],
    "srhd_autotune_step": [ctypes.POINTER(srhd_patches), _vp, _vp,
                           ctypes.POINTER(srhd_step_params), _int,
                           ctypes.POINTER(srhd_tune_entry), _int, ctypes.POINTER(_int), _vp],
    "srhd_fill_ghosts_coarse": [_i64, _int, _vp, _vp, _vp, _i64, _int, _vp, _vp, ctypes.c_double,
                                ctypes.c_double, _vp, _vp, _vp],
    "srhd_restrict": [_i64, _vp, _vp, _i64, _vp, _i64, _vp, _vp],
    "srhd_flux_accumulate": [_i64, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp],
    "srhd_flux_correct": [_i64, _vp, _i64, _vp, _vp, _i64, _vp, ctypes.c_double, _vp, _vp],
    "srhd_autotune_step_grid": [ctypes.POINTER(srhd_grid), _vp, ctypes.c_double, _vp, _vp, _vp,
                                _vp, _vp, ctypes.POINTER(srhd_step_params), _int,
                                ctypes.POINTER(srhd_tune_entry), _int, ctypes.POINTER(_int), _vp],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _int
_lib.srhd_last_error.argtypes = []
_lib.srhd_last_error.restype = ctypes.c_char_p
_lib.srhd_cfl_work_bytes.argtypes = []
_lib.srhd_cfl_work_bytes.restype = ctypes.c_size_t
_lib.srhd_abi_version.argtypes = []
_lib.srhd_abi_version.restype = _int
_lib.srhd_mlp_workspace_bytes.argtypes = [_i64]
_lib.srhd_mlp_workspace_bytes.restype = ctypes.c_size_t

EXPORTS = tuple(_sig) + ("srhd_last_error", "srhd_cfl_work_bytes", "srhd_abi_version",
                         "srhd_mlp_workspace_bytes")
MLP_NPARAM = 4481


class SrhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libsrhd error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != OK:
        raise SrhdError(rc, _lib.srhd_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("expected float64 or float32 tensor, got %s" % t.dtype)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous GPU tensors")


# ------------------------------------------------------------------------------- conversions
def srhd_prim2cons(prim, cons=None, gamma=None):
    """prim [5][n] -> cons [5][n] (same dtype); gamma selects the polytropic EoS."""
    _need_cuda(prim)
    if cons is None:
        cons = torch.empty_like(prim)
    _need_cuda(cons)
    n = prim.shape[-1]
    e = _eos(gamma)
    _check(_lib.srhd_prim2cons(_dtype_code(prim), n, _ptr(prim), _ptr(cons), ctypes.byref(e),
                               _stream()))
    return cons


def srhd_cons2prim(cons, prim=None, status=None, iters=None, guess=None, max_iter=0, gamma=None):
    """cons [5][n] -> prim [5][n]; status int8 [n] and iters uint8 [n] if given (or True);
    gamma selects the polytropic EoS."""
    _need_cuda(cons)
    n = cons.shape[-1]
    if prim is None:
        prim = torch.empty_like(cons)
    if status is True:
        status = torch.empty(n, dtype=torch.int8, device=cons.device)
    if iters is True:
        iters = torch.empty(n, dtype=torch.uint8, device=cons.device)
    _need_cuda(prim, status, iters)
    g = guess if guess is not None else srhd_guess(GUESS_ANALYTIC, None, max_iter)
    e = _eos(gamma)
    _check(_lib.srhd_cons2prim(_dtype_code(cons), n, _ptr(cons), _ptr(prim), _ptr(status),
                               _ptr(iters), ctypes.byref(g), ctypes.byref(e), _stream()))
    return prim, status, iters


# ------------------------------------------------------------------------------- patches
def srhd_fill_ghosts(interior, neighbor, ghost=3, padded=None):
    """interior [Q][5][8][8][8] + neighbour table [P][27] int32 -> padded [P][5][N][N][N]."""
    _need_cuda(interior, neighbor)
    if neighbor.dtype != torch.int32:
        raise TypeError("neighbour table must be int32")
    P = neighbor.shape[0]
    N = 8 + 2 * ghost
    if padded is None:
        padded = torch.empty((P, 5, N, N, N), dtype=interior.dtype, device=interior.device)
    _need_cuda(padded)
    _check(_lib.srhd_fill_ghosts(_dtype_code(interior), P, ghost, interior.shape[0],
                                 _ptr(interior), _ptr(neighbor),
                                 _ptr(padded), _stream()))
    return padded


_cfl_work = {}


def _work(device):
    key = (device.type, device.index)
    if key not in _cfl_work:
        n = int(_lib.srhd_cfl_work_bytes())
        _cfl_work[key] = torch.empty(n, dtype=torch.uint8, device=device)
    return _cfl_work[key]


def srhd_cfl_dt(interior, dh, c_cfl=0.5, dt_lev=None, work=None, gamma=None):
    """Per-level time step (device float64 [n_level]) from interior cons [P][5][8][8][8];
    gamma selects the polytropic EoS."""
    _need_cuda(interior)
    dh = [float(x) for x in dh]
    nl = len(dh)
    if dt_lev is None:
        dt_lev = torch.empty(nl, dtype=torch.float64, device=interior.device)
    if work is None:
        work = _work(interior.device)
    arr = (ctypes.c_double * nl)(*dh)
    e = _eos(gamma)
    _check(_lib.srhd_cfl_dt(_dtype_code(interior), interior.shape[0], _ptr(interior), nl, arr,
                            float(c_cfl), _ptr(dt_lev), _ptr(work), ctypes.byref(e), _stream()))
    return dt_lev


def new_stats(device):
    return torch.zeros(STATS_WORDS, dtype=torch.int64, device=device)


def stats_dict(stats):
    v = stats.cpu().tolist()
    return dict(zip(STATS_FIELDS, v[:len(STATS_FIELDS)]))


def srhd_stats_reset(stats):
    _check(_lib.srhd_stats_reset(_ptr(stats), _stream()))


class Sched:
    """Launch schedule of a step: groups == 0 is one workgroup per patch; groups > 0 a
    persistent grid claiming `chunk` patches at a time from a device queue (owned here);
    occupancy 2 selects the kernel variant that fits two workgroups per compute unit."""

    def __init__(self, groups=0, chunk=1, device="cuda:0", occupancy=0):
        self.groups, self.chunk, self.occupancy = int(groups), int(chunk), int(occupancy)
        self.queue = torch.zeros(QUEUE_WORDS, dtype=torch.int64, device=device)

    def c(self):
        return srhd_sched(self.groups, self.chunk, self.occupancy, self.queue.data_ptr())

    def __repr__(self):
        return "Sched(groups=%d, chunk=%d, occupancy=%d)" % (self.groups, self.chunk, self.occupancy)


def _patches(padded, dh, level, ghost):
    P = padded.shape[0]
    N = padded.shape[-1]
    d = srhd_patches()
    d.n_patch = P
    d.ghost = (N - 8) // 2 if ghost is None else ghost
    d.dtype = _dtype_code(padded)
    d.padded = padded.data_ptr()
    d.level = None if level is None else level.data_ptr()
    dh = [float(x) for x in dh]
    d.n_level = len(dh)
    for i, h in enumerate(dh):
        d.dh[i] = h
    return d


def defer_workspace(n_patch, device):
    """Workspace of the precision guard and the learned-guess split for a step of n_patch
    patches."""
    return torch.empty(2 * n_patch + 4, dtype=torch.int64, device=device)


def _guard(prm, kappa_max, defer, n_patch, device, learned_split=True):
    """Set the precision guard and the learned-guess split of prm; returns the workspace (kept
    alive by the caller)."""
    prm.kappa_max = float(kappa_max)
    prm.learned_split = int(bool(learned_split))
    guard = prm.kappa_max != 0.0 and prm.prec != PREC_FP64
    split = prm.learned_split and prm.guess.kind == GUESS_MLP
    if not (guard or split):
        prm.defer = None
        return None
    if defer is None:
        defer = defer_workspace(n_patch, device)
    elif defer.dtype != torch.int64 or defer.numel() < 2 * n_patch + 4 or not defer.is_cuda:
        raise ValueError("defer must be a CUDA int64 tensor of at least 2 n_patch + 4 words")
    prm.defer = defer.data_ptr()
    return defer


def _params(theta, riemann, prec, max_retry, guess, sched, energy=ENERGY_REDUCED, integrator=MHM,
            flux_out=None, gamma=None):
    prm = srhd_step_params()
    prm.theta = float(theta)
    prm.riemann = int(riemann)
    prm.prec = int(prec)
    prm.max_retry = int(max_retry)
    prm.guess = guess if guess is not None else srhd_guess(GUESS_ANALYTIC, None, 0)
    prm.sched = sched.c() if sched is not None else srhd_sched(0, 1, 0, None)
    prm.energy = int(energy)
    prm.integrator = int(integrator)
    prm.flux_out = None if flux_out is None else flux_out.data_ptr()
    prm.eos = _eos(gamma)
    return prm


def srhd_step_occupancy(prec, guess_kind=GUESS_ANALYTIC, gather=False, occupancy=0,
                        energy=ENERGY_REDUCED, integrator=MHM, gamma=None):
    prm = _params(1.5, HLLC, prec, 4, srhd_guess(int(guess_kind), None, 0), None, energy,
                  integrator, gamma=gamma)
    prm.sched = srhd_sched(0, 1, int(occupancy), None)
    rc = _lib.srhd_step_occupancy(ctypes.byref(prm), int(bool(gather)))
    _check(min(rc, 0))
    return rc


def _table(table, n):
    return [(table[i].groups, table[i].chunk, table[i].occupancy, table[i].ms) for i in range(n.value)]


def srhd_autotune_step(padded, dt_lev, dh, level=None, out=None, theta=1.5, riemann=HLLC,
                       prec=PREC_FP64, max_retry=4, ghost=None, guess=None, reps=2,
                       energy=ENERGY_REDUCED, integrator=MHM, kappa_max=KAPPA_MAX_DEFAULT,
                       defer=None, learned_split=True):
    """Times the candidate schedules of srhd_fluid_step on these patches; returns (Sched of the
    fastest, [(groups, chunk, occupancy, ms per step), ...])."""
    _need_cuda(padded, dt_lev, level)
    P = padded.shape[0]
    if out is None:
        out = torch.empty((P, 5, 8, 8, 8), dtype=torch.float64, device=padded.device)
    sch = Sched(0, 1, padded.device)
    d = _patches(padded, dh, level, ghost)
    prm = _params(theta, riemann, prec, max_retry, guess, sch, energy, integrator)
    ws = _guard(prm, kappa_max, defer, P, padded.device, learned_split)  # noqa: F841
    table = (srhd_tune_entry * 32)()
    n = _int(0)
    _check(_lib.srhd_autotune_step(ctypes.byref(d), _ptr(out), _ptr(dt_lev), ctypes.byref(prm),
                                   int(reps), table, 32, ctypes.byref(n), _stream()))
    sch.groups, sch.chunk, sch.occupancy = prm.sched.groups, prm.sched.chunk, prm.sched.occupancy
    return sch, _table(table, n)


def _grid(cons, prims, neighbor, dh, level, net_mask=None):
    gr = srhd_grid()
    gr.n_patch = cons.shape[0]
    gr.cons = cons.data_ptr()
    gr.prims = prims.data_ptr()
    gr.neighbor = neighbor.data_ptr()
    gr.level = None if level is None else level.data_ptr()
    gr.net_mask = None if net_mask is None else net_mask.data_ptr()
    dh = [float(x) for x in dh]
    gr.n_level = len(dh)
    for i, h in enumerate(dh):
        gr.dh[i] = h
    return gr


def srhd_autotune_step_grid(cons, prims, neighbor, dh, smax_in=None, c_cfl=0.5, dt_lev=None,
                            level=None, theta=1.5, riemann=HLLC, prec=PREC_FP64, max_retry=4,
                            guess=None, reps=2, kappa_max=KAPPA_MAX_DEFAULT, defer=None,
                            learned_split=True, net_in=None, integrator=MHM):
    """Times the candidate schedules of srhd_fluid_step_grid on this block; returns (Sched of
    the fastest, [(groups, chunk, occupancy, ms per step), ...])."""
    _need_cuda(cons, prims, neighbor, smax_in, dt_lev, level, net_in)
    cons_out = torch.empty_like(cons)
    prims_out = torch.empty_like(prims)
    smax_out = torch.empty(1, dtype=torch.int64, device=cons.device)
    net_out = None if net_in is None else torch.empty_like(net_in)
    sch = Sched(0, 1, cons.device)
    gr = _grid(cons, prims, neighbor, dh, level, net_in)
    prm = _params(theta, riemann, prec, max_retry, guess, sch, integrator=integrator)
    ws = _guard(prm, kappa_max, defer, cons.shape[0], cons.device, learned_split)  # noqa: F841
    table = (srhd_tune_entry * 32)()
    n = _int(0)
    _check(_lib.srhd_autotune_step_grid(ctypes.byref(gr), _ptr(smax_in), float(c_cfl), _ptr(dt_lev),
                                        _ptr(cons_out), _ptr(prims_out), _ptr(smax_out),
                                        _ptr(net_out), ctypes.byref(prm), int(reps), table, 32,
                                        ctypes.byref(n), _stream()))
    sch.groups, sch.chunk, sch.occupancy = prm.sched.groups, prm.sched.chunk, prm.sched.occupancy
    return sch, _table(table, n)


def srhd_fluid_step(padded, dt_lev, dh, level=None, out=None, theta=1.5, riemann=HLLC,
                    prec=PREC_FP64, max_retry=4, stats=None, ghost=None, guess=None, sched=None,
                    energy=ENERGY_REDUCED, integrator=MHM, flux_out=None, gamma=None,
                    kappa_max=KAPPA_MAX_DEFAULT, defer=None, learned_split=True):
    """One MUSCL-Hancock (or, integrator=VL, VL) step: padded cons [P][5][N][N][N] -> interior
    [P][5][8][8][8].  energy=ENERGY_TOTAL runs the original scheme on (D, M, E); flux_out
    ([P][6][5][64] FP64) receives the fluxes through the patch faces; gamma selects the
    polytropic EoS.  With an FP32 bulk (prec MIXED or FP32) the precision guard steps the patches
    holding a cell with 1 + M^2 > kappa_max in FP64 (0 turns it off); with a learned guess and
    learned_split the network runs only in a second launch over the patches that consult it;
    defer (int64, >= 2 P + 4 words) is their workspace, allocated per call when None."""
    _need_cuda(padded, dt_lev, level, stats, flux_out)
    P = padded.shape[0]
    N = padded.shape[-1]
    g = (N - 8) // 2 if ghost is None else ghost
    if out is None:
        out = torch.empty((P, 5, 8, 8, 8), dtype=torch.float64, device=padded.device)
    _need_cuda(out)
    d = _patches(padded, dh, level, g)
    prm = _params(theta, riemann, prec, max_retry, guess, sched, energy, integrator, flux_out, gamma)
    ws = _guard(prm, kappa_max, defer, P, padded.device, learned_split)  # noqa: F841
    _check(_lib.srhd_fluid_step(ctypes.byref(d), _ptr(out), _ptr(dt_lev), ctypes.byref(prm),
                                _ptr(stats), _stream()))
    return out


STATIC_MAX_PATCH = 1048576


def srhd_fluid_step_static(padded, dt_lev, dh, level=None, out=None, theta=1.5, riemann=HLLC,
                           prec=PREC_FP64, max_retry=4, stats=None, ghost=None, guess=None,
                           groups=0, chunk=1, occupancy=0, kappa_max=KAPPA_MAX_DEFAULT,
                           learned_split=True):
    """srhd_fluid_step without caller work buffers: the precision guard's list and the persistent
    schedule's counters live in the library's static device array (at most STATIC_MAX_PATCH
    patches; concurrent calls on one GPU race).  `out` must be supplied by a caller that cannot
    allocate; it is allocated here only for convenience."""
    _need_cuda(padded, dt_lev, level, stats)
    P = padded.shape[0]
    N = padded.shape[-1]
    g = (N - 8) // 2 if ghost is None else ghost
    if out is None:
        out = torch.empty((P, 5, 8, 8, 8), dtype=torch.float64, device=padded.device)
    _need_cuda(out)
    d = _patches(padded, dh, level, g)
    prm = _params(theta, riemann, prec, max_retry, guess, None)
    prm.sched = srhd_sched(int(groups), int(chunk), int(occupancy), None)
    prm.kappa_max = float(kappa_max)
    prm.learned_split = int(bool(learned_split))
    prm.defer = None
    _check(_lib.srhd_fluid_step_static(ctypes.byref(d), _ptr(out), _ptr(dt_lev),
                                       ctypes.byref(prm), _ptr(stats), _stream()))
    return out


def prims_dtype(prec):
    return torch.float64 if prec == PREC_FP64 else torch.float32


def new_net_mask(n_patch, device):
    """Network masks of a gather-layout state (int32 [n_patch]): bit (rz + 1) 9 + (ry + 1) 3 +
    (rx + 1) of patch p marks a cell with L above the learned guess's gate in region (rx, ry,
    rz) of the patch (per axis 0: every cell, -1 / +1: the two lowest / highest layers)."""
    return torch.zeros(max(int(n_patch), 1), dtype=torch.int32, device=device)


def _need_mask(m, P):
    if m is not None and (m.dtype != torch.int32 or m.numel() < P):
        raise ValueError("a network mask array is int32 with at least %d entries" % P)


def srhd_grid_prims(cons, prec=PREC_FP64, prims=None, smax_bits=None, guess=None, net_mask=None):
    """Interior cons [P][5][8][8][8] -> (prims in the step's bulk type, S_max bits int64 [1]);
    net_mask (int32 [P]) receives the state's network masks."""
    _need_cuda(cons, net_mask)
    P = cons.shape[0]
    if prims is None:
        prims = torch.empty(cons.shape, dtype=prims_dtype(prec), device=cons.device)
    if smax_bits is None:
        smax_bits = torch.empty(1, dtype=torch.int64, device=cons.device)
    _need_cuda(prims, smax_bits)
    g = guess if guess is not None else srhd_guess(GUESS_ANALYTIC, None, 0)
    _need_mask(net_mask, P)
    _check(_lib.srhd_grid_prims(int(prec), P, _ptr(cons), _ptr(prims), _ptr(smax_bits),
                                _ptr(net_mask), ctypes.byref(g), _stream()))
    return prims, smax_bits


def smax_value(bits):
    """The double whose bit pattern is stored in an int64 tensor."""
    return bits.cpu().view(torch.float64).item()


def srhd_fluid_step_grid(cons, prims, neighbor, dh, smax_in=None, c_cfl=0.5, dt_lev=None,
                         level=None, cons_out=None, prims_out=None, smax_out=None, dt_used=None,
                         theta=1.5, riemann=HLLC, prec=PREC_FP64, max_retry=4, stats=None,
                         guess=None, sched=None, gamma=None, kappa_max=KAPPA_MAX_DEFAULT,
                         defer=None, learned_split=True, net_in=None, net_out=None,
                         integrator=MHM):
    """One MUSCL-Hancock (or, integrator=VL, VL) step of a block of same-level patches (ghosts
    gathered from neighbour interiors).  net_in: the input state's network masks (with a learned guess and learned_split they fix the
    split's list before the step, which then runs both kernels concurrently); net_out receives
    the output's.  Returns (cons_out, prims_out, smax_out)."""
    _need_cuda(cons, prims, neighbor, smax_in, dt_lev, level, stats, net_in, net_out)
    P = cons.shape[0]
    if cons_out is None:
        cons_out = torch.empty_like(cons)
    if prims_out is None:
        prims_out = torch.empty(cons.shape, dtype=prims_dtype(prec), device=cons.device)
    if smax_out is None:
        smax_out = torch.empty(1, dtype=torch.int64, device=cons.device)
    _need_cuda(cons_out, prims_out, smax_out, dt_used)
    if prims.dtype != prims_dtype(prec) or prims_out.dtype != prims_dtype(prec):
        raise TypeError("primitives must be %s for this precision" % prims_dtype(prec))
    _need_mask(net_in, P)
    _need_mask(net_out, P)
    gr = _grid(cons, prims, neighbor, dh, level, net_in)
    prm = _params(theta, riemann, prec, max_retry, guess, sched, integrator=integrator,
                  gamma=gamma)
    ws = _guard(prm, kappa_max, defer, P, cons.device, learned_split)  # noqa: F841
    _check(_lib.srhd_fluid_step_grid(ctypes.byref(gr), _ptr(smax_in), float(c_cfl), _ptr(dt_lev),
                                     _ptr(cons_out), _ptr(prims_out), _ptr(smax_out),
                                     _ptr(net_out), _ptr(dt_used), ctypes.byref(prm), _ptr(stats),
                                     _stream()))
    return cons_out, prims_out, smax_out


# ------------------------------------------------------------------------------- learned guess
class Mlp:
    """Device parameters of the learned guess plus the ctypes descriptors that point at them.

    w: uint16 BF16 weights [4352] (W1[64][3], W2[64][64], W3[64]); bias: float32 [129];
    norm: float32 [8] (input mean[3], input std[3], output mean, output std); features: FEAT_CONS
    or FEAT_L; gate: the network is consulted for states with L > gate only."""

    def __init__(self, w, bias, norm, features=FEAT_CONS, gate=0.0):
        self.w, self.bias, self.norm = w, bias, norm
        self.features, self.gate = int(features), float(gate)
        _need_cuda(w, bias, norm)
        if w.data_ptr() % 16:
            raise ValueError("weights must be 16-byte aligned")
        self.desc = srhd_mlp(w.data_ptr(), bias.data_ptr(), norm.data_ptr(), self.features,
                             self.gate)

    def guess(self, max_iter=0):
        g = srhd_guess(GUESS_MLP, ctypes.pointer(self.desc), max_iter)
        g._keep = self        # keep the parameters alive with the descriptor
        return g


def srhd_mlp_features(cons, prim=None, feat=None, target=None, features=FEAT_CONS):
    """cons [5][n] (and optionally prim [5][n]) -> feat float32 [3][n] (and target log ht [n])."""
    _need_cuda(cons, prim)
    n = cons.shape[-1]
    if feat is None:
        feat = torch.empty((3, n), dtype=torch.float32, device=cons.device)
    if prim is not None and target is None:
        target = torch.empty(n, dtype=torch.float32, device=cons.device)
    _check(_lib.srhd_mlp_features(_dtype_code(cons), int(features), n, _ptr(cons), _ptr(prim),
                                  _ptr(feat), _ptr(target), _stream()))
    return feat, target


def srhd_mlp_forward(mlp, feat, y=None):
    _need_cuda(feat)
    n = feat.shape[-1]
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=feat.device)
    _check(_lib.srhd_mlp_forward(ctypes.byref(mlp.desc), n, _ptr(feat), _ptr(y), _stream()))
    return y


def srhd_mlp_workspace_bytes(batch):
    return int(_lib.srhd_mlp_workspace_bytes(int(batch)))


def srhd_mlp_grad(mlp, feat, target, grad=None, loss=None, ws=None):
    _need_cuda(feat, target)
    n = feat.shape[-1]
    dev = feat.device
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if ws is None:
        ws = torch.empty(srhd_mlp_workspace_bytes(n), dtype=torch.uint8, device=dev)
    _check(_lib.srhd_mlp_grad(ctypes.byref(mlp.desc), n, _ptr(feat), _ptr(target), _ptr(grad),
                              _ptr(loss), _ptr(ws), _stream()))
    return grad, loss


def srhd_mlp_adam(master, m1, m2, grad, step, lr, mlp):
    _check(_lib.srhd_mlp_adam(_ptr(master), _ptr(m1), _ptr(m2), _ptr(grad), int(step),
                              float(lr), _ptr(mlp.w), _ptr(mlp.bias), _stream()))


def abi_version():
    return _lib.srhd_abi_version()


# ---------------------------------------------------------------- AMR neighbour operations
NB_COARSE = -2


def srhd_fill_ghosts_coarse(fine_padded, neighbor, parent, octant, coarse_old, coarse_new=None,
                            alpha=0.0, theta=1.5, counts=None):
    """Fills, in place, the ghost cells of fine_padded [Pf][5][N][N][N] whose neighbour slot is
    NB_COARSE from the padded parents coarse_old (and coarse_new, time weight alpha).  counts: an
    optional uint64 [2] device tensor accumulating (interpolated cells, primitive fallbacks)."""
    _need_cuda(fine_padded, neighbor, parent, octant, coarse_old, coarse_new, counts)
    g = (fine_padded.shape[-1] - 8) // 2
    gc = (coarse_old.shape[-1] - 8) // 2
    _check(_lib.srhd_fill_ghosts_coarse(fine_padded.shape[0], g, _ptr(neighbor), _ptr(parent),
                                        _ptr(octant), coarse_old.shape[0], gc, _ptr(coarse_old),
                                        _ptr(coarse_new), float(alpha), float(theta),
                                        _ptr(fine_padded), _ptr(counts), _stream()))
    return fine_padded


def srhd_restrict(coarse, parent_of, child, fine):
    """coarse[parent_of[q]] = average of the children child[q][0..7] of fine, in place."""
    _need_cuda(coarse, parent_of, child, fine)
    _check(_lib.srhd_restrict(parent_of.shape[0], _ptr(parent_of), _ptr(child), fine.shape[0],
                              _ptr(fine), coarse.shape[0], _ptr(coarse), _stream()))
    return coarse


def srhd_flux_accumulate(acc, flux, beta, weight):
    """acc = beta * acc + weight * flux (same shapes, FP64)."""
    _need_cuda(acc, flux)
    _check(_lib.srhd_flux_accumulate(acc.numel(), _ptr(acc), _ptr(flux), float(beta), float(weight),
                                     _stream()))
    return acc


def srhd_flux_correct(coarse, faces, coarse_flux, fine_flux, dh_c, skipped=None):
    """Coarse-fine flux correction of coarse [Pc][5][8][8][8] in place; faces int32 [n][6]."""
    _need_cuda(coarse, faces, coarse_flux, fine_flux, skipped)
    _check(_lib.srhd_flux_correct(faces.shape[0], _ptr(faces), coarse.shape[0], _ptr(coarse),
                                  _ptr(coarse_flux), fine_flux.shape[0], _ptr(fine_flux),
                                  float(dh_c), _ptr(skipped), _stream()))
    return coarse
