"""CPU oracle for the SRHD step (arXiv:2012.11130): plain, slow, FP64.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` import this package.  It shares no code with the HIP library and never imports
it.  The scalar C core is ``srhd_oracle.c``; this module loads it with ctypes and adds numpy
batch wrappers.  Each C function cites the passage of the paper it follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ST_OK, ST_UNPHYSICAL, ST_FALLBACK, ST_NOCONV = 0, 1, 2, 3
HLLC, HLLE = 0, 1

_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    scal = {
        "or_h_of_theta": [_d], "or_htilde_of_theta": [_d], "or_theta_of_htilde": [_d],
        "or_dtheta_dhtilde": [_d], "or_cs2": [_d], "or_f_given_theta": [_d, _d, _d],
        "or_f": [_d, _d], "or_dfdh": [_d, _d], "or_guess_cold": [_d, _d], "or_guess_hot": [_d],
        "or_guess_threshold": [_d], "or_guess_analytic": [_d, _d],
        "or_L_exact": [_d] * 5, "or_L_naive": [_d] * 5, "or_L_total_energy": [_d] * 5,
        "or_slope": [_d, _d, _d, _d],
    }
    for name, args in scal.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _d
    L.or_sum_exact.argtypes = [_p, ctypes.c_int]
    L.or_sum_exact.restype = _d
    L.or_solve_htilde.argtypes = [_d, _d, ctypes.POINTER(ctypes.c_int)]
    L.or_solve_htilde.restype = _d
    L.or_prim2cons_one.argtypes = [_p, _p]
    L.or_prim2cons_one.restype = None
    L.or_cons2prim_one.argtypes = [_p, _p, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int)]
    L.or_cons2prim_one.restype = ctypes.c_int
    L.or_prim2cons.argtypes = [_i64, _p, _p]
    L.or_prim2cons.restype = None
    L.or_cons2prim.argtypes = [_i64, _p, _p, _p, _p]
    L.or_cons2prim.restype = None
    L.or_L_batch.argtypes = [_i64, _p, ctypes.c_int, _p]
    L.or_L_batch.restype = None
    L.or_smax_prim.argtypes = [_p]
    L.or_smax_prim.restype = _d
    L.or_patch_smax.argtypes = [_i64, _p, _p, ctypes.POINTER(_i64)]
    L.or_patch_smax.restype = None
    L.or_flux.argtypes = [ctypes.c_int, _p, _p, _p]
    L.or_flux.restype = None
    L.or_wavespeeds.argtypes = [ctypes.c_int, _p, ctypes.POINTER(_d), ctypes.POINTER(_d)]
    L.or_wavespeeds.restype = None
    for name in ("or_hlle", "or_hllc"):
        fn = getattr(L, name)
        fn.argtypes = [ctypes.c_int, _p, _p, _p]
        fn.restype = None
    L.or_fluid_step.argtypes = [_i64, ctypes.c_int, _p, _p, _p, _p, _d, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, _p, _p, _p]
    L.or_fill_ghosts_coarse.argtypes = [_i64, ctypes.c_int, _p, _p, _p, _i64, ctypes.c_int, _p, _p,
                                        _d, _d, _p, _p]
    L.or_fill_ghosts_coarse.restype = ctypes.c_int
    L.or_set_eos.argtypes = [_d]
    L.or_set_eos.restype = ctypes.c_int
    L.or_get_eos.argtypes = []
    L.or_get_eos.restype = _d
    L.or_restrict.argtypes = [_i64, _p, _p, _p, _p]
    L.or_restrict.restype = None
    L.or_flux_correct.argtypes = [_i64, _p, _p, _p, _p, _d]
    L.or_flux_correct.restype = _i64
    L.or_prim2cons_total.argtypes = [_i64, _p, _p]
    L.or_prim2cons_total.restype = None
    L.or_cons2prim_total_one.argtypes = [_p, _p, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int)]
    L.or_cons2prim_total_one.restype = ctypes.c_int
    L.or_is_physical.argtypes = [_p]
    L.or_is_physical.restype = ctypes.c_int
    L.or_fluid_step.restype = ctypes.c_int
    L.or_fill_ghosts.argtypes = [_i64, ctypes.c_int, _i64, _p, _p, _p]
    L.or_fill_ghosts.restype = ctypes.c_int
    L.or_extract_interior.argtypes = [_i64, ctypes.c_int, _p, _p]
    L.or_extract_interior.restype = None
    L.or_num_threads.argtypes = []
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_num_threads.argtypes = [ctypes.c_int]
    L.or_set_num_threads.restype = None
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- scalar EoS / inversion pieces
def h_of_theta(th): return lib().or_h_of_theta(float(th))
def htilde_of_theta(th): return lib().or_htilde_of_theta(float(th))
def theta_of_htilde(ht): return lib().or_theta_of_htilde(float(ht))
def dtheta_dhtilde(ht): return lib().or_dtheta_dhtilde(float(ht))
def cs2(th): return lib().or_cs2(float(th))
def f_given_theta(ht, th, m2): return lib().or_f_given_theta(float(ht), float(th), float(m2))
def f(ht, m2): return lib().or_f(float(ht), float(m2))
def dfdh(ht, m2): return lib().or_dfdh(float(ht), float(m2))
def guess_cold(L, m2): return lib().or_guess_cold(float(L), float(m2))
def guess_hot(L): return lib().or_guess_hot(float(L))
def guess_threshold(m2): return lib().or_guess_threshold(float(m2))
def guess_analytic(L, m2): return lib().or_guess_analytic(float(L), float(m2))
def slope(wl, wc, wr, theta): return lib().or_slope(float(wl), float(wc), float(wr), float(theta))


def L_exact(D, Mx, My, Mz, Et):
    return lib().or_L_exact(float(D), float(Mx), float(My), float(Mz), float(Et))


def L_naive(D, Mx, My, Mz, Et):
    return lib().or_L_naive(float(D), float(Mx), float(My), float(Mz), float(Et))


def L_total_energy(D, Mx, My, Mz, E):
    return lib().or_L_total_energy(float(D), float(Mx), float(My), float(Mz), float(E))


def sum_exact(xs):
    a = _f64(xs)
    return lib().or_sum_exact(_ptr(a), int(a.size))


def solve_htilde(L, m2):
    it = ctypes.c_int(0)
    r = lib().or_solve_htilde(float(L), float(m2), ctypes.byref(it))
    return r, it.value


def is_physical(u):
    u = _f64(u)
    return bool(lib().or_is_physical(_ptr(u)))


def prim2cons_one(w):
    w = _f64(w)
    u = np.empty(5)
    lib().or_prim2cons_one(_ptr(w), _ptr(u))
    return u


def cons2prim_one(u):
    u = _f64(u)
    w = np.empty(5)
    ht = ctypes.c_double(0)
    it = ctypes.c_int(0)
    st = lib().or_cons2prim_one(_ptr(u), _ptr(w), ctypes.byref(ht), ctypes.byref(it))
    return w, st, ht.value, it.value


def smax_prim(w):
    w = _f64(w)
    return lib().or_smax_prim(_ptr(w))


def flux(d, w):
    w = _f64(w)
    u = prim2cons_one(w)
    F = np.empty(5)
    lib().or_flux(int(d), _ptr(w), _ptr(u), _ptr(F))
    return F


def wavespeeds(d, w):
    w = _f64(w)
    lm, lp = ctypes.c_double(0), ctypes.c_double(0)
    lib().or_wavespeeds(int(d), _ptr(w), ctypes.byref(lm), ctypes.byref(lp))
    return lm.value, lp.value


def riemann(d, wl, wr, solver=HLLC):
    wl, wr = _f64(wl), _f64(wr)
    F = np.empty(5)
    fn = lib().or_hllc if solver == HLLC else lib().or_hlle
    fn(int(d), _ptr(wl), _ptr(wr), _ptr(F))
    return F


# ---------------------------------------------------------------- batch forms
def prim2cons(prim, scheme=0):
    """prim [5][n] (rho, Ux, Uy, Uz, p) -> cons [5][n] (D, Mx, My, Mz, Et), FP64; with scheme=1
    the original scheme's (D, Mx, My, Mz, E), E the total energy of Eq. 5c."""
    prim = _f64(prim)
    n = prim.shape[-1]
    cons = np.empty_like(prim)
    (lib().or_prim2cons_total if scheme else lib().or_prim2cons)(n, _ptr(prim), _ptr(cons))
    return cons


def cons2prim_total_one(u):
    """Original scheme: (D, M, E) -> (prim, status) with the naive L of Eq. 21."""
    u = _f64(u)
    w = np.empty(5)
    ht = ctypes.c_double()
    it = ctypes.c_int()
    st = lib().or_cons2prim_total_one(_ptr(u), _ptr(w), ctypes.byref(ht), ctypes.byref(it))
    return w, st


def cons2prim(cons):
    """cons [5][n] -> (prim [5][n], status int8 [n], bracketed-solver iterations int32 [n])."""
    cons = _f64(cons)
    n = cons.shape[-1]
    prim = np.empty_like(cons)
    st = np.empty(n, dtype=np.int8)
    it = np.empty(n, dtype=np.int32)
    lib().or_cons2prim(n, _ptr(cons), _ptr(prim), _ptr(st), _ptr(it))
    return prim, st, it


def L_batch(cons, mode="exact"):
    cons = _f64(cons)
    n = cons.shape[-1]
    out = np.empty(n)
    lib().or_L_batch(n, _ptr(cons), {"exact": 0, "naive": 1, "total": 2}[mode], _ptr(out))
    return out


def patch_smax(interior):
    """Max signal speed (Eqs. 26-27) over each patch of interior cons [P][5][512]."""
    interior = _f64(interior)
    P = interior.shape[0]
    s = np.empty(P)
    bad = ctypes.c_int64(0)
    lib().or_patch_smax(P, _ptr(interior), _ptr(s), ctypes.byref(bad))
    return s, bad.value


def cfl_dt(interior, level, dh_lev, c_cfl=0.5):
    """Eq. 28 with one global S_max: dt_l = C dh_l / max S_max (so dt_l = dt_0 / 2^l)."""
    s, bad = patch_smax(interior)
    smax = float(np.max(s)) if s.size else 0.0
    dh_lev = np.asarray(dh_lev, dtype=np.float64)
    return np.array([c_cfl * h / smax for h in dh_lev]), smax, bad


def fill_ghosts(interior, neighbor, ghost=3):
    """Padded patches for the rows of ``neighbor`` (slot 13 = own index into ``interior``)."""
    interior = _f64(interior)
    neighbor = np.ascontiguousarray(neighbor, dtype=np.int32)
    P = neighbor.shape[0]
    N = 8 + 2 * ghost
    padded = np.empty((P, 5, N, N, N))
    rc = lib().or_fill_ghosts(P, ghost, interior.shape[0], _ptr(interior), _ptr(neighbor),
                              _ptr(padded))
    if rc != 0:
        raise ValueError("neighbour table leaves a ghost cell without a source")
    return padded


def extract_interior(padded, ghost=3):
    padded = _f64(padded)
    P = padded.shape[0]
    out = np.empty((P, 5, 8, 8, 8))
    lib().or_extract_interior(P, ghost, _ptr(padded), _ptr(out))
    return out


def fluid_step(padded, dt_lev, dh_lev, level=None, theta=1.5, solver=HLLC, ghost=3,
               max_retry=4, scheme=0, integrator=0, bflux=False):
    """One MUSCL-Hancock step of every padded patch [P][5][N][N][N] -> interior [P][5][8][8][8].

    Returns (out, counts) with counts = (unphysical states in the final attempt, non-converged
    inversions, solver iterations, retried patch attempts, VL predictor fallbacks); with
    bflux=True, (out, counts, fluxes [P][6][5][64] through the patch faces in the final attempt).
    """
    padded = _f64(padded)
    P = padded.shape[0]
    out = np.empty((P, 5, 8, 8, 8))
    counts = np.zeros(5, dtype=np.int64)
    bf = np.empty((P, 6, 5, 64)) if bflux else None
    dt_lev = _f64(np.atleast_1d(dt_lev))
    dh_lev = _f64(np.atleast_1d(dh_lev))
    lv = None if level is None else np.ascontiguousarray(level, dtype=np.int8)
    rc = lib().or_fluid_step(P, ghost, _ptr(padded), None if lv is None else _ptr(lv),
                             _ptr(dh_lev), _ptr(dt_lev), float(theta), int(solver),
                             int(max_retry), int(scheme), int(integrator), _ptr(out), _ptr(counts),
                             None if bf is None else _ptr(bf))
    if rc != 0:
        raise ValueError("ghost depth must be at least %d" % (3 if integrator else 2))
    if bflux:
        return out, counts, bf
    return out, counts


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n):
    lib().or_set_num_threads(int(n))


# ---------------------------------------------------------------- AMR neighbour operations
NB_COARSE = -2


def fill_ghosts_coarse(fine_padded, neighbor, parent, octant, coarse_old, coarse_new=None,
                       alpha=0.0, theta=1.5, ghost=3, ghost_c=3):
    """Fill, in place, the ghost cells of fine padded patches whose neighbour slot is NB_COARSE
    by limited linear interpolation from the padded parents (conserved variables; primitive
    variables where the conserved result fails Eq. 30).  Returns (interpolated, fallbacks)."""
    assert fine_padded.flags.c_contiguous and fine_padded.dtype == np.float64
    neighbor = np.ascontiguousarray(neighbor, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    octant = np.ascontiguousarray(octant, dtype=np.int8)
    co = _f64(coarse_old)
    cn = None if coarse_new is None else _f64(coarse_new)
    counts = np.zeros(2, dtype=np.int64)
    rc = lib().or_fill_ghosts_coarse(fine_padded.shape[0], ghost, _ptr(neighbor), _ptr(parent),
                                     _ptr(octant), co.shape[0], ghost_c, _ptr(co),
                                     None if cn is None else _ptr(cn), float(alpha), float(theta),
                                     _ptr(fine_padded), _ptr(counts))
    if rc != 0:
        raise ValueError("bad parent index or too few coarse ghost layers")
    return int(counts[0]), int(counts[1])


def restrict(coarse, parent_of, child, fine):
    """Overwrite coarse[parent_of[p]] with the average of its eight children child[p][0..7]."""
    assert coarse.flags.c_contiguous and coarse.dtype == np.float64
    parent_of = np.ascontiguousarray(parent_of, dtype=np.int32)
    child = np.ascontiguousarray(child, dtype=np.int32)
    fine = _f64(fine)
    lib().or_restrict(parent_of.shape[0], _ptr(parent_of), _ptr(child), _ptr(fine), _ptr(coarse))


def flux_correct(coarse, faces, coarse_flux, fine_flux, dh_c):
    """Coarse-fine flux correction in place; faces [n][6] = (coarse, side, fine[4]).  Returns
    the number of coarse cells left uncorrected because the corrected state fails Eq. 30."""
    assert coarse.flags.c_contiguous and coarse.dtype == np.float64
    faces = np.ascontiguousarray(faces, dtype=np.int32).reshape(-1, 6)
    return int(lib().or_flux_correct(faces.shape[0], _ptr(faces), _ptr(coarse),
                                     _ptr(_f64(coarse_flux)), _ptr(_f64(fine_flux)), float(dh_c)))



# ---------------------------------------------------------------- equation of state
class eos:
    """Context manager selecting the oracle's EoS: eos(0) the TM EoS (the default), eos(Gamma)
    the polytropic EoS h = 1 + Gamma Theta / (Gamma - 1), 1 < Gamma <= 2."""

    def __init__(self, gamma):
        self.gamma = float(gamma)

    def __enter__(self):
        self.prev = lib().or_get_eos()
        if lib().or_set_eos(self.gamma) != 0:
            raise ValueError("Gamma must lie in (1, 2]")
        return self

    def __exit__(self, *exc):
        lib().or_set_eos(self.prev)
        return False
