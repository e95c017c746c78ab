"""Error metrics shared by the parity tests (numpy, host side)."""
import numpy as np

import oracle as O


def prim_errors(gpu, ref, ok):
    """Per-field relative errors of primitive states [5][n] over the mask ok:
    rho and p pointwise relative; U normwise per state, max|dU_i| / max(|U|, 1e-300)."""
    g, r = gpu[:, ok], ref[:, ok]
    e = {}
    e["rho"] = np.max(np.abs(g[0] / r[0] - 1)) if g.shape[1] else 0.0
    e["p"] = np.max(np.abs(g[4] / r[4] - 1)) if g.shape[1] else 0.0
    un = np.maximum(np.sqrt((r[1:4] ** 2).sum(axis=0)), 1e-300)
    e["U"] = np.max(np.max(np.abs(g[1:4] - r[1:4]), axis=0) / un) if g.shape[1] else 0.0
    return e


def step_errors(gpu, ref):
    """One-step output [P][5][8][8][8]: pointwise relative for D and Et (both positive);
    each momentum component normwise against the grid maximum of |M| (a component that is zero
    in exact arithmetic carries only round-off, so its own maximum is no scale)."""
    e = {}
    e["D"] = float(np.max(np.abs(gpu[:, 0] / ref[:, 0] - 1)))
    e["Et"] = float(np.max(np.abs(gpu[:, 4] / ref[:, 4] - 1)))
    scale = max(float(np.max(np.sqrt((ref[:, 1:4] ** 2).sum(axis=1)))), 1e-300)
    for k, name in ((1, "Mx"), (2, "My"), (3, "Mz")):
        e[name] = float(np.max(np.abs(gpu[:, k] - ref[:, k]))) / scale
    return e


def soa(a):
    """[P][5][8][8][8] -> [5][P*512]."""
    P = a.shape[0]
    return np.ascontiguousarray(a.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1))


def unsoa(a, P):
    return np.ascontiguousarray(a.reshape(5, P, 512).transpose(1, 0, 2).reshape(P, 5, 8, 8, 8))


def oracle_cons(grid):
    return unsoa(O.prim2cons(soa(grid.prim)), grid.n_patch)


# ----------------------------------------------------------------------------- Eq. 20 bounds
U32 = 2.0 ** -24          # unit roundoff of FP32
U64 = 2.0 ** -53          # unit roundoff of FP64


def kappa_prim(prim):
    """Eq. 20's conversion condition number 1 + M^2 of primitive states [5][...] (rho, U, p),
    M = U / U_s the Mach number in four-velocities, U_s^2 = c_s^2 / (1 - c_s^2)."""
    rho, p = prim[0], prim[4]
    th = (p / rho).ravel()
    uniq, inv = np.unique(th, return_inverse=True)
    cs2 = np.array([O.cs2(t) for t in uniq])[inv].reshape(rho.shape)
    u2 = prim[1] ** 2 + prim[2] ** 2 + prim[3] ** 2
    return 1.0 + u2 * (1.0 - cs2) / cs2


def stencil_mask():
    """The cells of a patch's [-2, 10)^3 box that one MUSCL-Hancock step reads: the half-step
    cells (the interior and the first ghost layer across each face) and their face neighbours.
    Boolean [12][12][12] indexed [z][y][x]."""
    def half(i, j, k):
        out = 0
        for c in (i, j, k):
            if 0 <= c < 8:
                continue
            if c in (-1, 8):
                out += 1
            else:
                return False
        return out <= 1
    m = np.zeros((12, 12, 12), dtype=bool)
    for k in range(-2, 10):
        for j in range(-2, 10):
            for i in range(-2, 10):
                m[k + 2, j + 2, i + 2] = any(half(i + a, j + b, k + c) for a, b, c in
                                             ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0),
                                              (0, -1, 0), (0, 0, 1), (0, 0, -1)))
    return m


def tile_max(q, neighbor):
    """Per patch, the largest value of a per-cell quantity q [P][8][8][8] over the cells its
    step reads (ghost cells by the oracle's fill: periodic / outflow copies)."""
    P = q.shape[0]
    five = np.zeros((P, 5, 8, 8, 8))
    five[:, 0] = q
    pad = O.fill_ghosts(five, neighbor, 2)[:, 0]
    m = stencil_mask()
    return pad.reshape(P, -1)[:, m.ravel()].max(axis=1)


def patch_errors(gpu, ref):
    """Per patch [P]: the largest of the pointwise relative errors of D and Et and of the momentum
    errors against the grid maximum of |M| (the metric of step_errors, patch by patch)."""
    eD = np.max(np.abs(gpu[:, 0] / ref[:, 0] - 1).reshape(gpu.shape[0], -1), axis=1)
    eE = np.max(np.abs(gpu[:, 4] / ref[:, 4] - 1).reshape(gpu.shape[0], -1), axis=1)
    scale = max(float(np.max(np.sqrt((ref[:, 1:4] ** 2).sum(axis=1)))), 1e-300)
    eM = np.max(np.abs(gpu[:, 1:4] - ref[:, 1:4]).reshape(gpu.shape[0], -1), axis=1) / scale
    return np.maximum(np.maximum(eD, eE), eM)


# one-step error bound of a step per patch, (C_KAPPA kappa_tile + C_FLUX) u with u the unit
# roundoff of the bulk arithmetic (the derivation is in tests/test_gpu_guard.py)
C_KAPPA = 16.0
C_FLUX = 32.0


def step_bound(kappa_tile, u=U32):
    return (C_KAPPA * np.asarray(kappa_tile) + C_FLUX) * u


def _stencil_cells(pad):
    """[P][5][1376]: the cells of padded patches [P][5][N][N][N] that one step reads."""
    P, N = pad.shape[0], pad.shape[-1]
    g = (N - 8) // 2
    box = pad[:, :, g - 2:g + 10, g - 2:g + 10, g - 2:g + 10].reshape(P, 5, -1)
    return box[:, :, stencil_mask().ravel()]


def kappa_tile_padded(pad, whole=False):
    """Per patch [P]: the largest kappa = 1 + M^2 over the cells its MUSCL-Hancock step reads (or,
    whole=True, over every padded cell: the VL step reads a third ghost layer), from padded
    conserved patches (reduced energy) by the oracle's inversion; unphysical cells are skipped."""
    cells = pad.reshape(pad.shape[0], 5, -1) if whole else _stencil_cells(pad)
    P = cells.shape[0]
    prim, st, _ = O.cons2prim(np.ascontiguousarray(cells.transpose(1, 0, 2).reshape(5, -1)))
    k = kappa_prim(prim).reshape(P, -1)
    k[(st == 1).reshape(P, -1)] = 1.0
    return np.nanmax(np.where(np.isfinite(k), k, 1.0), axis=1)


def cond_total_tile_padded(pad):
    """Per patch [P]: the largest condition number of the original scheme's L = x^2 - m^2 - 1
    (x = E/D, m = |M|/D; Eq. 21's amplification) over the cells its step reads, from padded
    total-energy patches: (x^2 + m^2 + 1) / |x^2 - m^2 - 1|."""
    c = _stencil_cells(pad)
    x2 = (c[:, 4] / c[:, 0]) ** 2
    m2 = (c[:, 1] ** 2 + c[:, 2] ** 2 + c[:, 3] ** 2) / c[:, 0] ** 2
    with np.errstate(divide="ignore"):
        k = (x2 + m2 + 1.0) / np.abs(x2 - m2 - 1.0)
    return k.max(axis=1)
