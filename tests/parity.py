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
