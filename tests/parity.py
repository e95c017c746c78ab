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
