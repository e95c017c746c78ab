"""Multi-step driver over the CPU oracle (test helper): prims -> cons, then per step
CFL time step (Eqs. 26-28), ghost fill and one MUSCL-Hancock step."""
import numpy as np

import oracle as O


def initial_cons(grid):
    P = grid.n_patch
    prim = grid.prim.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1)
    cons = O.prim2cons(prim)
    return np.ascontiguousarray(cons.reshape(5, P, 512).transpose(1, 0, 2)).reshape(P, 5, 8, 8, 8)


def to_prim(cons):
    P = cons.shape[0]
    c = cons.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1)
    w, st, _ = O.cons2prim(c)
    return w.reshape(5, P, 512).transpose(1, 0, 2).reshape(P, 5, 8, 8, 8), st


def run(grid, cons, n_steps=None, t_end=None, c_cfl=0.5, theta=1.5, solver=O.HLLC, ghost=3,
        dt_fixed=None, stats=None):
    """Advance ``cons`` [P][5][8][8][8]; returns (cons, time, steps).  ``stats`` (a list)
    receives the per-step oracle counters."""
    t, k = 0.0, 0
    while True:
        if n_steps is not None and k >= n_steps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        if dt_fixed is None:
            dt_lev, _, _ = O.cfl_dt(cons, None, grid.dh_lev, c_cfl)
            dt = dt_lev[0]
        else:
            dt = dt_fixed
        if t_end is not None:
            dt = min(dt, t_end - t)
        pad = O.fill_ghosts(cons, grid.neighbor, ghost)
        cons, cnt = O.fluid_step(pad, [dt], grid.dh_lev, None, theta, solver, ghost)
        assert cnt[0] == 0, "unphysical inversion"
        if stats is not None:
            stats.append(cnt)
        t += dt
        k += 1
    return cons, t, k
