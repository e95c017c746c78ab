"""Multi-step driver over the CPU oracle (test helper): prims -> cons, then per step
CFL time step (Eqs. 26-28), ghost fill and one MUSCL-Hancock step."""
import math

import numpy as np

import oracle as O
import workloads as W


def initial_cons(grid, scheme=0):
    P = grid.n_patch
    prim = grid.prim.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1)
    cons = O.prim2cons(prim, scheme=scheme)
    return np.ascontiguousarray(cons.reshape(5, P, 512).transpose(1, 0, 2)).reshape(P, 5, 8, 8, 8)


def to_prim(cons, scheme=0):
    P = cons.shape[0]
    c = cons.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1)
    if scheme:
        w = np.empty_like(c)
        st = np.empty(c.shape[1], dtype=np.int8)
        for i in range(c.shape[1]):
            w[:, i], st[i] = O.cons2prim_total_one(c[:, i])
    else:
        w, st, _ = O.cons2prim(c)
    return w.reshape(5, P, 512).transpose(1, 0, 2).reshape(P, 5, 8, 8, 8), st


def run(grid, cons, n_steps=None, t_end=None, c_cfl=0.5, theta=1.5, solver=O.HLLC, ghost=3,
        dt_fixed=None, stats=None, scheme=0, integrator=0):
    """Advance ``cons`` [P][5][8][8][8]; returns (cons, time, steps).  ``stats`` (a list)
    receives the per-step oracle counters.  scheme=1 runs the original scheme on (D, M, E); its
    CFL time step is taken from Et = E - D (the time step only needs the signal speeds).
    integrator=1 runs the VL predictor-corrector instead of MUSCL-Hancock."""
    t, k = 0.0, 0
    while True:
        if n_steps is not None and k >= n_steps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        if dt_fixed is None:
            c = cons
            if scheme:
                c = cons.copy()
                c[:, 4] -= c[:, 0]
            dt_lev, _, _ = O.cfl_dt(c, None, grid.dh_lev, c_cfl)
            dt = dt_lev[0]
        else:
            dt = dt_fixed
        if t_end is not None:
            dt = min(dt, t_end - t)
        pad = O.fill_ghosts(cons, grid.neighbor, ghost)
        cons, cnt = O.fluid_step(pad, [dt], grid.dh_lev, None, theta, solver, ghost, scheme=scheme,
                                 integrator=integrator)
        assert cnt[0] == 0, "unphysical inversion"
        if stats is not None:
            stats.append(cnt)
        t += dt
        k += 1
    return cons, t, k


def sine_x_l1(n, theta0, amp, t_frac, theta_lim=1.5, scheme=0, integrator=0):
    """Right-moving linear acoustic wave along x on an n-cell periodic row; returns the L1
    density error (Eq. 31) after t_frac of a period; scheme=1 runs the original scheme."""
    g = W.PatchGrid("w", np.zeros((n // 8, 5, 8, 8, 8)), n // 8, 1, 1, True, 1.0 / n)
    x, _, _ = W.patch_cell_centres(n // 8, 1, 1, 1.0 / n)
    rho0, p0 = 1.0, theta0
    cs2 = O.cs2(theta0)
    cs = math.sqrt(cs2)
    h0 = O.h_of_theta(theta0)
    s = np.sin(2 * np.pi * x)
    # linear eigenvector of a right-moving sound wave: dp = h cs^2 drho, dv = cs drho / rho
    g.prim[:, 0] = rho0 * (1 + amp * s)
    g.prim[:, 4] = p0 + h0 * cs2 * rho0 * amp * s
    g.prim[:, 1] = cs * amp * s
    # the grid average of sin over a cell is sin(centre) * sinc(dh): compare like with like
    t_end = t_frac / cs
    c0 = initial_cons(g, scheme)
    c1, t, k = run(g, c0, t_end=t_end, theta=theta_lim, scheme=scheme, integrator=integrator)
    w, _ = to_prim(c1, scheme)
    exact = rho0 * (1 + amp * np.sin(2 * np.pi * (x - cs * t)))
    return np.mean(np.abs(1 - w[:, 0] / exact))
