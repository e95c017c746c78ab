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


def amr_setup(nc, lo, hi, prim_fn):
    """Two-level hierarchy of workloads.two_level with primitive state prim_fn(x, y, z) -> [5] arrays;
    returns (geometry, coarse cons, fine cons), the refined coarse patches holding the average of
    their children."""
    t = W.two_level(nc, lo, hi)
    def cons_of(xyz):
        x, y, z = xyz
        w = np.stack(prim_fn(x, y, z), axis=1)                  # [P][5][8][8][8]
        P = w.shape[0]
        c = O.prim2cons(w.reshape(P, 5, 512).transpose(1, 0, 2).reshape(5, -1))
        return np.ascontiguousarray(c.reshape(5, P, 512).transpose(1, 0, 2)).reshape(P, 5, 8, 8, 8)
    cc = cons_of(t["coarse_xyz"])
    cf = cons_of(t["fine_xyz"])
    O.restrict(cc, t["parent_of"], t["child"], cf)
    return t, cc, cf


def amr_step(t, cc, cf, c_cfl=0.5, theta=1.5, correct=True, integrator=0):
    """One coarse step and two fine sub-steps of the two-level hierarchy with the oracle:
    same-level ghost fill, coarse-to-fine ghost interpolation (time-interpolated for the second
    sub-step), restriction and coarse-fine flux correction.  Returns (cc, cf, dt_c, info)."""
    dh = [t["dh_c"], t["dh_f"]]
    both = np.concatenate([cc, cf])
    lev = np.concatenate([np.zeros(cc.shape[0]), np.ones(cf.shape[0])])
    dt_lev, _, _ = O.cfl_dt(both, lev, dh, c_cfl)
    pad_c = O.fill_ghosts(cc, t["coarse_neighbor"], 3)
    cn, cnt_c, fc = O.fluid_step(pad_c, [dt_lev[0]], [dh[0]], theta=theta, bflux=True,
                                 integrator=integrator)
    pad_cn = O.fill_ghosts(cn, t["coarse_neighbor"], 3)
    ff = np.zeros((cf.shape[0], 6, 5, 64))
    f = cf
    info = {"coarse_counts": cnt_c, "fine_counts": [], "interp": []}
    for sub in range(2):
        pad_f = O.fill_ghosts(f, t["fine_neighbor"], 3)
        info["interp"].append(O.fill_ghosts_coarse(pad_f, t["fine_neighbor"], t["parent"], t["octant"],
                                                   pad_c, pad_cn if sub else None, 0.5 * sub, theta))
        f, cnt_f, flux = O.fluid_step(pad_f, [dt_lev[1]], [dh[1]], theta=theta, bflux=True,
                                      integrator=integrator)
        ff += dt_lev[1] * flux
        info["fine_counts"].append(cnt_f)
    O.restrict(cn, t["parent_of"], t["child"], f)
    info["skipped"] = O.flux_correct(cn, t["faces"], dt_lev[0] * fc, ff, dh[0]) if correct else 0
    return cn, f, dt_lev[0], info


def amr_totals(t, cc, cf):
    """Sum of each conserved variable times the cell volume over the unrefined coarse cells and
    the fine cells."""
    keep = ~t["refined"]
    return (cc[keep].sum(axis=(0, 2, 3, 4)) * t["dh_c"] ** 3 +
            cf.sum(axis=(0, 2, 3, 4)) * t["dh_f"] ** 3)
