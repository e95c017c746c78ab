"""Pins of the oracle with the polytropic EoS of Sec. 2.2, h = 1 + Gamma Theta / (Gamma - 1).

* the sound speed is the general ideal-gas result c_s^2 = Theta h' / (h (h' - 1)) (50 digits);
* cons -> prim inverts the definitional forward map E = rho h gamma^2 - p, M = rho h gamma U,
  D = rho gamma (50 digits), over cold to hot and slow to ultra-relativistic states;
* Gamma = 5/3 agrees with TM for a cold gas and Gamma = 4/3 for a hot one (the limits of Sec. 2.2),
  through a whole step;
* shock tubes converge to the exact solution of App. C's construction with the polytropic EoS
  (MUSCL-Hancock and VL), whose fans keep the isentrope p rho^-Gamma and whose shocks satisfy
  the Taub adiabat."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.exact_riemann import GammaLaw, RiemannTM
from tests import oracle_driver as drv

mp.mp.dps = 50


@pytest.mark.parametrize("gamma", [4 / 3, 1.5, 5 / 3, 2.0])
def test_sound_speed_matches_thermodynamic_definition(gamma):
    g = mp.mpf(gamma)
    h = lambda t: 1 + g * t / (g - 1)
    with O.eos(gamma):
        for th in np.logspace(-10, 10, 21):
            T = mp.mpf(th)
            hp = mp.diff(h, T)
            ref = T * hp / (h(T) * (hp - 1))
            assert abs(mp.mpf(O.cs2(th)) / ref - 1) < 1e-14, th


def test_eos_selection_is_checked():
    with pytest.raises(ValueError):
        with O.eos(2.5):
            pass
    with O.eos(1.4):
        assert abs(O.h_of_theta(1.0) - (1 + 1.4 / 0.4)) < 1e-15
    assert abs(O.h_of_theta(1.0) - (2.5 + math.sqrt(3.25))) < 1e-15      # TM again


def _forward_mp(w, gamma):
    rho, ux, uy, uz, p = (mp.mpf(float(v)) for v in w)
    g = mp.mpf(gamma)
    th = p / rho
    h = 1 + g * th / (g - 1)
    gam = mp.sqrt(1 + ux * ux + uy * uy + uz * uz)
    D = rho * gam
    M = [rho * h * gam * u for u in (ux, uy, uz)]
    E = rho * h * gam * gam - p
    return D, M, E - D


@pytest.mark.parametrize("gamma", [4 / 3, 5 / 3])
def test_cons2prim_inverts_the_definitional_forward_map(gamma):
    prim = W.conversion_batch(300, seed=21)
    with O.eos(gamma):
        cons = O.prim2cons(prim)
        w, st, _ = O.cons2prim(cons)
    U = 2.0 ** -53
    ok = 0
    for i in range(cons.shape[1]):
        if st[i] != O.ST_OK:
            continue
        D, M, Et = _forward_mp(w[:, i], gamma)
        u = cons[:, i]
        assert abs(mp.mpf(u[0]) / D - 1) < 16 * U, i
        Mn = mp.sqrt(sum(m * m for m in M))
        for k in range(3):
            assert abs(mp.mpf(u[1 + k]) - M[k]) <= 64 * U * max(Mn, mp.mpf(1e-300)), i
        L = lambda d, m, e: (e * e + 2 * e * d - sum(x * x for x in m)) / (d * d)
        Lx = L(mp.mpf(u[0]), [mp.mpf(v) for v in u[1:4]], mp.mpf(u[4]))
        assert abs(L(D, M, Et) / Lx - 1) < 1e-9, i
        ok += 1
    assert ok > 250


def _blast_step(gamma, theta_scale):
    g = W.blast(16, seed=3)
    g.prim[:, 4] = np.where(g.extra["labels"] == 1, 10.0, 1.0) * theta_scale * g.prim[:, 0]
    if gamma:
        with O.eos(gamma):
            c0 = drv.initial_cons(g)
            c1, _, _ = drv.run(g, c0, n_steps=2)
    else:
        c0 = drv.initial_cons(g)
        c1, _, _ = drv.run(g, c0, n_steps=2)
    return c1


def test_limits_of_the_tm_eos():
    # cold: TM -> Gamma = 5/3 with h differing at O(Theta^2); hot: TM -> Gamma = 4/3 with h
    # differing at O(1/Theta)
    for gamma, scale, tol in ((5 / 3, 1e-7, 1e-5), (4 / 3, 1e7, 1e-5)):
        a, b = _blast_step(gamma, scale), _blast_step(0, scale)
        for f in range(5):
            s = np.abs(b[:, f]).max()
            assert np.max(np.abs(a[:, f] - b[:, f])) < tol * s, (gamma, f)
    # and the two EoS do differ in between
    a, b = _blast_step(5 / 3, 1.0), _blast_step(0, 1.0)
    assert np.max(np.abs(a[:, 4] / b[:, 4] - 1)) > 1e-2


def test_exact_solver_isentrope_and_taub_adiabat():
    eos = GammaLaw(mp.mpf(5) / 3)
    ex = RiemannTM((10.0, 0.0, 40.0 / 3.0), (1.0, 0.0, 1e-6), x0=0.5, eos=eos)
    g = mp.mpf(5) / 3
    L = ex.L
    for x in np.linspace(0.2, 0.48, 8):
        r, U, p = ex.sample(x, 0.4)
        assert abs((p / r ** g) / (L.p / L.rho ** g) - 1) < 1e-25
    rd, pd = ex.rho_R_star, ex.p_star
    hd = eos.h_of(pd / rd)
    R = ex.R
    res = R.h ** 2 - hd ** 2 - (hd / rd + R.h / R.rho) * (R.p - pd)
    assert abs(res / hd ** 2) < 1e-30


def _tube_l1(n, left, right, t_end, gamma, integrator):
    l5 = (left[0], left[1], 0.0, 0.0, left[2])
    r5 = (right[0], right[1], 0.0, 0.0, right[2])
    g = W.riemann_1d(n, l5, r5, x0=0.5)
    with O.eos(gamma):
        c, t, _ = drv.run(g, drv.initial_cons(g), t_end=t_end, integrator=integrator)
        w, _ = drv.to_prim(c)
    x = g.extra["x"][:, 0, 0, :].reshape(-1)
    rho = w[:, 0, 0, 0, :].reshape(-1)
    ex = RiemannTM(left, right, x0=0.5, eos=GammaLaw(mp.mpf(gamma)))
    ref = np.array([float(ex.sample(xx, t)[0]) for xx in x])
    return np.mean(np.abs(1 - rho / ref))


@pytest.mark.slow
@pytest.mark.parametrize("gamma,left,right", [(5 / 3, (10.0, 0.0, 40.0 / 3.0), (1.0, 0.0, 1e-6)),
                                              (4 / 3, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))])
@pytest.mark.parametrize("integrator", [0, 1])
def test_shock_tubes_converge_to_the_exact_solution(gamma, left, right, integrator):
    e = [_tube_l1(n, left, right, 0.3, gamma, integrator) for n in (32, 64, 128)]
    print("Gamma %.3f integrator %d: L1 %s" % (gamma, integrator, e))
    assert e[1] < 0.75 * e[0] and e[2] < 0.75 * e[1], e
    assert e[2] < 0.05, e
