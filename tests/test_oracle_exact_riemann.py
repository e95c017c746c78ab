"""Pins of the exact TM Riemann solver (App. C) against the paper's printed exact solution of
the mixed-limits problem, and of the oracle's step against that solver (L1 error of a 1D shock
tube decreasing with resolution)."""
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.exact_riemann import RiemannTM, Side, h_of
from tests import oracle_driver as drv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tm_riemann_mixed_limits.txt")


@pytest.fixture(scope="module")
def mixed():
    return RiemannTM((1e2, 1e-3, 1e-4), (1e-12, -1e2, 1e-10), x0=0.05)


def test_table_of_the_exact_solution(mixed):
    rows = np.loadtxt(GOLDEN)
    pos = mixed.wave_positions(80)
    for x, r, U, p in rows:
        rr, UU, pp = (float(v) for v in mixed.sample(x, 80))
        assert abs(rr / r - 1) < 1e-13, (x, rr, r)
        assert abs(pp / p - 1) < 1e-13, (x, pp, p)
        # between contact and shock the printed U differs from its own rarefaction side by
        # 4.6e-10 (the shock side of the contact); elsewhere it is exact to round-off
        tol = 1e-9 if pos["contact"] < x < pos["right_shock"] else 1e-13
        assert abs(UU / U - 1) < tol, (x, UU, U)


def test_wave_positions_against_table(mixed):
    x = np.loadtxt(GOLDEN)[:, 0]
    pos = {k: float(v) for k, v in mixed.wave_positions(80).items()}
    assert abs(pos["left_head"] - x[2]) < 1e-12          # first row inside the fan
    assert abs(pos["left_tail"] - x[14]) < 1e-12         # last row of the fan
    assert x[15] < pos["contact"] < x[16]
    assert x[17] < pos["right_shock"] < x[18]
    # the shock runs far ahead of the rarefaction head: speed ratio ~ 1.15e3
    shock_speed = (pos["right_shock"] - 0.05) / 80
    head_speed = (0.05 - pos["left_head"]) / 80
    assert 1100 < shock_speed / head_speed < 1200


def test_isentrope_and_taub_adiabat_hold(mixed):
    # the fan and the left star state share one isentrope constant (Eq. C2b); the shocked state
    # satisfies the Taub adiabat (Eq. C3) with the right state upstream
    L = Side(1e2, 1e-3, 1e-4)
    for x in np.linspace(0.03, 0.2, 9):
        r, U, p = mixed.sample(x, 80)
        th = p / r
        assert abs((p / r ** (mp.mpf(5) / 3)) * (h_of(th) - th) / (L.K * L.rho ** 0) - 1) < 1e-25
    R = Side(1e-12, -1e2, 1e-10)
    rd, pd = mixed.rho_R_star, mixed.p_star
    hd = h_of(pd / rd)
    res = R.h ** 2 - hd ** 2 - (hd / rd + R.h / R.rho) * (R.p - pd)
    assert abs(res / hd ** 2) < 1e-30


def _tube_l1(n, left, right, t_end, x0=0.5, theta=1.5):
    """L1 density error (Eq. 31) of the oracle's run of a 1D tube (states (rho, U, p))."""
    l5 = (left[0], left[1], 0.0, 0.0, left[2])
    r5 = (right[0], right[1], 0.0, 0.0, right[2])
    g = W.riemann_1d(n, l5, r5, x0=x0)
    c, t, _ = drv.run(g, drv.initial_cons(g), t_end=t_end, theta=theta)
    w, _ = drv.to_prim(c)
    # every row of cells across y and z carries the same profile: take the first one
    x = g.extra["x"][:, 0, 0, :].reshape(-1)
    rho = w[:, 0, 0, 0, :].reshape(-1)
    ex = RiemannTM(left, right, x0=x0)
    ref = np.array([float(ex.sample(xx, t)[0]) for xx in x])
    return np.mean(np.abs(1 - rho / ref))


@pytest.mark.slow
@pytest.mark.parametrize("left,right", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),       # Theta ~ 1
                                        ((1.0, 0.0, 1e-2), (0.1, 0.0, 1e-5))])     # cold
def test_step_converges_to_exact_solution(left, right):
    # shock tubes with the TM EoS: with a shock and a contact in the solution the L1 error falls
    # at first order (about halving per doubling of the resolution)
    e = [_tube_l1(n, left, right, 0.3) for n in (32, 64, 128)]
    assert e[1] < 0.7 * e[0] and e[2] < 0.7 * e[1], e
    assert e[2] < 0.02, e
