"""Pins of the oracle's EoS pieces (Sec. 2.2, Eqs. 10, 14, 16, 22, A2) against facts that do not
reuse its formulas: the Taub relation that characterises the TM enthalpy (Eq. 12 with
equality), the general ideal-gas sound speed c_s^2 = Theta h' / (h (h' - 1)), limits stated in
the text, inverse relations and numerical derivatives."""
import numpy as np
import pytest
import mpmath as mp

import oracle as O

mp.mp.dps = 50
U = 2.0 ** -53
THETAS = np.logspace(-14, 14, 113)


def test_tm_enthalpy_is_the_taub_root():
    # TM satisfies (h - Theta)(h - 4 Theta) = 1 with h > 4 Theta; the oracle's h must be the
    # double nearest to that root (within a few ulps), judged in 50-digit arithmetic.
    for th in THETAS:
        h = O.h_of_theta(th)
        T, H = mp.mpf(th), mp.mpf(h)
        g = (H - T) * (H - 4 * T) - 1
        dg = 2 * H - 5 * T
        assert abs(g / dg) / H <= 4 * U, th


def test_htilde_is_h_minus_one_without_cancellation():
    # Eq. 22 must equal h - 1 to a few ulps of ht itself, including Theta -> 0 where h - 1
    # would lose every digit.
    for th in THETAS:
        ht = O.htilde_of_theta(th)
        T = mp.mpf(th)
        # the exact root of (h - T)(h - 4T) = 1, minus 1, in high precision
        H = (5 * T + mp.sqrt(9 * T * T + 4)) / 2
        assert abs(mp.mpf(ht) / (H - 1) - 1) <= 4 * U, th


def test_theta_of_htilde_inverts_eq22():
    for th in THETAS:
        r = O.theta_of_htilde(O.htilde_of_theta(th))
        assert abs(r / th - 1) <= 8 * U, th


def test_cold_and_hot_enthalpy_limits():
    # ht -> 5/2 Theta (non-relativistic, Gamma = 5/3) and h -> 4 Theta (ultra-relativistic,
    # Gamma = 4/3); Sec. 2.2 and the Gamma bounds of Eq. 12.
    assert abs(O.htilde_of_theta(1e-12) / 2.5e-12 - 1) < 1e-11
    assert abs(O.h_of_theta(1e12) / 4e12 - 1) < 1e-12


def test_effective_gamma_between_4_3_and_5_3():
    # Gamma_eff from h = 1 + Gamma/(Gamma-1) Theta (Eq. 11) must lie in [4/3, 5/3] (Sec. 2.2).
    for th in np.logspace(-8, 8, 65):
        ht = O.htilde_of_theta(th)
        g = ht / (ht - th)
        assert 4.0 / 3.0 - 1e-12 <= g <= 5.0 / 3.0 + 1e-12


def _cs2_thermo(th):
    # General ideal gas p = rho Theta: isentropic dh = dp / rho gives
    # c_s^2 = (dp/drho)_s / h = Theta h' / (h (h' - 1)), with h' = dh/dTheta.
    T = mp.mpf(th)
    h = lambda t: (5 * t + mp.sqrt(9 * t * t + 4)) / 2  # Taub root
    hp = mp.diff(h, T)
    return T * hp / (h(T) * (hp - 1))


def test_sound_speed_matches_thermodynamic_definition():
    for th in np.logspace(-10, 10, 41):
        c = O.cs2(th)
        assert abs(mp.mpf(c) / _cs2_thermo(th) - 1) < 1e-14, th


def test_sound_speed_limits():
    assert abs(O.cs2(1e-12) / (5.0 / 3.0 * 1e-12) - 1) < 1e-10      # NR: 5/3 Theta
    assert abs(O.cs2(1e12) - 1.0 / 3.0) < 1e-12                        # UR: c / sqrt(3)
    cs = [O.cs2(t) for t in np.logspace(-10, 10, 200)]
    assert all(b >= a - 4 * U for a, b in zip(cs, cs[1:]))             # monotone in Theta


def test_dtheta_dhtilde_matches_numerical_derivative():
    for ht in np.logspace(-10, 10, 61):
        d = O.dtheta_dhtilde(ht)
        e = ht * 1e-6
        num = (O.theta_of_htilde(ht + e) - O.theta_of_htilde(ht - e)) / (2 * e)
        assert abs(d / num - 1) < 1e-7, ht
