"""Pins of the oracle's conversions (Sec. 2.3: Eqs. 8, 5, 15-18, 22, 23, 30; App. A; App. B).

None of these re-types the oracle's formulas:
  * the exact left-hand side L is checked bit for bit against rational arithmetic;
  * prim -> cons is checked against the definitions D = rho gamma, M = rho h gamma U and the
    identity Et = rho [gamma U^2/(gamma+1) + gamma^2 ht - Theta] (from E = rho h gamma^2 - p),
    in 50-digit arithmetic;
  * cons -> prim is checked as the inverse of that forward map (the plain definition of the
    inversion), by a closed form for static gas, by exact power-of-two scale invariance, and by
    the round-trip error model of Eq. 20 / App. B;
  * the initial guesses are checked as the root of Eq. A3 and the asymptote intersection.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import workloads as W

mp.mp.dps = 50
U = 2.0 ** -53
EPS = np.finfo(np.float64).eps


def _L_rational(u):
    D, Mx, My, Mz, Et = (Fraction(float(v)) for v in u)
    return (Et * Et + 2 * Et * D - Mx * Mx - My * My - Mz * Mz), D


def test_sum_exact_is_correctly_rounded():
    rng = np.random.default_rng(7)
    for trial in range(3000):
        n = rng.integers(1, 12)
        xs = rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, size=n)
        if trial % 3 == 0:           # heavy cancellation
            xs = np.concatenate([xs, -xs[:-1] * (1 + 1e-15 * rng.standard_normal(n - 1))])
        assert O.sum_exact(xs) == math.fsum(xs.tolist())
    # half-way case: 1 + 2^-53 + tiny must round up
    assert O.sum_exact([1.0, 2.0 ** -53, 2.0 ** -120]) == 1.0 + 2.0 ** -52
    assert O.sum_exact([1.0, 2.0 ** -53]) == 1.0


def test_L_exact_is_rational_rounding():
    prim = W.conversion_batch(4000, seed=11)
    cons = O.prim2cons(prim)
    for i in range(cons.shape[1]):
        N, D = _L_rational(cons[:, i])
        ref = (float(N) / float(D)) / float(D)
        assert O.L_exact(*cons[:, i]) == ref


def _forward_mp(w):
    """Definitional prim -> cons in 50 digits: D = rho gamma, M = rho h gamma U,
    Et = rho [gamma U^2/(gamma+1) + gamma^2 ht - Theta]; h from the Taub root."""
    rho, ux, uy, uz, p = (mp.mpf(float(v)) for v in w)
    U2 = ux * ux + uy * uy + uz * uz
    g = mp.sqrt(1 + U2)
    th = p / rho
    h = (5 * th + mp.sqrt(9 * th * th + 4)) / 2
    ht = h - 1
    D = rho * g
    M = [rho * h * g * c for c in (ux, uy, uz)]
    Et = rho * (g * U2 / (g + 1) + g * g * ht - th)
    return D, M, Et, ht


def test_prim2cons_matches_definitions():
    prim = W.conversion_batch(400, seed=12)
    cons = O.prim2cons(prim)
    for i in range(prim.shape[1]):
        D, M, Et, _ = _forward_mp(prim[:, i])
        u = cons[:, i]
        assert abs(mp.mpf(u[0]) / D - 1) < 4 * U
        Mn = mp.sqrt(sum(m * m for m in M))
        for k in range(3):
            assert abs(mp.mpf(u[1 + k]) - M[k]) <= 8 * U * Mn
        assert abs(mp.mpf(u[4]) / Et - 1) < 32 * U, i


def test_prim2cons_cold_gas_has_no_cancellation():
    # Theta = 1e-12 at rest: Et = p * 3/2 (1 + O(Theta)), far below the rest mass D.
    u = O.prim2cons_one([2.0, 0.0, 0.0, 0.0, 2e-12])
    assert abs(u[4] / (1.5 * 2e-12) - 1) < 1e-11


def test_cons2prim_inverts_the_definitional_forward_map():
    # The plain definition of the inversion: the physical state whose prim->cons equals the
    # input.  Map the oracle's answer forward in 50 digits and compare D, M and the exact L.
    prim = W.conversion_batch(600, seed=13)
    cons = O.prim2cons(prim)
    w, st, _ = O.cons2prim(cons)
    checked = 0
    for i in range(cons.shape[1]):
        N, Dq = _L_rational(cons[:, i])
        Lx = mp.mpf(N.numerator) / mp.mpf(N.denominator) / (mp.mpf(float(Dq)) ** 2)
        if st[i] != O.ST_OK:
            assert Lx <= EPS * 1.01
            continue
        D, M, Et, _ = _forward_mp(w[:, i])
        u = cons[:, i]
        assert abs(mp.mpf(u[0]) / D - 1) < 8 * U
        Mn = mp.sqrt(sum(m * m for m in M))
        for k in range(3):
            assert abs(mp.mpf(u[1 + k]) - M[k]) <= 16 * U * max(Mn, mp.mpf(1e-300))
        Lw = (Et * Et + 2 * Et * D - sum(m * m for m in M)) / (D * D)
        assert abs(Lw / Lx - 1) < 64 * U, (i, float(Lw), float(Lx))
        checked += 1
    assert checked > 500


def test_static_gas_closed_form():
    # U = 0: Eq. 15 becomes (ht + 1 - Theta)^2 - 1 = x^2 + 2x with x = Et/D, and with the TM
    # relation this gives Theta = x (x + 2) / (3 (1 + x)) exactly.
    rng = np.random.default_rng(14)
    for th0 in np.concatenate([np.logspace(-10, 8, 37), 10 ** rng.uniform(-10, 8, 50)]):
        rho = 10 ** rng.uniform(-6, 6)
        u = O.prim2cons_one([rho, 0.0, 0.0, 0.0, rho * th0])
        w, st, _, _ = O.cons2prim_one(u)
        assert st == O.ST_OK
        x = mp.mpf(u[4]) / mp.mpf(u[0])
        th = x * (x + 2) / (3 * (1 + x))
        assert abs(mp.mpf(w[4]) / mp.mpf(w[0]) / th - 1) < 8 * U, th0
        assert w[0] == u[0] and w[1] == 0.0


def test_scale_invariance_is_exact_for_powers_of_two():
    prim = W.conversion_batch(300, seed=15)
    cons = O.prim2cons(prim)
    w1, s1, _ = O.cons2prim(cons)
    w2, s2, _ = O.cons2prim(cons * 2.0 ** 37)
    ok = s1 == O.ST_OK
    assert np.array_equal(s1, s2)
    assert np.array_equal(w2[0, ok], w1[0, ok] * 2.0 ** 37)
    assert np.array_equal(w2[4, ok], w1[4, ok] * 2.0 ** 37)
    assert np.array_equal(w2[1:4, ok], w1[1:4, ok])


def _kappa_eq20(w):
    """Eq. 20's bracket (the 'new scheme' error amplification), evaluated exactly."""
    rho, ux, uy, uz, p = (mp.mpf(float(v)) for v in w)
    U2 = ux * ux + uy * uy + uz * uz
    g2 = 1 + U2
    T = p / rho
    hp1 = (5 * T + mp.sqrt(9 * T * T + 4)) / 2
    beta2 = U2 / g2
    num = g2 * hp1 ** 2 * (1 + beta2) + T * T / g2 - 2 * hp1 * T - 1
    den = hp1 ** 2 + T * T / g2 - 2 * hp1 * T - 1
    return num / den


def test_round_trip_within_eq20_bound():
    prim = W.conversion_batch(3000, seed=16)
    cons = O.prim2cons(prim)
    w, st, _ = O.cons2prim(cons)
    worst = 0.0
    for i in range(prim.shape[1]):
        if st[i] != O.ST_OK:
            # only states whose rounded cons are genuinely (near-)unphysical may fail
            assert _kappa_eq20(prim[:, i]) * U > 1e-3
            continue
        h0 = O.htilde_of_theta(prim[4, i] / prim[0, i])
        h2 = O.htilde_of_theta(w[4, i] / w[0, i])
        err = abs(1 - h0 / h2)
        k = float(_kappa_eq20(prim[:, i]))
        if k * U > 1e-2:
            continue        # outside the first-order regime of Eq. 19-20
        worst = max(worst, err / (k * U))
        assert err <= 8 * k * U + 16 * U, (i, err, k)
    assert worst > 0.05   # the bound is not vacuous: some states come close to it


def test_appendix_b_error_curve():
    # App. B: Theta = 1e-8, Mach 1e-4..1e6, U along x = y = z.  The new scheme's round-trip error
    # follows (1 + M^2) eps; the original (total-energy) scheme's follows Eq. 21, ~ 4 eps/(3 Theta)
    # at low Mach (Eq. 32).
    th = 1e-8
    Us = math.sqrt(O.cs2(th) / (1 - O.cs2(th)))
    new_err, naive_ok = [], []
    for mach in np.logspace(-4, 6, 21):
        Um = mach * Us
        w0 = np.array([1.0, Um / math.sqrt(3), Um / math.sqrt(3), Um / math.sqrt(3), th])
        u1 = O.prim2cons_one(w0)
        w2, st, _, _ = O.cons2prim_one(u1)
        assert st == O.ST_OK
        h0 = O.htilde_of_theta(th)
        e = abs(1 - h0 / O.htilde_of_theta(w2[4] / w2[0]))
        assert e <= 8 * (1 + mach ** 2) * U + 16 * U, (mach, e)
        new_err.append(e)
        # the original scheme's left-hand side computed from E = Et + D loses ~1/Theta digits
        Lo = O.L_total_energy(u1[0], u1[1], u1[2], u1[3], u1[4] + u1[0])
        Lx = O.L_exact(*u1)
        naive_ok.append(abs(Lo / Lx - 1))
    # at low Mach the new scheme is at round-off while the original is ~1e-8 off (Eq. 32)
    assert max(new_err[:6]) < 1e-14
    assert min(naive_ok[:6]) > 1e-10


def _eq20_kappa(w):
    """Eq. 20's amplification factor (the bracket multiplying eps) from the primitive state, in
    50-digit arithmetic: [gamma^2 h^2 (1 + beta^2) + T^2/gamma^2 - 2 h T - 1] /
    [h^2 + T^2/gamma^2 - 2 h T - 1], h = ht + 1, T = Theta (the denominator written as
    ht (ht + 2) + ... so that a cold gas keeps its digits)."""
    rho, ux, uy, uz, p = (mp.mpf(float(v)) for v in w)
    th = p / rho
    U2 = ux * ux + uy * uy + uz * uz
    g2 = 1 + U2
    beta2 = U2 / g2
    a = mp.mpf(9) / 4 * th * th
    ht = mp.mpf(5) / 2 * th + a / (1 + mp.sqrt(a + 1))
    h = ht + 1
    num = g2 * h * h * (1 + beta2) + th * th / g2 - 2 * h * th - 1
    den = ht * (ht + 2) + th * th / g2 - 2 * h * th
    return num / den


def test_naive_L_rounding_and_eq20_error():
    # The paper-literal left-hand side x^2 + 2x - m^2 from the divided variables x = Et/D,
    # m = |M|/D.  (1) Against the same expression evaluated exactly on the correctly rounded
    # quotients (Python's float division is IEEE's): at most a few roundings of the terms, so
    # |error| <= 4u (x^2 + 2|x| + m^2).  (2) Against the exact L of the stored conserved
    # variables its relative error follows Eq. 20, (1 + Mach^2) eps (App. B, Theta = 1e-8, U along
    # x = y = z), and the bound is attained: a dropped term, a sign or a wrong quotient fails one
    # of the two.
    th = 1e-8
    Us = math.sqrt(O.cs2(th) / (1 - O.cs2(th)))
    rng = np.random.default_rng(23)
    states = [np.array([1.0, m * Us / math.sqrt(3), m * Us / math.sqrt(3), m * Us / math.sqrt(3), th])
              for m in np.logspace(-4, 6, 41)]
    prim = W.conversion_batch(200, seed=31)
    states += [prim[:, i] for i in range(prim.shape[1])]
    worst, big = 0.0, 0
    for w in states:
        u = O.prim2cons_one(w)
        Ln = O.L_naive(*u)
        D = u[0]
        x = Fraction(u[4] / D)
        ms = [Fraction(u[k] / D) for k in (1, 2, 3)]
        m2 = sum(v * v for v in ms)
        Lq = x * x + 2 * x - m2
        scale = x * x + 2 * abs(x) + m2
        assert abs(Fraction(Ln) - Lq) <= 4 * Fraction(U) * scale, w
        num, Dr = _L_rational(u)
        L = num / (Dr * Dr)
        if L <= 0:
            continue
        err = abs(float((Fraction(Ln) - L) / L))
        kappa = float(_eq20_kappa(w))
        assert err <= 8 * kappa * U + 8 * U, (w, err, kappa)
        worst = max(worst, err / (kappa * U))
        big += err > 1e-10
    assert worst > 0.1          # the bound is attained, not vacuous
    assert big >= 5             # and the amplification is visible at high Mach
    # the batch entry point evaluates the same function
    cons = np.stack([O.prim2cons_one(w) for w in states[:50]], axis=1)
    Lb = O.L_batch(cons, mode="naive")
    assert all(Lb[i] == O.L_naive(*cons[:, i]) for i in range(cons.shape[1]))


def test_unphysical_states_are_flagged():
    good = O.prim2cons_one([1.0, 0.5, 0.0, 0.0, 1.0])
    assert O.cons2prim_one(good)[1] == O.ST_OK
    for bad in ([-1.0, 0, 0, 0, 1.0], [0.0, 0, 0, 0, 1.0], [1.0, 0, 0, 0, 0.0],
                [1.0, 0, 0, 0, -1e-3], [np.nan, 0, 0, 0, 1.0], [1.0, np.inf, 0, 0, 1.0]):
        w, st, _, _ = O.cons2prim_one(bad)
        assert st == O.ST_UNPHYSICAL and np.all(np.isnan(w))
    # L = x^2 + 2x - m^2 <= eps (Eq. 30): momentum exceeding the energy budget
    x = 0.5
    m = math.sqrt(x * (x + 2))
    w, st, _, _ = O.cons2prim_one([1.0, m * 1.0000001, 0.0, 0.0, x])
    assert st == O.ST_UNPHYSICAL
    w, st, _, _ = O.cons2prim_one([1.0, m * 0.99, 0.0, 0.0, x])
    assert st == O.ST_OK


def test_inversion_function_is_increasing_and_derivative_is_right():
    for m2 in (0.0, 1e-6, 1.0, 1e4, 1e12):
        hs = np.logspace(-10, 8, 200)
        fs = [O.f(h, m2) for h in hs]
        assert all(b > a for a, b in zip(fs, fs[1:]))
        for h in hs[::10]:
            e = h * 1e-6
            num = (O.f(h + e, m2) - O.f(h - e, m2)) / (2 * e)
            d = O.dfdh(h, m2)
            assert d >= 1.2 * (1 - 1e-12)       # slope 6/5 at the origin, convex
            assert abs(d / num - 1) < 1e-6, (h, m2)


def test_bracketed_root_solves_the_equation():
    rng = np.random.default_rng(17)
    for _ in range(500):
        L = 10 ** rng.uniform(-15, 12)
        m2 = 10 ** rng.uniform(-10, 12)
        ht, it = O.solve_htilde(L, m2)
        assert abs(O.f(ht, m2) / L - 1) < 16 * U
        assert it < 200


def test_cold_guess_is_root_of_eq_a3():
    rng = np.random.default_rng(18)
    for _ in range(200):
        L = 10 ** rng.uniform(-12, 4)
        m2 = 10 ** rng.uniform(-8, 10)
        g = mp.mpf(O.guess_cold(L, m2))
        a = mp.mpf(43) / 125 + mp.mpf(4) / (25 * (1 + mp.mpf(m2)))
        r = mp.mpf(6) / 5 * g + a * g * g - mp.mpf(L)
        assert abs(r / mp.mpf(L)) < 16 * U


def test_cold_guess_is_second_order_accurate():
    # Eq. A3 keeps the O(ht^2) term: the guess error is O(ht^2) relative, i.e. O(L^2)
    for m2 in (0.0, 1.0, 1e6):
        errs = []
        for L in (1e-2, 1e-3, 1e-4):
            root, _ = O.solve_htilde(L, m2)
            errs.append(abs(O.guess_cold(L, m2) / root - 1))
        assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50


def test_hot_guess_and_threshold():
    for m2 in (0.0, 1.0, 1e6):
        root, _ = O.solve_htilde(1e12, m2)
        assert abs(O.guess_hot(1e12) / root - 1) < 1e-5
        # Eq. A7 is the L where the cold quadratic and the hot asymptote (9/16) ht^2 cross
        a = mp.mpf(43) / 125 + mp.mpf(4) / (25 * (1 + mp.mpf(m2)))
        hx = (mp.mpf(6) / 5) / (mp.mpf(9) / 16 - a)
        Lx = mp.mpf(9) / 16 * hx * hx
        assert abs(mp.mpf(O.guess_threshold(m2)) / Lx - 1) < 8 * U
        # at the threshold both guesses agree
        t = O.guess_threshold(m2)
        assert abs(O.guess_cold(t, m2) / O.guess_hot(t) - 1) < 1e-12
