"""Pins of the oracle's reconstruction and Riemann fluxes (Sec. 3.2; fluxes of Eqs. 4a, 4b, 7).

Checked against properties, not re-typed formulas: the limiter on constant/linear/extremal data
and the TVD bound; the energy-flux identity (Et + p + D) v_d = M_d; the signal speeds against
the three-velocity form of relativistic velocity addition; HLLC/HLLE consistency, upwinding,
mirror symmetry, the HLL-average consistency of the HLLC star states and the exact resolution
of a stationary contact."""
import math

import mpmath as mp
import numpy as np

import oracle as O

mp.mp.dps = 40
U = 2.0 ** -53


def test_slope_limiter_properties():
    th = 1.5
    assert O.slope(2.0, 2.0, 2.0, th) == 0.0                     # constant
    assert O.slope(1.0, 2.0, 3.0, th) == 1.0                     # linear: exact difference
    assert O.slope(3.0, 2.0, 1.0, th) == -1.0
    assert O.slope(1.0, 3.0, 2.0, th) == 0.0                     # extremum
    assert O.slope(1.0, 1.0, 5.0, th) == 0.0                     # flat on one side
    # van Leer branch: 2 dl dr/(dl+dr) with dl = 1, dr = 3 -> 1.5; theta*min = 1.5
    assert abs(O.slope(0.0, 1.0, 4.0, 2.0) - 1.5) < 1e-15
    # generalized minmod branch: theta |dl| is smaller than van Leer's value
    assert abs(O.slope(0.0, 1.0, 101.0, 1.0) - 1.0) < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(5000):
        a, b, c = rng.standard_normal(3) * 10 ** rng.uniform(-10, 10)
        for t in (1.0, 1.5, 2.0):
            s = O.slope(a, b, c, t)
            lo, hi = min(a, b, c), max(a, b, c)
            for face in (b - 0.5 * s, b + 0.5 * s):
                assert lo - 1e-15 * abs(lo) <= face <= hi + 1e-15 * abs(hi)
            assert abs(s) <= 2 * min(abs(b - a), abs(c - b)) * (1 + 1e-15)


def _rand_prim(rng, n):
    out = []
    for _ in range(n):
        rho = 10 ** rng.uniform(-4, 4)
        th = 10 ** rng.uniform(-8, 4)
        Umag = 10 ** rng.uniform(-4, 3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        out.append(np.array([rho, *(Umag * d), rho * th]))
    return out


def test_energy_flux_identity():
    rng = np.random.default_rng(4)
    for w in _rand_prim(rng, 300):
        u = O.prim2cons_one(w)
        for d in range(3):
            F = O.flux(d, w)
            # (Et + p + D) v_d = (E + p) v_d = rho h gamma U_d = M_d
            assert abs(F[4] + F[0] - u[1 + d]) <= 1e-13 * (abs(u[1 + d]) + abs(F[0]))
            assert abs(F[0] - u[0] * w[1 + d] / math.sqrt(1 + w[1] ** 2 + w[2] ** 2 + w[3] ** 2)) \
                <= 4 * U * abs(F[0])


def test_signal_speeds_against_velocity_addition():
    rng = np.random.default_rng(5)
    for w in _rand_prim(rng, 300):
        th = mp.mpf(w[4]) / mp.mpf(w[0])
        cs2 = mp.mpf(O.cs2(float(th)))
        g = mp.sqrt(1 + sum(mp.mpf(x) ** 2 for x in w[1:4]))
        v = [mp.mpf(x) / g for x in w[1:4]]
        v2 = sum(x * x for x in v)
        for d in range(3):
            vd = v[d]
            rad = mp.sqrt(cs2 * (1 - v2) * (1 - v2 * cs2 - vd * vd * (1 - cs2)))
            lm = (vd * (1 - cs2) - rad) / (1 - v2 * cs2)
            lp = (vd * (1 - cs2) + rad) / (1 - v2 * cs2)
            a, b = O.wavespeeds(d, w)
            assert abs(a - lm) <= 1e-13 and abs(b - lp) <= 1e-13
            assert -1 < a < b < 1
    # at rest the speeds are +-c_s; with U_perp = 0 they are (v +- c_s)/(1 +- v c_s)
    a, b = O.wavespeeds(0, [1.0, 0.0, 0.0, 0.0, 1.0])
    cs = math.sqrt(O.cs2(1.0))
    assert abs(a + cs) < 1e-15 and abs(b - cs) < 1e-15
    Ux = 3.0
    v = Ux / math.sqrt(1 + Ux * Ux)
    a, b = O.wavespeeds(0, [1.0, Ux, 0.0, 0.0, 1.0])
    assert abs(a - (v - cs) / (1 - v * cs)) < 1e-14 and abs(b - (v + cs) / (1 + v * cs)) < 1e-14


def test_riemann_consistency_and_upwinding():
    rng = np.random.default_rng(6)
    for w in _rand_prim(rng, 200):
        for d in range(3):
            F = O.flux(d, w)
            for s in (O.HLLC, O.HLLE):
                G = O.riemann(d, w, w, s)
                assert np.allclose(G, F, rtol=1e-10, atol=1e-300), (d, s)
    # supersonic to the right: both signal speeds positive -> left flux
    wl = np.array([1.0, 50.0, 0.0, 0.0, 1e-4])
    wr = np.array([2.0, 40.0, 1.0, 0.0, 2e-4])
    for s in (O.HLLC, O.HLLE):
        assert np.array_equal(O.riemann(0, wl, wr, s), O.flux(0, wl))
        # and mirrored: supersonic to the left -> right flux
        ml, mr = wr * [1, -1, 1, 1, 1], wl * [1, -1, 1, 1, 1]
        assert np.array_equal(O.riemann(0, ml, mr, s), O.flux(0, mr))


def test_riemann_mirror_symmetry():
    rng = np.random.default_rng(8)
    ws = _rand_prim(rng, 200)
    for wl, wr in zip(ws[::2], ws[1::2]):
        for s in (O.HLLC, O.HLLE):
            F = O.riemann(0, wl, wr, s)
            flip = np.array([1, -1, 1, 1, 1.0])
            G = O.riemann(0, wr * flip, wl * flip, s)
            # mass, transverse momenta and energy fluxes change sign; normal momentum does not
            ref = F * np.array([-1, 1, -1, -1, -1.0])
            # HLLC works with the total energy E = Et + D and p* = F^m - l* F^E, so its rounding
            # is relative to the scale of the states and fluxes that enter the HLL average.
            ul, ur = O.prim2cons_one(wl), O.prim2cons_one(wr)
            fl, fr = O.flux(0, wl), O.flux(0, wr)
            scale = np.abs(ul) + np.abs(ur) + np.abs(fl) + np.abs(fr)
            scale[4] += ul[0] + ur[0] + abs(fl[0]) + abs(fr[0])
            assert np.all(np.abs(G - ref) <= 1e-13 * scale), s


def test_hllc_resolves_stationary_contact():
    # Different densities, equal pressure, zero velocity: HLLC has no mass flux across the
    # contact and the momentum flux is the pressure; HLLE smears it (non-zero mass flux).
    wl = np.array([10.0, 0.0, 0.0, 0.0, 1.0])
    wr = np.array([0.1, 0.0, 0.0, 0.0, 1.0])
    F = O.riemann(0, wl, wr, O.HLLC)
    assert abs(F[0]) < 1e-13 and abs(F[1] - 1.0) < 1e-14 and abs(F[4]) < 1e-13
    G = O.riemann(0, wl, wr, O.HLLE)
    assert abs(G[0]) > 1e-3


def test_hllc_star_state_satisfies_contact_jump_conditions():
    # Inside the star region the HLLC flux is the physical flux of a star state moving with the
    # contact: F_D = D* l*, F_Mx = Mx* l* + p*, F_My = My* l*, F_Mz = Mz* l*, and the total-energy
    # flux F_Et + F_D equals Mx* = (E* + p*) l*.  The star state is recovered from the flux as
    # U*_K = U_K + (F - F_K) / S_K on the side K that the contact speed selects.
    rng = np.random.default_rng(9)
    checked = 0
    for _ in range(400):
        ws = []
        for _ in range(2):
            rho = 10 ** rng.uniform(-2, 2)
            th = 10 ** rng.uniform(-4, 2)
            Ux, Uy, Uz = rng.uniform(-2, 2, size=3)
            ws.append(np.array([rho, Ux, Uy, Uz, rho * th]))
        wl, wr = ws
        d = 0
        F = O.riemann(d, wl, wr, O.HLLC)
        lmL, lpL = O.wavespeeds(d, wl)
        lmR, lpR = O.wavespeeds(d, wr)
        sl, sr = min(lmL, lmR), max(lpL, lpR)
        if not (sl < 0 < sr):
            continue
        for w, S in ((wl, sl), (wr, sr)):
            u, f = O.prim2cons_one(w), O.flux(d, w)
            us = u + (F - f) / S
            ls = F[0] / us[0]
            if (S < 0) != (ls >= 0):
                continue            # this side's star state is not the one selected
            ps = F[1] - us[1] * ls
            Es = us[4] + us[0]
            sc = np.abs(u).max() + np.abs(f).max()
            assert abs(F[2] - us[2] * ls) <= 1e-10 * sc
            assert abs(F[3] - us[3] * ls) <= 1e-10 * sc
            assert abs((F[4] + F[0]) - us[1]) <= 1e-10 * sc
            assert abs(us[1] - (Es + ps) * ls) <= 1e-10 * sc
            assert us[0] > 0
            checked += 1
    assert checked > 100


def test_cold_limit_matches_newtonian_hllc_mass_flux_sign():
    # Cold, slow gas: the relativistic fluxes approach the Newtonian ones: mass flux rho v,
    # momentum rho v^2 + p (Eqs. 4a-4b with gamma -> 1).
    w = np.array([2.0, 1e-4, 0.0, 0.0, 2e-8])
    F = O.flux(0, w)
    assert abs(F[0] / (2.0 * 1e-4) - 1) < 1e-7
    assert abs(F[1] / (2.0 * 1e-8 + 2e-8) - 1) < 1e-6
