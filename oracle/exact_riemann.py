"""Exact solution of the 1D relativistic Riemann problem with the Taub-Mathews EoS (App. C).

TEST INFRASTRUCTURE ONLY (part of the oracle).  Written from App. C's equations in 40-digit
arithmetic (mpmath), in four-velocity throughout:

* the pressure p* between the two waves solves U_C_L(p*) = U_C_R(p*) (Eq. C1 with the relative
  four-velocity of the two contact-side states equal to zero);
* behind a rarefaction: the isentrope (p / rho^(5/3))(h - Theta) = const (Eq. C2b) -- equivalently
  Theta (h - Theta) = K rho^(2/3), whose inverse is Theta = C / sqrt(1 + 3C) with C = K rho^(2/3) --
  and the Riemann invariant dU/drho = +-c_s gamma / rho (Eq. C2a), i.e. the rapidity changes by
  +-int c_s drho / rho; the upper sign belongs to the right wave, the lower to the left one;
* behind a shock: the Taub adiabat h_u^2 - h_d^2 = (h_d/rho_d + h_u/rho_u)(p_u - p_d) (Eq. C3)
  solved for h_d with rho_d = p_d / Theta(h_d) (Eqs. 16, 18); the mass flux J (Eq. C4); the shock
  and downstream four-velocities by Lorentz boosts (Eqs. C5-C6: the shock moves at +-J/rho_u
  relative to the upstream gas, the downstream gas at -+J/rho_d relative to the shock);
* inside a rarefaction fan the fluid rapidity is that of xi = x/t plus (right wave: minus) that of
  the sound speed, the four-velocity form of U(xi) = Relative(xi/sqrt(1-xi^2), +-c_s/sqrt(1-c_s^2)).

States are (rho, U, p) with U the x four-velocity.  The wave pattern is chosen by the sign of
each side: p* < p_K gives a rarefaction on side K, p* >= p_K a shock.

The same construction holds for the polytropic EoS of Sec. 2.2 (GammaLaw): only h(Theta), its
inverse, the sound speed and the isentrope (Theta = K rho^(Gamma - 1)) change.
"""
import mpmath as mp

mp.mp.dps = 40


def _f(x):
    return mp.mpf(x)


def h_of(th):
    """Eq. 10."""
    return _f(5) / 2 * th + mp.sqrt(_f(9) / 4 * th * th + 1)


def theta_of_h(h):
    """Eq. 16 with ht = h - 1."""
    ht = h - 1
    return (2 * ht * ht + 4 * ht) / (5 * ht + 5 + mp.sqrt(9 * ht * ht + 18 * ht + 25))


def cs2_of(th):
    """Eq. 14."""
    h = h_of(th)
    return th / (3 * h) * (5 * h - 8 * th) / (h - th)


def rapidity(U):
    return mp.asinh(U)


def relative(U1, U2):
    """Four-velocity of U1 seen from a frame moving with U2 (sinh of the rapidity difference)."""
    return U1 * mp.sqrt(1 + U2 * U2) - U2 * mp.sqrt(1 + U1 * U1)


class TaubMathews:
    """The TM EoS (Eqs. 10, 14, 16) and its isentrope (Eq. C2b)."""
    h_of = staticmethod(h_of)
    theta_of_h = staticmethod(theta_of_h)
    cs2_of = staticmethod(cs2_of)

    @staticmethod
    def isentrope_constant(rho, th, h):
        return th * (h - th) / rho ** (_f(2) / 3)                        # Eq. C2b

    @staticmethod
    def theta_isentrope(K, rho):
        C = K * rho ** (_f(2) / 3)
        return C / mp.sqrt(1 + 3 * C)

    def rho_isentrope(self, K, p, rho0, p0):
        lr = mp.findroot(lambda lr: mp.exp(lr) * self.theta_isentrope(K, mp.exp(lr)) - p,
                         mp.log(rho0 * (p / p0) ** (_f(3) / 5)))
        return mp.exp(lr)


class GammaLaw:
    """The polytropic EoS h = 1 + Gamma Theta / (Gamma - 1) (Sec. 2.2): c_s^2 = Gamma Theta / h and
    the isentrope p = K rho^Gamma."""

    def __init__(self, gamma):
        self.g = _f(gamma)

    def h_of(self, th):
        return 1 + self.g * th / (self.g - 1)

    def theta_of_h(self, h):
        return (h - 1) * (self.g - 1) / self.g

    def cs2_of(self, th):
        return self.g * th / self.h_of(th)

    def isentrope_constant(self, rho, th, h):
        return th / rho ** (self.g - 1)

    def theta_isentrope(self, K, rho):
        return K * rho ** (self.g - 1)

    def rho_isentrope(self, K, p, rho0, p0):
        return (p / K) ** (1 / self.g)


class Side:
    def __init__(self, rho, U, p, eos=None):
        self.eos = eos if eos is not None else TaubMathews()
        self.rho, self.U, self.p = _f(rho), _f(U), _f(p)
        self.th = self.p / self.rho
        self.h = self.eos.h_of(self.th)
        self.K = self.eos.isentrope_constant(self.rho, self.th, self.h)

    def theta_isentrope(self, rho):
        return self.eos.theta_isentrope(self.K, rho)

    def rho_isentrope(self, p):
        """Density on this state's isentrope at pressure p (p = rho Theta, Theta(rho) above)."""
        return self.eos.rho_isentrope(self.K, p, self.rho, self.p)

    def riemann_integral(self, rho):
        """int_{rho_K}^{rho} c_s / rho' drho' along the isentrope (Eq. C2a)."""
        f = lambda lr: mp.sqrt(self.eos.cs2_of(self.theta_isentrope(mp.exp(lr))))
        return mp.quad(f, [mp.log(self.rho), mp.log(rho)])

    def behind_rarefaction(self, p, sign):
        """(U, rho) behind a rarefaction of this side reaching pressure p; sign +1 right wave."""
        rho = self.rho_isentrope(p)
        phi = rapidity(self.U) + sign * self.riemann_integral(rho)
        return mp.sinh(phi), rho

    def behind_shock(self, p, sign):
        """(U_down, rho_down, U_shock) behind a shock of this side with downstream pressure p."""
        hu, ru, pu = self.h, self.rho, self.p

        def taub(hd):
            rd = p / self.eos.theta_of_h(hd)
            return hu * hu - hd * hd - (hd / rd + hu / ru) * (pu - p)
        # the downstream enthalpy lies above the upstream one for p > p_u; bracket it
        lo, hi = hu, hu * 2
        while taub(hi) > 0:
            hi *= 2
        hd = mp.findroot(taub, (lo, hi), solver="anderson")
        rd = p / self.eos.theta_of_h(hd)
        J = mp.sqrt((p - pu) / (hu / ru - hd / rd))                        # Eq. C4
        a = J / ru
        Us = sign * a * mp.sqrt(1 + self.U ** 2) + self.U * mp.sqrt(1 + a * a)   # Eq. C5
        b = J / rd
        Ud = -sign * b * mp.sqrt(1 + Us * Us) + Us * mp.sqrt(1 + b * b)          # Eq. C6
        return Ud, rd, Us

    def behind(self, p, sign):
        if p < self.p:
            U, rho = self.behind_rarefaction(p, sign)
            return U, rho, None
        if p == self.p:
            return self.U, self.rho, None
        U, rho, Us = self.behind_shock(p, sign)
        return U, rho, Us


class RiemannTM:
    """Exact solution for left/right states (rho, U, p) with the discontinuity at x0; eos: the TM
    EoS (default) or a GammaLaw."""

    def __init__(self, left, right, x0=0.0, eos=None):
        self.eos = eos if eos is not None else TaubMathews()
        self.L, self.R = Side(*left, eos=self.eos), Side(*right, eos=self.eos)
        self.x0 = _f(x0)
        g = lambda lp: self.L.behind(mp.exp(lp), -1)[0] - self.R.behind(mp.exp(lp), +1)[0]
        lo = mp.log(min(self.L.p, self.R.p)) - 40
        hi = mp.log(max(self.L.p, self.R.p)) + 40
        # bisection to a tight bracket, then a secant finish (both functions are monotone)
        for _ in range(120):
            mid = (lo + hi) / 2
            if g(mid) > 0:
                lo = mid
            else:
                hi = mid
        lp = mp.findroot(g, (lo, hi), solver="secant")
        self.p_star = mp.exp(lp)
        self.U_star, self.rho_L_star, self.Us_L = self.L.behind(self.p_star, -1)
        UR, self.rho_R_star, self.Us_R = self.R.behind(self.p_star, +1)
        self.U_star_R = UR

    # ---------------------------------------------------------------- sampling
    @staticmethod
    def _speed(U):
        return U / mp.sqrt(1 + U * U)

    def _fan_left_edges(self):
        csL = mp.sqrt(self.eos.cs2_of(self.L.th))
        vL = self._speed(self.L.U)
        head = (vL - csL) / (1 - vL * csL)
        ths = self.p_star / self.rho_L_star
        css = mp.sqrt(self.eos.cs2_of(ths))
        vs = self._speed(self.U_star)
        tail = (vs - css) / (1 - vs * css)
        return head, tail

    def _fan_right_edges(self):
        csR = mp.sqrt(self.eos.cs2_of(self.R.th))
        vR = self._speed(self.R.U)
        head = (vR + csR) / (1 + vR * csR)
        ths = self.p_star / self.rho_R_star
        css = mp.sqrt(self.eos.cs2_of(ths))
        vs = self._speed(self.U_star_R)
        tail = (vs + css) / (1 + vs * css)
        return head, tail

    def _in_fan(self, side, xi, sign):
        """(rho, U, p) inside a rarefaction fan at xi: rapidity(U) = atanh(xi) - sign atanh(c_s)
        and rapidity(U) = rapidity(U_K) + sign int c_s drho/rho."""
        def g(lr):
            rho = mp.exp(lr)
            cs = mp.sqrt(self.eos.cs2_of(side.theta_isentrope(rho)))
            return (rapidity(side.U) + sign * side.riemann_integral(rho)) - (mp.atanh(xi) - sign * mp.atanh(cs))
        lo = mp.log(min(side.rho, self.rho_L_star if sign < 0 else self.rho_R_star))
        hi = mp.log(side.rho)
        lr = mp.findroot(g, (lo, hi), solver="anderson")
        rho = mp.exp(lr)
        th = side.theta_isentrope(rho)
        cs = mp.sqrt(self.eos.cs2_of(th))
        U = mp.sinh(mp.atanh(xi) - sign * mp.atanh(cs))
        return rho, U, rho * th

    def sample(self, x, t):
        """(rho, U, p) at position x and time t > 0."""
        xi = (_f(x) - self.x0) / _f(t)
        vc = self._speed(self.U_star)
        # left wave
        if self.L.p > self.p_star:
            head, tail = self._fan_left_edges()
            if xi < head:
                return self.L.rho, self.L.U, self.L.p
            if xi < tail:
                return self._in_fan(self.L, xi, -1)
            if xi < vc:
                return self.rho_L_star, self.U_star, self.p_star
        else:
            vs = self._speed(self.Us_L) if self.Us_L is not None else vc
            if xi < vs:
                return self.L.rho, self.L.U, self.L.p
            if xi < vc:
                return self.rho_L_star, self.U_star, self.p_star
        # right wave
        if self.R.p > self.p_star:
            head, tail = self._fan_right_edges()
            if xi > head:
                return self.R.rho, self.R.U, self.R.p
            if xi > tail:
                return self._in_fan(self.R, xi, +1)
            return self.rho_R_star, self.U_star_R, self.p_star
        vs = self._speed(self.Us_R) if self.Us_R is not None else vc
        if xi > vs:
            return self.R.rho, self.R.U, self.R.p
        return self.rho_R_star, self.U_star_R, self.p_star

    def wave_positions(self, t):
        """Positions at time t of the left-wave edges, the contact and the right-wave edges."""
        t = _f(t)
        out = {}
        if self.L.p > self.p_star:
            head, tail = self._fan_left_edges()
            out["left_head"], out["left_tail"] = self.x0 + head * t, self.x0 + tail * t
        else:
            out["left_shock"] = self.x0 + self._speed(self.Us_L) * t
        out["contact"] = self.x0 + self._speed(self.U_star) * t
        if self.R.p > self.p_star:
            head, tail = self._fan_right_edges()
            out["right_head"], out["right_tail"] = self.x0 + head * t, self.x0 + tail * t
        else:
            out["right_shock"] = self.x0 + self._speed(self.Us_R) * t
        return out
