"""Equations of state, critical points and Maxwell equal-area coexistence.

TEST INFRASTRUCTURE ONLY (part of the oracle): used by the test suite and by
the script that writes the stored coexistence densities; never by the product
path.

The paper (Sec. 2.2, Sec. 3.1) names five equations of state -- Carnahan-
Starling (CS), Peng-Robinson (PR), Redlich-Kwong (RK), Redlich-Kwong-Soave
(RKS) and van der Waals (VdW) -- with parameters taken from Yuan & Schaefer
(2006), and compares simulated coexistence densities with Maxwell's
construction (Table 1).  The textbook forms written here are:

  CS : p = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2,  eta = b rho / 4
  VdW: p = rho R T / (1 - b rho) - a rho^2
  RK : p = rho R T / (1 - b rho) - a rho^2 / (sqrt(T) (1 + b rho))
  RKS: p = rho R T / (1 - b rho) - a al(T) rho^2 / (1 + b rho),
       al = [1 + (0.480 + 1.574 w - 0.176 w^2)(1 - sqrt(T/Tc))]^2
  PR : p = rho R T / (1 - b rho) - a al(T) rho^2 / (1 + 2 b rho - b^2 rho^2),
       al = [1 + (0.37464 + 1.54226 w - 0.26992 w^2)(1 - sqrt(T/Tc))]^2

Maxwell's construction: liquid and vapour densities rho_l > rho_v share the
saturation pressure p_s, and the area between the isotherm and p_s vanishes in
the specific volume v = 1/rho:  int_{rho_v}^{rho_l} (p(rho) - p_s) / rho^2 drho = 0.
Root finding and quadrature are SciPy's (brentq, quad).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from scipy import integrate, optimize


@dataclass(frozen=True)
class EOS:
    kind: str            # "CS", "VdW", "RK", "RKS", "PR"
    a: float
    b: float
    R: float = 1.0
    omega: float = 0.344  # acentric factor (RKS, PR)

    def rho_limit(self) -> float:
        """Upper end of the physical density range (pole of the repulsive term)."""
        return 4.0 / self.b if self.kind == "CS" else 1.0 / self.b

    def pressure(self, rho: float, T: float, Tc: float | None = None) -> float:
        a, b, R = self.a, self.b, self.R
        if self.kind == "CS":
            eta = b * rho / 4.0
            return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2
        if self.kind == "VdW":
            return rho * R * T / (1 - b * rho) - a * rho ** 2
        if self.kind == "RK":
            return rho * R * T / (1 - b * rho) - a * rho ** 2 / (math.sqrt(T) * (1 + b * rho))
        al = 1.0
        if Tc is not None:
            tr = T / Tc
            w = self.omega
            if self.kind == "RKS":
                al = (1 + (0.480 + 1.574 * w - 0.176 * w * w) * (1 - math.sqrt(tr))) ** 2
            else:
                al = (1 + (0.37464 + 1.54226 * w - 0.26992 * w * w) * (1 - math.sqrt(tr))) ** 2
        if self.kind == "RKS":
            return rho * R * T / (1 - b * rho) - a * al * rho ** 2 / (1 + b * rho)
        if self.kind == "PR":
            return rho * R * T / (1 - b * rho) - a * al * rho ** 2 / (1 + 2 * b * rho - b * b * rho ** 2)
        raise ValueError(self.kind)


# Parameter sets used by the paper's benchmarks: CS a=1, b=4, R=1; VdW
# a=9/49, b=2/21 (Sec. 3.3.1); RK/RKS/PR a=2/49, b=2/21 with the acentric factor
# of water (Yuan & Schaefer 2006).
CS = EOS("CS", 1.0, 4.0)
VDW = EOS("VdW", 9.0 / 49.0, 2.0 / 21.0)
RK = EOS("RK", 2.0 / 49.0, 2.0 / 21.0)
RKS = EOS("RKS", 2.0 / 49.0, 2.0 / 21.0)
PR = EOS("PR", 2.0 / 49.0, 2.0 / 21.0)
ALL = {"CS": CS, "PR": PR, "RK": RK, "RKS": RKS, "VdW": VDW}


def _dp(eos: EOS, rho: float, T: float, Tc=None, h=None) -> float:
    h = h or 1e-6 * eos.rho_limit()
    return (eos.pressure(rho + h, T, Tc) - eos.pressure(rho - h, T, Tc)) / (2 * h)


def _d2p(eos: EOS, rho: float, T: float, Tc=None) -> float:
    h = 1e-4 * eos.rho_limit()
    return (eos.pressure(rho + h, T, Tc) - 2 * eos.pressure(rho, T, Tc)
            + eos.pressure(rho - h, T, Tc)) / (h * h)


def critical_point(eos: EOS) -> tuple[float, float]:
    """(T_c, rho_c): the top of the spinodal curve, where dp/drho = d2p/drho2 = 0.
    T_spin(rho) is the temperature at which dp/drho vanishes at density rho;
    T_c is its maximum.  For RKS and PR the factor al(T) equals 1 at T = T_c, so
    the critical point is that of al = 1."""
    lim = eos.rho_limit()

    def t_spin(r):
        return optimize.brentq(lambda T: _dp(eos, r, T), 1e-10, 1e3, xtol=1e-16, rtol=1e-15)

    res = optimize.minimize_scalar(lambda r: -t_spin(r), bounds=(1e-3 * lim, 0.9 * lim),
                                   method="bounded", options={"xatol": 1e-13 * lim})
    return -res.fun, res.x


def maxwell(eos: EOS, Tr: float) -> tuple[float, float, float]:
    """Coexistence (rho_v, rho_l, p_sat) at reduced temperature Tr = T / T_c."""
    Tc, rc = critical_point(eos)
    T = Tr * Tc
    tc_arg = Tc if eos.kind in ("RKS", "PR") else None
    p = lambda r: eos.pressure(r, T, tc_arg)
    dp = lambda r: _dp(eos, r, T, tc_arg)
    lim = eos.rho_limit()
    # spinodal points: local maximum (vapour side) and minimum (liquid side)
    r_infl = optimize.brentq(lambda r: _d2p(eos, r, T, tc_arg), 1e-3 * lim, 0.9 * lim, xtol=1e-15)
    s1 = optimize.brentq(dp, 1e-9 * lim, r_infl, xtol=1e-16)
    top = 0.999999 * lim
    s2 = optimize.brentq(dp, r_infl, top, xtol=1e-16)
    p_hi, p_lo = p(s1), max(p(s2), 1e-14 * abs(p(s1)))

    def roots(ps):
        rv = optimize.brentq(lambda r: p(r) - ps, 1e-14 * lim, s1, xtol=1e-17, rtol=1e-15)
        rl = optimize.brentq(lambda r: p(r) - ps, s2, top, xtol=1e-17, rtol=1e-15)
        return rv, rl

    def area(ps):
        rv, rl = roots(ps)
        val, _ = integrate.quad(lambda r: (p(r) - ps) / (r * r), rv, rl,
                                epsabs=1e-15, epsrel=1e-13, limit=400, points=[s1, s2])
        return val

    eps = 1e-12 * (p_hi - p_lo)
    ps = optimize.brentq(area, p_lo + eps, p_hi - eps, xtol=1e-18, rtol=1e-14)
    rv, rl = roots(ps)
    return rv, rl, ps


def cs_psi_arg_max_density(Tr: float, alpha: float = 1.0) -> float:
    """Largest density below which the CS square-root argument alpha p - rho/3
    stays non-positive (with g_kk = -1 psi is real there)."""
    Tc, _ = critical_point(CS)
    T = Tr * Tc
    f = lambda r: alpha * CS.pressure(r, T) - r / 3.0
    # f < 0 for small rho (p ~ rho R T < rho/3); find the first sign change
    grid = [CS.rho_limit() * k / 4000.0 for k in range(1, 3999)]
    prev = grid[0]
    for r in grid[1:]:
        if f(r) > 0:
            return optimize.brentq(f, prev, r, xtol=1e-15)
        prev = r
    return CS.rho_limit()
