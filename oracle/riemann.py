"""Exact solution of the one-dimensional Riemann problem between two
stiffened gases (test infrastructure: only tests may use it).

Each side k is a stiffened gas p = (gamma_k - 1) rho e - gamma_k pinf_k
(the NASG EOS of Sec. 2.3 with b = q = 0); the gas-liquid Riemann problem of
Sec. 4.2.1 is one such pair (air and water).  The solution follows the
classical construction for the Euler equations (two nonlinear waves around a
contact; across each wave the Rankine-Hugoniot or isentropic relations of that
side's material), written in p + pinf_k, in which a stiffened gas behaves as
an ideal gas.  The star pressure is the root of
    f_L(p*) + f_R(p*) + u_R - u_L = 0
found by bisection to round-off; the solution is sampled at x / t.
"""
import math

import numpy as np


class Side:
    def __init__(self, rho, u, p, gamma, pinf=0.0):
        self.rho, self.u, self.p, self.g, self.pinf = float(rho), float(u), float(p), float(gamma), float(pinf)
        if not (self.rho > 0 and self.p + self.pinf > 0 and self.g > 1):
            raise ValueError("inadmissible side state")
        self.a = math.sqrt(self.g * (self.p + self.pinf) / self.rho)

    def f(self, ps):
        """Velocity jump across the wave that brings this side to pressure ps."""
        g, pb, psb = self.g, self.p + self.pinf, ps + self.pinf
        if psb > pb:  # shock: Rankine-Hugoniot
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * pb
            return (psb - pb) * math.sqrt(A / (psb + B))
        # rarefaction: isentrope p + pinf ~ rho^gamma, Riemann invariant
        return 2.0 * self.a / (g - 1.0) * ((psb / pb) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def rho_star(self, ps):
        g, pb, psb = self.g, self.p + self.pinf, ps + self.pinf
        if psb > pb:
            r = (g - 1.0) / (g + 1.0)
            return self.rho * (psb / pb + r) / (r * psb / pb + 1.0)
        return self.rho * (psb / pb) ** (1.0 / g)


def star_state(L, R):
    """(p*, u*) of the Riemann problem L | R."""
    def F(ps):
        return L.f(ps) + R.f(ps) + R.u - L.u
    # p* + pinf_k > 0 on both sides
    lo = max(-L.pinf, -R.pinf) + 1e-14 * max(L.p + L.pinf, R.p + R.pinf)
    if F(lo) > 0:
        raise ValueError("vacuum forms: no star state")
    hi = max(L.p, R.p, 1.0)
    while F(hi) < 0:
        hi *= 2.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if F(mid) < 0:
            lo = mid
        else:
            hi = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (L.u + R.u) + 0.5 * (R.f(ps) - L.f(ps))
    return ps, us


def sample(L, R, x, t, x0=0.0):
    """Exact (rho, u, p) at the points x (array) at time t > 0, initial jump at x0.
    Also returns the side (0 left material, 1 right material) of each point."""
    ps, us = star_state(L, R)
    xs = (np.asarray(x, dtype=np.float64) - x0) / t
    rho = np.empty_like(xs)
    u = np.empty_like(xs)
    p = np.empty_like(xs)
    side = np.empty(xs.shape, dtype=np.int64)
    for i, s in enumerate(xs.ravel()):
        left = s < us
        K, sgn = (L, -1.0) if left else (R, 1.0)
        side.flat[i] = 0 if left else 1
        g, pb, psb = K.g, K.p + K.pinf, ps + K.pinf
        if psb > pb:  # shock on this side
            S = K.u + sgn * K.a * math.sqrt((g + 1.0) / (2.0 * g) * psb / pb + (g - 1.0) / (2.0 * g))
            ahead = s < S if left else s > S
            val = (K.rho, K.u, K.p) if ahead else (K.rho_star(ps), us, ps)
        else:  # rarefaction: head, tail, fan
            a_star = K.a * (psb / pb) ** ((g - 1.0) / (2.0 * g))
            head = K.u + sgn * K.a
            tail = us + sgn * a_star
            if (left and s <= head) or (not left and s >= head):
                val = (K.rho, K.u, K.p)
            elif (left and s >= tail) or (not left and s <= tail):
                val = (K.rho_star(ps), us, ps)
            else:
                # inside the fan: u - sgn a = s (characteristic), invariant
                # u - sgn 2a/(g-1) constant from the undisturbed side
                c = 2.0 / (g + 1.0) - sgn * (g - 1.0) / ((g + 1.0) * K.a) * (K.u - s)
                uf = 2.0 / (g + 1.0) * (-sgn * K.a + (g - 1.0) / 2.0 * K.u + s)
                rf = K.rho * c ** (2.0 / (g - 1.0))
                pf = pb * c ** (2.0 * g / (g - 1.0)) - K.pinf
                val = (rf, uf, pf)
        rho.flat[i], u.flat[i], p.flat[i] = val
    return rho, u, p, side
