"""Manufactured smooth solutions for the oracle's convergence pins (test infrastructure).

Adapted from the sinusoidal solution eq. non_poly_sol (Sec. 5.1) to the unit
square with the interface at y = 1/2 (solid below, fluid above):

  fluid potential   u   = eta^2 sin(w pi eta) sin(w pi x) sin(theta pi t + phi),  eta = 2(y - 1/2)
  solid displacement u_x = u_y = zeta^2 cos(w pi zeta / 2) sin(w pi x) cos(theta pi t + phi),
                     zeta = 2(1/2 - y)

with p = du/dt, m = grad(u)/rho (so rho dm/dt - grad p = 0), v = du/dt and
s = C grad_sym(u) (so C^{-1} ds/dt - grad_sym v = 0).  The sources follow from
eq. continuous_acoustic and eq. continuous_elastic_eq:
  f^f = (1/kappa) d2u/dt2 - div(grad u / rho),   f^s = rho d2u/dt2 - div(s).
For odd w every field and its first derivatives vanish on the interface, so
the coupling conditions eq. continuous_coupling hold, and p = 0, v = 0 on the
outer boundary (homogeneous Dirichlet, Sec. 2.1).

Derivatives are taken symbolically (sympy) so the forcing is exact.
"""
from __future__ import annotations

import numpy as np
import sympy as sp

X, Y, T = sp.symbols("x y t", real=True)
SQ2 = sp.sqrt(2)


def _lam(expr):
    f = sp.lambdify((X, Y, T), expr, "numpy")

    def g(x, y, t, _f=f):
        return np.broadcast_to(np.asarray(_f(x, y, t), dtype=np.float64), np.shape(x)).copy()
    return g


class Manufactured:
    """Exact fields and separable forcing of the adapted sinusoidal solution."""

    def __init__(self, omega=1, theta=np.sqrt(2.0), phase=0.0, rho_f=1.0, kappa=1.0,
                 rho_s=1.0, lam=1.0, mu=1.0):
        w, th, ph = sp.nsimplify(omega), sp.Float(theta, 30), sp.Float(phase, 30)
        rf, ka, rs = sp.Float(rho_f, 30), sp.Float(kappa, 30), sp.Float(rho_s, 30)
        la, mu_ = sp.Float(lam, 30), sp.Float(mu, 30)
        eta = 2 * (Y - sp.Rational(1, 2))
        zeta = 2 * (sp.Rational(1, 2) - Y)
        u = eta ** 2 * sp.sin(w * sp.pi * eta) * sp.sin(w * sp.pi * X) * sp.sin(th * sp.pi * T + ph)
        us = zeta ** 2 * sp.cos(w * sp.pi * zeta / 2) * sp.sin(w * sp.pi * X) * sp.cos(th * sp.pi * T + ph)
        ux, uy = us, us
        p = sp.diff(u, T)
        mx, my = sp.diff(u, X) / rf, sp.diff(u, Y) / rf
        ff = sp.diff(u, T, 2) / ka - (sp.diff(mx, X) + sp.diff(my, Y))
        vx, vy = sp.diff(ux, T), sp.diff(uy, T)
        exx, eyy = sp.diff(ux, X), sp.diff(uy, Y)
        exy = (sp.diff(ux, Y) + sp.diff(uy, X)) / 2
        tr = exx + eyy
        sxx, syy, sxy = la * tr + 2 * mu_ * exx, la * tr + 2 * mu_ * eyy, 2 * mu_ * exy
        fsx = rs * sp.diff(ux, T, 2) - (sp.diff(sxx, X) + sp.diff(sxy, Y))
        fsy = rs * sp.diff(uy, T, 2) - (sp.diff(sxy, X) + sp.diff(syy, Y))
        self.fluid = [_lam(e) for e in (p, mx, my)]
        self.solid = [_lam(e) for e in (vx, vy, sxx, syy, SQ2 * sxy)]
        # forcing split as spatial part x time factor (sin(theta pi t + phase) for the fluid,
        # cos(theta pi t + phase) = sin(theta pi t + phase + pi/2) for the solid)
        tf = sp.sin(th * sp.pi * T + ph)
        ts = sp.cos(th * sp.pi * T + ph)
        self._ff_sp = _lam(sp.simplify(ff / tf))
        self._fs_sp = [_lam(sp.simplify(fsx / ts)), _lam(sp.simplify(fsy / ts))]
        self.omega_t = float(theta) * np.pi
        self.phase = float(phase)
        self.exprs = dict(u=u, us=us, ff=ff, fsx=fsx, fsy=fsy, p=p, mx=mx, my=my)

    def fields(self, t):
        """(fluid 3 callables, solid 5 callables) of (x, y) at time t."""
        fl = [lambda x, y, f=f: f(x, y, t) for f in self.fluid]
        so = [lambda x, y, f=f: f(x, y, t) for f in self.solid]
        return fl, so

    def forcing_terms(self):
        """Spatial load functions and (omega, phase) of the two separable terms:
        term 0 acts on the fluid p rows, term 1 on the solid v rows."""
        z = lambda x, y: np.zeros_like(x)
        f0 = ([lambda x, y: self._ff_sp(x, y, 0.0), z, z], [z] * 5)
        f1 = ([z] * 3, [lambda x, y: self._fs_sp[0](x, y, 0.0), lambda x, y: self._fs_sp[1](x, y, 0.0), z, z, z])
        return [f0, f1], np.array([self.omega_t, self.omega_t]), np.array([self.phase, self.phase + np.pi / 2])


class StandingWave:
    """Pure acoustic standing wave p = cos(sqrt(2) pi c t) sin(pi x) sin(pi y) on the unit
    square with m from rho dm/dt = grad p (zero source, Dirichlet-compatible)."""

    def __init__(self, rho=1.0, c=1.0):
        self.rho, self.c = rho, c
        self.w = np.sqrt(2.0) * np.pi * c

    def fields(self, t):
        w, r = self.w, self.rho
        p = lambda x, y: np.cos(w * t) * np.sin(np.pi * x) * np.sin(np.pi * y)
        mx = lambda x, y: np.sin(w * t) / (w * r) * np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
        my = lambda x, y: np.sin(w * t) / (w * r) * np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
        z = lambda x, y: np.zeros_like(x)
        return [p, mx, my], [z] * 5
