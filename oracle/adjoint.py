"""Receiver misfit and its discrete adjoint gradient for the explicit Runge-Kutta path.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain and slow.  misfit_gradient keeps
every stage state of every step in memory (small meshes, short runs); misfit_gradient_checkpointed
keeps the state every `every` steps and recomputes one segment's stage states at a time during
the reverse sweep (the same arithmetic, for long runs on larger meshes).

Forward (Sec. 4.2, eq. ERK / eq. ex_solve): U^{n+1} = U^n + dt sum_i b_i k_i, k_i = L Y_i + M^{-1} F(t_i),
Y_1 = U^n, Y_{i+1} = U^n + dt a_{i+1,i} k_i (tableaux whose matrix is subdiagonal: ERK(2), ERK(4)).
Misfit J = 1/2 dt sum_{n=1..N} sum_r |R_r U^n - d_r^n|^2, R_r the point evaluation of p (fluid) or
v (solid) at receiver r (the sensors of Sec. 5.2).
Reverse sweep of each step from lambda = lambda^{n+1}:
  mu_s = dt b_s lambda,  mu_i = dt b_i lambda + dt a_{i+1,i} L^T mu_{i+1}  (i = s-1 .. 1),
  lambda^n = lambda + sum_i L^T mu_i + dJ/dU^n,
  dJ/dtheta += sum_i mu_i^T (d/dtheta)(L Y_i + M^{-1} F(t_i)).
"""
from __future__ import annotations

import numpy as np

from .oracle import ERK_TABLEAUX


class Receivers:
    """Point evaluation R_r of p (field 0, fluid) or (v_x, v_y) (field 1, solid) in the cell basis."""

    def __init__(self, o, xy, field):
        self.o = o
        self.items = []
        for (x, y), f in zip(np.asarray(xy, float), np.asarray(field)):
            c = o.locate(x, y)
            if c < 0:
                raise ValueError("receiver outside the mesh")
            if int(f) != int(o.medium[c]):
                raise ValueError("receiver field does not match the medium of its cell")
            phi = o.basis(c, x, y)[0]
            idx = [o.offsets[c] + comp * o.N + np.arange(o.N) for comp in range(1 + int(f))]
            self.items.append((idx, phi))

    def apply(self, U):
        out = np.zeros((len(self.items), 2))
        for r, (idx, phi) in enumerate(self.items):
            for comp, ix in enumerate(idx):
                out[r, comp] = phi @ U[ix]
        return out

    def apply_T(self, res):
        out = np.zeros(self.o.ndof)
        for r, (idx, phi) in enumerate(self.items):
            for comp, ix in enumerate(idx):
                out[ix] += res[r, comp] * phi
        return out


def forward(o, U0, t0, dt, nsteps, s=4, n0=0):
    """Stage states Y_i and stage derivatives k_i of every step, and U^0..U^N; the steps are
    steps n0 .. n0 + nsteps - 1 of a run started at t0 (stage times t0 + (n + c_i) dt)."""
    A, b, c = ERK_TABLEAUX[s]
    U = np.array(U0, float, copy=True)
    Us, stages = [U], []
    for n in range(n0, n0 + nsteps):
        Ys, ks = [], []
        for i in range(s):
            Y = U + dt * sum(A[i, j] * ks[j] for j in range(i)) if i else U
            ks.append(o.rhs(Y, t0 + (n + c[i]) * dt))
            Ys.append(Y)
        U = U + dt * sum(b[i] * ks[i] for i in range(s))
        Us.append(U)
        stages.append((Ys, ks))
    return Us, stages


def misfit(rec, Us, d_obs, dt):
    """J = 1/2 dt sum_{n>=1} |R U^n - d^n|^2 (d_obs[n-1] holds the data of step n)."""
    return 0.5 * dt * sum(float(np.sum((rec.apply(Us[n]) - d_obs[n - 1]) ** 2)) for n in range(1, len(Us)))


def misfit_gradient(o, U0, t0, dt, nsteps, rec, d_obs, s=4):
    """J and dJ/dtheta [n_cells, 3] (fluid: rho, c, 0; solid: rho, lambda, mu)."""
    A, b, c = ERK_TABLEAUX[s]
    for i in range(s):
        for j in range(i - 1):
            if A[i, j] != 0.0:
                raise ValueError("the reverse sweep here assumes a subdiagonal Runge-Kutta matrix")
    Us, stages = forward(o, U0, t0, dt, nsteps, s)
    J = misfit(rec, Us, d_obs, dt)
    lam = dt * rec.apply_T(rec.apply(Us[nsteps]) - d_obs[nsteps - 1])
    grad = np.zeros((o.nc, 3))
    for n in reversed(range(nsteps)):
        Ys, ks = stages[n]
        total = lam.copy()
        ybar_next = None
        for i in reversed(range(s)):
            mu = dt * b[i] * lam
            if i < s - 1:
                mu = mu + dt * A[i + 1, i] * ybar_next
            ybar = o.rhs_T(mu)
            o.grad_terms(Ys[i], ks[i], mu, grad)
            total += ybar
            ybar_next = ybar
        if n >= 1:
            total += dt * rec.apply_T(rec.apply(Us[n]) - d_obs[n - 1])
        lam = total
    return J, grad


def _check_subdiagonal(A, s):
    for i in range(s):
        for j in range(i - 1):
            if A[i, j] != 0.0:
                raise ValueError("the reverse sweep here assumes a subdiagonal Runge-Kutta matrix")


def _reverse_step(o, A, b, s, dt, lam, Ys, ks, grad):
    """One step of the reverse sweep (module docstring) from lambda^{n+1}; returns
    lambda^{n+1} + sum_i L^T mu_i, to which the caller adds dJ/dU^n."""
    total = lam.copy()
    ybar_next = None
    for i in reversed(range(s)):
        mu = dt * b[i] * lam
        if i < s - 1:
            mu = mu + dt * A[i + 1, i] * ybar_next
        ybar = o.rhs_T(mu)
        o.grad_terms(Ys[i], ks[i], mu, grad)
        total += ybar
        ybar_next = ybar
    return total


def misfit_gradient_checkpointed(o, U0, t0, dt, nsteps, rec, d_obs, every=50, s=4, return_traces=False):
    """J and dJ/dtheta as misfit_gradient, with checkpoints: the forward pass keeps U^n for
    n = 0, every, 2 every, ...; the reverse sweep, segment by segment from the last, recomputes the
    stage states of the segment from its checkpoint and runs the reverse steps of its steps.
    With return_traces, also the receiver values R U^n of the forward pass [nsteps, n_rec, 2]."""
    A, b, c = ERK_TABLEAUX[s]
    _check_subdiagonal(A, s)
    ckpt = {}
    U = np.array(U0, float, copy=True)
    terms, traces = [], []
    for g0 in range(0, nsteps, every):
        ckpt[g0] = U
        Us, _ = forward(o, U, t0, dt, min(every, nsteps - g0), s, n0=g0)
        for m in range(1, len(Us)):
            r = rec.apply(Us[m])
            traces.append(r)
            terms.append(float(np.sum((r - d_obs[g0 + m - 1]) ** 2)))
        U = Us[-1]
    J = 0.5 * dt * sum(terms)
    lam = dt * rec.apply_T(rec.apply(U) - d_obs[nsteps - 1])
    grad = np.zeros((o.nc, 3))
    for g0 in reversed(range(0, nsteps, every)):
        Us, stages = forward(o, ckpt[g0], t0, dt, min(every, nsteps - g0), s, n0=g0)
        for m in reversed(range(len(stages))):
            Ys, ks = stages[m]
            lam_n = _reverse_step(o, A, b, s, dt, lam, Ys, ks, grad)
            n = g0 + m
            if n >= 1:
                lam_n += dt * rec.apply_T(rec.apply(Us[m]) - d_obs[n - 1])
            lam = lam_n
    return (J, grad, np.array(traces)) if return_traces else (J, grad)
