"""Algorithm algo_CFL (Sec. 5.1): bracketing of the explicit stability limit by energy growth.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Sequential, as the paper states it: start
from a number of steps N over the simulated time T_f, run the undriven problem, and judge the run
by its relative energy increase; while the run is stable, reduce N by delta N and run again.  The
last stable and the first unstable N bracket the limit, CFL* = c dt / h with dt = T_f / N.

Readings (the paper's text is brief here):
  * the relative energy increase of a run is the largest, over its steps n, of the increase over
    the initial energy and over the previous step's energy, (E_n - E_0)/E_0 and
    (E_n - E_{n-1})/E_{n-1} (the paper speaks of an energy increase; its algorithm prints the
    same quotients inside absolute values, which would also flag the dissipation of the
    stabilisation);  a non-finite energy counts as an infinite increase;
  * "reduce N by delta N" is N <- N - max(1, floor(delta N)).
"""
from __future__ import annotations

import math

import numpy as np


def energy_increase(E0, E):
    """Largest relative energy increase of a run with initial energy E0 and energies E[n] after
    step n + 1 (inf when an energy is not finite or E0 is not positive)."""
    if not (E0 > 0.0) or not math.isfinite(E0):
        return math.inf
    g, prev = 0.0, E0
    for e in E:
        if not math.isfinite(e):
            return math.inf
        g = max(g, (e - E0) / E0, (e - prev) / prev)
        prev = e
    return g


def candidates(n_start, delta, count):
    """The first `count` step counts N_0 = n_start, N_{j+1} = N_j - max(1, floor(delta N_j))."""
    out, n = [], int(n_start)
    while len(out) < count and n >= 1:
        out.append(n)
        n -= max(1, int(math.floor(delta * n)))
    return out


def cfl_bracket(oracle, U0, t_final, n_start, delta=0.01, eps=0.05, s=4, max_tries=1000):
    """Run Algorithm algo_CFL on the oracle from the state U0: returns (last stable N, first
    unstable N, [(N, energy increase), ...] in the order tried); 0 where none was found."""
    E0 = oracle.energy(U0)
    tried, stable = [], 0
    for n in candidates(n_start, delta, max_tries):
        _, E = oracle.erk(U0, 0.0, t_final / n, n, s=s, energies=True)
        g = energy_increase(E0, E)
        tried.append((n, g))
        if g > eps:
            return stable, n, tried
        stable = n
    return stable, 0, tried
