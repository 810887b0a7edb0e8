"""CPU pins of Algorithm algo_CFL (Sec. 5.1) as the oracle runs it (oracle/cfl.py): the energy
criterion and the step-count sequence on hand-made inputs, the bracket against the strict
spectral stability limit of the condensed operator, and the ratios of CFL* between stage counts
against the paper's Table tab::ratio_ERK (tests/golden/cfl_ratio_erk.txt)."""
import math
import os
from math import factorial

import numpy as np
import pytest

from synth import meshes as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfl_ratio_erk.txt")


def test_energy_increase_criterion():
    from oracle.cfl import energy_increase
    assert energy_increase(1.0, [0.99, 0.98, 0.5]) == 0.0             # decay is not an increase
    assert energy_increase(1.0, [0.99, 1.02, 1.05, 1.08]) == pytest.approx(0.08)
    assert energy_increase(1.0, [0.5, 0.54]) == pytest.approx(0.08)   # over the previous energy
    assert energy_increase(2.0, [2.2]) == pytest.approx(0.1)
    assert energy_increase(1.0, [1.0, float("nan")]) == math.inf
    assert energy_increase(0.0, [1.0]) == math.inf


def test_candidate_step_counts():
    from oracle.cfl import candidates
    assert candidates(100, 0.01, 4) == [100, 99, 98, 97]             # floor(0.99) = 0 -> at least 1
    assert candidates(250, 0.01, 4) == [250, 248, 246, 244]
    assert candidates(1000, 0.05, 3) == [1000, 950, 903]
    assert candidates(2, 0.5, 5) == [2, 1]


def _strict_dt(lam, s):
    """Largest dt with |R(dt lambda)| <= 1 on the spectrum, R(z) = sum_{j<=s} z^j / j! (the
    amplification polynomial of every tableau of eq. ERK)."""
    def ok(dt):
        z = dt * lam
        return np.max(np.abs(sum(z ** j / factorial(j) for j in range(s + 1)))) <= 1 + 1e-12
    lo, hi = 0.0, 1.0
    while ok(hi):
        hi *= 2
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ok(mid) else (lo, mid)
    return lo


@pytest.mark.parametrize("shape,p_split", [("quads", 0.0), ("triangles", 1.0)])
@pytest.mark.parametrize("s", [2, 4])
def test_bracket_meets_spectral_limit(shape, p_split, s):
    """From a random state (every eigenmode excited) over T_f = 1, the first unstable step of
    Algorithm algo_CFL lies above the strict spectral limit dt* of the oracle's dense operator,
    and the last stable one within 2 % of it (delta = 2 %)."""
    from oracle import Oracle
    from oracle.cfl import cfl_bracket
    m = M.with_materials(M.bilayer_vertical(4, p_split=p_split, seed=3))
    o = Oracle(m, 1)
    dts = _strict_dt(np.linalg.eigvals(o.dense_operator()), s)
    U0 = np.random.default_rng(3).standard_normal(o.ndof)
    ns, nu, tried = cfl_bracket(o, U0, 1.0, int(math.ceil(1.0 / (0.7 * dts))), delta=0.02, s=s)
    assert ns > 0 and nu > 0
    assert 1.0 / nu > dts
    assert 1.0 / ns < 1.02 * dts


def _paper_initial_state(o, omega=5.0, theta=math.sqrt(2.0)):
    """L2 projection of the sinusoidal solution of eq. non_poly_sol at t = 0 on the CFL geometry
    (rho = 1, lambda = mu = 1 in the solid): p = theta pi x^2 sin(w pi x) sin(w pi y), m = 0;
    v = 0, s = C grad_sym(u) with u_x = u_y = x^2 cos(w pi x / 2) sin(w pi y) (s_3 carries the
    sqrt(2) of the E basis)."""
    pi = math.pi
    dudx = lambda x, y: (2 * x * np.cos(omega * pi * x / 2)
                         - x ** 2 * (omega * pi / 2) * np.sin(omega * pi * x / 2)) * np.sin(omega * pi * y)
    dudy = lambda x, y: x ** 2 * np.cos(omega * pi * x / 2) * omega * pi * np.cos(omega * pi * y)
    fluid = [lambda x, y: theta * pi * x ** 2 * np.sin(omega * pi * x) * np.sin(omega * pi * y),
             lambda x, y: 0 * x, lambda x, y: 0 * x]
    solid = [lambda x, y: 0 * x, lambda x, y: 0 * x,
             lambda x, y: (dudx(x, y) + dudy(x, y)) + 2 * dudx(x, y),
             lambda x, y: (dudx(x, y) + dudy(x, y)) + 2 * dudy(x, y),
             lambda x, y: math.sqrt(2.0) * (dudy(x, y) + dudx(x, y))]
    return o.project(fluid, solid)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_stage_count_ratios_match_paper(k):
    """With the paper's setting (CFL geometry at h = 1/8, sinusoidal initial state, T_f = 1,
    delta = 1 %), the CFL* brackets of ERK(3) and ERK(4) relative to ERK(2) reproduce the
    'Ratio wrt s' row of Table tab::ratio_ERK within 2 % (the ratios follow from the stability
    polynomials and the spectrum's shape).  The absolute values are not pinned: they depend on
    the readings of h and of the solid stabilisation speed (see the readings of the CFL step)."""
    from oracle import Oracle
    from oracle.cfl import cfl_bracket
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    paper = {(int(r[0]), int(r[1])): (float(r[2]), float(r[3])) for r in rows}
    n = 8
    o = Oracle(M.with_materials(M.bilayer_vertical(n)), k)
    U0 = _paper_initial_state(o)
    mid = {}
    for s in (2, 3, 4):
        n0 = int(math.ceil(1.0 / (0.8 * paper[(k, s)][0] / math.sqrt(3.0) / n)))
        ns, nu, _ = cfl_bracket(o, U0, 1.0, n0, delta=0.01, s=s)
        assert ns > 0 and nu > 0
        mid[s] = 0.5 * (1.0 / ns + 1.0 / nu)
    for s in (3, 4):
        assert mid[s] / mid[2] == pytest.approx(paper[(k, s)][1], rel=0.02)
