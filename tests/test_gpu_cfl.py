"""GPU tests of per-shot time steps (hho_set_dt_scale) and of the batched search of Algorithm
algo_CFL (hho_cfl_search) against the oracle's sequential search (oracle/cfl.py)."""
import math
import sys

import numpy as np
import pytest

from synth import meshes as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_per_shot_time_steps(dtype, tol):
    """Three shots with multipliers 1, 0.5, 0.3 of dt (a Ricker source in each, so the stage
    times matter too) against the oracle stepping each with its own dt; resetting the
    multipliers restores the common dt."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    say("case: per-shot dt, %s" % dtype)
    mesh = M.hanging_square(8, seed=21)
    o = Oracle(mesh, 2)
    o.set_point_sources([[0.4, 0.3]], [[0.0, 1.0]], 10.0, 0.05, 1.0)
    e = Engine(mesh, 2, dtype=dtype, n_shots=3)
    scales = [1.0, 0.5, 0.3]
    dt = e.dt_cfl(0.5)
    U0 = [np.random.default_rng(600 + i).standard_normal(o.ndof) for i in range(3)]
    for sh in range(3):
        e.set_state(U0[sh], shot=sh)
        e.set_sources(sh, [[0.4, 0.3]], [[0.0, 1.0]], 10.0, 0.05, 1.0)
    e.set_dt_scale(scales)
    e.erk_step(0.01, dt, 9)
    for sh in range(3):
        ref = o.erk(U0[sh], 0.01, dt * scales[sh], 9)
        err = rel(e.get_state(sh), ref)
        say("shot", sh, "rel L2", err)
        assert err < tol
    e.set_dt_scale(None)
    for sh in range(3):
        e.set_state(U0[sh], shot=sh)
    e.erk_step(0.0, dt, 3)
    assert rel(e.get_state(2), o.erk(U0[2], 0.0, dt, 3)) < tol
    with pytest.raises(Exception):
        e.set_dt_scale([1.0, 0.0, 1.0])
    e.close()


@pytest.mark.parametrize("s,shots", [(4, 8), (2, 5)])
def test_cfl_search_matches_oracle(s, shots):
    """hho_cfl_search with several rounds of simultaneous candidates gives the oracle's
    sequential bracket of Algorithm algo_CFL (same last stable and first unstable step count)
    and the same energy increase for every candidate judged (float64)."""
    from oracle import Oracle
    from oracle.cfl import cfl_bracket
    from paper_2505_15771_amd import Engine
    say("case: cfl search s=%d shots=%d" % (s, shots))
    mesh = M.with_materials(M.bilayer_vertical(4, p_split=0.5, seed=3))
    o = Oracle(mesh, 1)
    U0 = np.random.default_rng(44).standard_normal(o.ndof)
    n_start = 90 if s == 4 else 110
    ns, nu, tried = cfl_bracket(o, U0, 1.0, n_start, delta=0.02, s=s)
    say("oracle bracket", ns, nu, "after", len(tried), "runs")
    e = Engine(mesh, 1, rk_stages=s, n_shots=shots)
    for sh in range(shots):
        e.set_state(U0, shot=sh)
    gns, gnu, gtried = e.cfl_search(1.0, n_start, delta=0.02, eps=0.05)
    say("gpu bracket", gns, gnu, "after", len(gtried), "candidates")
    assert (gns, gnu) == (ns, nu)
    assert [t[0] for t in gtried] == [t[0] for t in tried]
    for (n1, g1), (n2, g2) in zip(gtried, tried):
        assert (math.isinf(g1) and math.isinf(g2)) or abs(g1 - g2) <= 1e-9 * max(1.0, abs(g2)), (n1, g1, g2)
    assert rel(e.get_state(0), U0) < 1e-15   # entry states restored
    e.close()


def test_cfl_search_edges_and_errors():
    """A first candidate that is already unstable gives (0, n_start); a search whose rounds run
    out reports no unstable candidate; bad arguments are refused without changing the state;
    the adjoint refuses a context with per-shot multipliers."""
    from paper_2505_15771_amd import Engine, HHOError
    mesh = M.with_materials(M.bilayer_vertical(3))
    e = Engine(mesh, 1, n_shots=4)
    U0 = np.random.default_rng(5).standard_normal(e.n_dof)
    for sh in range(4):
        e.set_state(U0, shot=sh)
    dt_big = 3.0 * e.dt_cfl(1.0)
    n_unstable = max(1, int(1.0 / dt_big))
    ns, nu, tried = e.cfl_search(1.0, n_unstable, delta=0.01)
    say("too large a step:", ns, nu, tried[:2])
    assert (ns, nu) == (0, n_unstable) and len(tried) == 1
    n_safe = int(np.ceil(1.0 / (0.2 * e.dt_cfl(1.0))))
    ns, nu, tried = e.cfl_search(1.0, n_safe, delta=0.001, max_rounds=1)
    assert nu == 0 and ns == tried[-1][0] and len(tried) == 4
    for bad in (dict(t_final=0.0, n_start=10), dict(t_final=1.0, n_start=0),
                dict(t_final=1.0, n_start=10, delta=1.5), dict(t_final=1.0, n_start=10, eps=0.0)):
        with pytest.raises(HHOError):
            e.cfl_search(**bad)
    assert rel(e.get_state(3), U0) < 1e-15
    e.close()
    a = Engine(mesh, 1)
    a.set_state(U0)
    a.set_dt_scale([0.5])
    with pytest.raises(HHOError):
        a.adjoint(0.0, a.dt_cfl(0.5), 4)
    a.set_dt_scale(None)
    J, g = a.adjoint(0.0, a.dt_cfl(0.5), 4)
    assert np.isfinite(J) and np.all(np.isfinite(g))
    a.close()


@pytest.mark.parametrize("medium", ["fluid", "solid"])
def test_cfl_against_stabilisation_weight(medium):
    """Algorithm algo_CFL over a sweep of the stabilisation weight on a pure medium (k = 1, 8x8
    quads): CFL*(eta) rises, peaks and falls, like min(eta + c1, 1/eta + c2) (Sec. 5.1), with the
    maximiser at the paper's optimal weights (Figure CFL_decoupled: eta^f = 0.8, eta^s = 1.5) with
    tau^f = eta / (rho c) and tau^s = eta rho c_S."""
    from paper_2505_15771_amd import Engine
    say("case: CFL vs eta, %s" % medium)
    code, c = (M.FLUID, 1.0) if medium == "fluid" else (M.SOLID, math.sqrt(3.0))
    mesh = M.with_materials(M.single_medium(8, code))
    etas = (0.4, 0.6, 0.8, 0.9, 1.0, 1.2, 1.6) if medium == "fluid" else (0.6, 1.0, 1.2, 1.4, 1.5, 1.6, 2.0, 2.8)
    cfl = []
    for eta in etas:
        e = Engine(mesh, 1, n_shots=16, **({"eta_f": eta} if medium == "fluid" else {"eta_s": eta}))
        U0 = M.random_state(np.full(1, e.n_dof), 9101)
        for sh in range(16):
            e.set_state(U0, shot=sh)
        ns, nu, _ = e.cfl_search(1.0, int(math.ceil(1.0 / (0.1 * e.dt_cfl(1.0)))), 0.02, 0.05)
        e.close()
        assert ns > 0 and nu > 0
        cfl.append(c * 8 / ns)
    say("  eta", etas, "CFL*", [round(v, 4) for v in cfl])
    best = int(np.argmax(cfl))
    lo, hi = (0.7, 0.9) if medium == "fluid" else (1.4, 1.6)
    assert lo <= etas[best] <= hi
    assert all(cfl[i] < cfl[i + 1] for i in range(best - 1)) or best == 0
    assert cfl[0] < 0.8 * cfl[best] and cfl[-1] < 0.8 * cfl[best]
