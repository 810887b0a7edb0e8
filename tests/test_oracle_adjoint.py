"""Pins of the oracle's discrete adjoint (receiver-misfit gradient w.r.t. per-cell materials).

* the transposed condensed operator satisfies <L x, y> = <x, L^T y> (dot-product test);
* the explicitly assembled blocks reproduce the condensed operator of eq. ex_solve;
* the stage-by-stage forward sweep equals the oracle's ERK stepping;
* the gradient matches central finite differences of J on fluid and solid cells, for every
  parameter (fluid rho, c; solid rho, lambda, mu), with a point source and receivers in both media,
  for k = 1, 2, 3 and both readings of the solid stabilisation speed (tau^s on c_P or on c_S: the
  derivative of tau with respect to the materials differs between them), on cells beside the
  fluid-solid interface (whose face solves couple the two media) and elsewhere;
* the checkpointed reverse sweep returns the same J and gradient as the sweep that stores every
  stage.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.adjoint import Receivers, forward, misfit, misfit_gradient, misfit_gradient_checkpointed
from synth import meshes as M


def small_mesh(seed=3):
    refine = np.random.default_rng(seed).random((6, 6)) < 0.25
    return M.with_materials(M.unit_square(6, p_split=0.5, seed=seed, refine=refine), perturb=0.1, seed=seed + 1)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_dot_product_and_blocks(k):
    mesh = small_mesh()
    o = Oracle(mesh, k)
    rng = np.random.default_rng(k)
    x, y = rng.standard_normal(o.ndof), rng.standard_normal(o.ndof)
    Lx, LTy = o.rhs(x), o.rhs_T(y)
    assert abs(Lx @ y - x @ LTy) < 1e-13 * np.linalg.norm(Lx) * np.linalg.norm(y)
    assert np.linalg.norm(-o.inv_mass(o.keff(x)) - Lx) < 1e-13 * np.linalg.norm(Lx)


def setup_problem(k=2, nsteps=25, stab_speed=0):
    mesh = small_mesh(5)
    src = [[0.45, 0.3]]
    rec_xy = [[0.3, 0.8], [0.7, 0.65], [0.25, 0.2], [0.8, 0.35]]
    rec_f = [0, 0, 1, 1]
    dt = 0.4 * 0.138 / 6 / np.sqrt(3.0)
    # synthetic observed data from a +-5 % perturbed model
    true = dict(mesh)
    rng = np.random.default_rng(77)
    for key in ("rho", "a", "b"):
        true[key] = np.asarray(mesh[key]) * (1 + rng.uniform(-0.05, 0.05, len(mesh["rho"])))
    ot = Oracle(true, k, stab_speed=stab_speed)
    ot.set_point_sources(src, [[0.0, 1.0]], 10.0, 0.12, 1.0)
    Us, _ = forward(ot, np.zeros(ot.ndof), 0.0, dt, nsteps)
    rt = Receivers(ot, rec_xy, rec_f)
    d_obs = np.array([rt.apply(Us[n]) for n in range(1, nsteps + 1)])
    return mesh, src, rec_xy, rec_f, dt, d_obs


def J_of(mesh, k, src, rec_xy, rec_f, dt, d_obs, nsteps, stab_speed=0):
    o = Oracle(mesh, k, stab_speed=stab_speed)
    o.set_point_sources(src, [[0.0, 1.0]], 10.0, 0.12, 1.0)
    Us, _ = forward(o, np.zeros(o.ndof), 0.0, dt, nsteps)
    return misfit(Receivers(o, rec_xy, rec_f), Us, d_obs, dt)


def test_forward_sweep_matches_erk():
    mesh = small_mesh()
    o = Oracle(mesh, 2)
    o.set_point_sources([[0.45, 0.3]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
    U0 = np.random.default_rng(1).standard_normal(o.ndof)
    Us, _ = forward(o, U0, 0.05, 1e-3, 6)
    ref = o.erk(U0, 0.05, 1e-3, 6)
    assert np.linalg.norm(Us[-1] - ref) <= 1e-14 * np.linalg.norm(ref)


def interface_cells(o):
    """Cells with a face on the fluid-solid interface, per medium."""
    _, fc, _ = o.face_info()
    both = fc[(fc[:, 0] >= 0) & (fc[:, 1] >= 0)]
    itf = both[o.medium[both[:, 0]] != o.medium[both[:, 1]]].reshape(-1)
    return [sorted(set(int(c) for c in itf if o.medium[c] == m)) for m in (0, 1)]


@pytest.mark.slow
@pytest.mark.parametrize("k,stab_speed", [(2, 0), (1, 1), (2, 1), (3, 1)])
def test_gradient_matches_finite_differences(k, stab_speed):
    nsteps = 25
    mesh, src, rec_xy, rec_f, dt, d_obs = setup_problem(k, nsteps, stab_speed)
    o = Oracle(mesh, k, stab_speed=stab_speed)
    o.set_point_sources(src, [[0.0, 1.0]], 10.0, 0.12, 1.0)
    rec = Receivers(o, rec_xy, rec_f)
    J, grad = misfit_gradient(o, np.zeros(o.ndof), 0.0, dt, nsteps, rec, d_obs)
    assert J > 0
    med = np.asarray(mesh["medium"])
    rng = np.random.default_rng(9 + k + 10 * stab_speed)
    itf_f, itf_s = interface_cells(o)
    cells = [int(rng.choice(itf_f)), int(rng.choice(itf_s))]
    cells += [int(c) for c in rng.choice(np.setdiff1d(np.where(med == 0)[0], cells), 2, replace=False)]
    cells += [int(c) for c in rng.choice(np.setdiff1d(np.where(med == 1)[0], cells), 2, replace=False)]
    checked = 0
    for c in cells:
        params = [("rho", 0), ("a", 1)] if med[c] == 0 else [("rho", 0), ("a", 1), ("b", 2)]
        for key, q in params:
            h = 1e-5 * abs(mesh[key][c])
            vals = []
            for sgn in (1, -1):
                m2 = dict(mesh)
                m2[key] = np.array(mesh[key], float, copy=True)
                m2[key][c] += sgn * h
                vals.append(J_of(m2, k, src, rec_xy, rec_f, dt, d_obs, nsteps, stab_speed))
            fd = (vals[0] - vals[1]) / (2 * h)
            scale = max(abs(fd), 1e-3 * np.max(np.abs(grad)))
            assert abs(grad[c, q] - fd) < 1e-6 * scale + 1e-12 * J, (c, key, grad[c, q], fd)
            checked += 1
    assert checked == 15


@pytest.mark.parametrize("k,every", [(1, 7), (2, 25), (2, 4)])
def test_checkpointed_sweep_matches_full_sweep(k, every):
    """Checkpoints every `every` steps (25 steps: a ragged last segment, one segment, many)."""
    nsteps = 25
    mesh, src, rec_xy, rec_f, dt, d_obs = setup_problem(k, nsteps)
    o = Oracle(mesh, k)
    o.set_point_sources(src, [[0.0, 1.0]], 10.0, 0.12, 1.0)
    rec = Receivers(o, rec_xy, rec_f)
    U0 = 0.01 * np.random.default_rng(4).standard_normal(o.ndof)
    J0, g0 = misfit_gradient(o, U0, 0.0, dt, nsteps, rec, d_obs)
    J1, g1 = misfit_gradient_checkpointed(o, U0, 0.0, dt, nsteps, rec, d_obs, every=every)
    assert J1 == J0
    assert np.linalg.norm(g1 - g0) <= 1e-14 * np.linalg.norm(g0)
