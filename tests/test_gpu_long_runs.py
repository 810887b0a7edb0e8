"""GPU parity over the full length of the workloads, against the FP64 oracle, checked per run.

* the 256 x 256 hybrid workload (two-material unit square, random quads / split triangles, every
  material +-10 %) at k = 2 for its 2000 RK4 steps, float64 and float32 stepping, with its Ricker
  point source and eight receivers (four of p in the fluid, four of v in the solid); at k = 3 in
  float32 for 500 steps from a random state;
* the adjoint workload as specified: 128 x 128 hybrid mesh, k = 2, 1000 steps with checkpoints
  every 50, 32 receivers, data from a +-5 % perturbed model: J and the gradient against the
  oracle's checkpointed reverse sweep, and against central finite differences (relative step
  1e-4, float64 forward runs) for every parameter of 20 seeded cells, 10 per medium;
* a mesh whose cells all have shapes of their own (every group pooled) for 70 steps, which
  replays the 64-, 4- and 2-step graphs, with a source, receivers and the energy history.

Besides the relative L2 norm of the whole state, the cells beside the fluid-solid interface are
checked on their own: the largest cell-wise error there, over the largest cell-wise norm there,
must meet the same tolerance (an error confined to the interface would hide in the global norm).
Tolerances: 1e-12 float64, 1e-5 float32 (state, traces, energies); adjoint: J 1e-11 and gradient
1e-11 relative in float64, in float32 2e-5 times the ratio of the trace amplitude to the residual
amplitude (J is a sum of squared residuals R U - d, which cancels that much of the traces).
"""
import sys

import numpy as np
import pytest

from synth import meshes as M

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def interface_cells(o):
    _, fc, _ = o.face_info()
    both = fc[(fc[:, 0] >= 0) & (fc[:, 1] >= 0)]
    return np.unique(both[o.medium[both[:, 0]] != o.medium[both[:, 1]]].reshape(-1))


def interface_error(o, cells, got, ref):
    """max over the given cells of |got_T - ref_T| / max over them of |ref_T| (Euclidean norms of
    the cell blocks)."""
    err = [np.linalg.norm(got[o.offsets[c]:o.offsets[c + 1]] - ref[o.offsets[c]:o.offsets[c + 1]]) for c in cells]
    mag = [np.linalg.norm(ref[o.offsets[c]:o.offsets[c + 1]]) for c in cells]
    return float(max(err) / max(max(mag), 1e-300))


REC_XY = np.array([[0.2, 0.75], [0.4, 0.75], [0.6, 0.75], [0.8, 0.75],
                   [0.2, 0.35], [0.4, 0.35], [0.6, 0.35], [0.8, 0.35]])
REC_F = np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32)
SRC, DIRS = [[0.5, 0.25]], [[0.0, 1.0]]


def _oracle_run(o, U, t0, dt, n, rec_xy, rec_f):
    """n oracle steps from U; receiver values after every step [n, n_rec, 2]."""
    tr = np.zeros((n, len(rec_f), 2))
    for m in range(n):
        U = o.erk(U, t0 + m * dt, dt, 1)
        for r, (x, y) in enumerate(rec_xy):
            v = o.point_values(U, x, y)[1]
            tr[m, r, :1 + int(rec_f[r])] = v[:1 + int(rec_f[r])]
    return U, tr


def _hybrid_run(k, dtypes, nsteps, block, random_start=False):
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    mesh = M.hybrid_square(256)
    o = Oracle(mesh, k)
    o.set_point_sources(SRC, DIRS, 10.0, 0.12, 1.0)
    itf = interface_cells(o)
    engines = {}
    for d in dtypes:
        e = Engine(mesh, k, dtype=d)
        e.set_sources(0, SRC, DIRS, 10.0, 0.12, 1.0)
        e.set_receivers(REC_XY, REC_F)
        e.autotune()  # the launch configuration the benchmark times
        engines[d] = e
    dt = engines[dtypes[0]].dt_cfl(0.5)
    U = 1e-3 * np.random.default_rng(2003).standard_normal(o.ndof) if random_start else np.zeros(o.ndof)
    for e in engines.values():
        e.set_state(U)
    t = 0.0
    for b in range(nsteps // block):
        U, tr = _oracle_run(o, U, t, dt, block, REC_XY, REC_F)
        for d, e in engines.items():
            e.erk_step(t, dt, block)
            got = e.get_state()
            eu, et, ei = rel(got, U), rel(e.traces(), tr), interface_error(o, itf, got, U)
            say("k=%d %s steps %d: state %.3e traces %.3e interface cells %.3e" % (k, d, (b + 1) * block, eu, et, ei))
            tol = TOL64 if d == "f64" else TOL32
            assert eu < tol and et < tol and ei < tol
        t += block * dt
    for e in engines.values():
        e.close()


def test_hybrid256_k2_2000_steps():
    """k = 2, 2000 steps (the paper-sized run), float64 and float32, checked every 500 steps."""
    say("case: hybrid 256 k=2, 2000 steps, f64 + f32, source + 8 receivers")
    _hybrid_run(2, ("f64", "f32"), 2000, 500)


def test_hybrid256_k3_float32_500_steps():
    """k = 3, float32, 500 steps from a seeded random state with the source: in 500 steps the
    Ricker pulse does not reach the interface, whose cells would hold only the exponentially small
    tail of the source (values near 1e-40, below float32's range, where the relative measure says
    nothing), so every cell starts with data."""
    say("case: hybrid 256 k=3, 500 steps, f32, random state + source + 8 receivers")
    _hybrid_run(3, ("f32",), 500, 250, random_start=True)


def test_adjoint_workload_as_specified():
    """J and dJ/d(materials) on the adjoint workload, float64 and float32, against the oracle's
    checkpointed reverse sweep; float64 gradient against central finite differences."""
    from oracle import Oracle
    from oracle.adjoint import Receivers, forward, misfit_gradient_checkpointed
    from paper_2505_15771_amd import Engine
    say("case: adjoint workload 128x128 k=2, 1000 steps, checkpoints every 50")
    k, nsteps, every, f0, t0 = 2, 1000, 50, 10.0, 0.12
    mesh = M.adjoint_square(128)
    true = M.perturbed_model(mesh, seed=5002, amount=0.05)
    rec_xy, rec_f = M.adjoint_receivers()
    dt = Engine(mesh, k).dt_cfl(0.5)
    # observed data: the oracle on the perturbed model
    ot = Oracle(true, k)
    ot.set_point_sources(SRC, DIRS, f0, t0, 1.0)
    rt = Receivers(ot, rec_xy, rec_f)
    d_obs = np.zeros((nsteps, len(rec_f), 2))
    U = np.zeros(ot.ndof)
    for g0 in range(0, nsteps, every):
        Us, _ = forward(ot, U, 0.0, dt, every, n0=g0)
        for m in range(1, len(Us)):
            d_obs[g0 + m - 1] = rt.apply(Us[m])
        U = Us[-1]
    del ot
    o = Oracle(mesh, k)
    o.set_point_sources(SRC, DIRS, f0, t0, 1.0)
    J0, g0, tr0 = misfit_gradient_checkpointed(o, np.zeros(o.ndof), 0.0, dt, nsteps, Receivers(o, rec_xy, rec_f),
                                               d_obs, every=every, return_traces=True)
    # float32: the traces carry a relative error of up to the stepping tolerance (1e-5); J is a sum
    # of squared residuals R U - d, about `amp` times smaller than the traces, so its relative error
    # and the gradient's are bounded by 2 x 1e-5 x amp
    amp = float(np.linalg.norm(tr0) / np.linalg.norm(tr0 - d_obs))
    say("oracle J", J0, "trace / residual amplitude", amp)
    res = {}
    for d in ("f64", "f32"):
        e = Engine(mesh, k, dtype=d)
        e.set_sources(0, SRC, DIRS, f0, t0, 1.0)
        e.set_receivers(rec_xy, rec_f)
        J, g = e.adjoint(0.0, dt, nsteps, d_obs, every)
        res[d] = g
        say(d, "J rel", abs(J - J0) / J0, "grad rel L2", rel(g, g0))
        if d == "f64":
            assert abs(J - J0) < 1e-11 * J0 and rel(g, g0) < 1e-11
        else:
            assert abs(J - J0) < 2e-5 * amp * J0 and rel(g, g0) < 2e-5 * amp
        e.close()
    # central finite differences of J (float64 forward runs on the GPU) on 20 seeded cells
    grad = res["f64"]

    def J_of(m2):
        e = Engine(m2, k)
        e.set_sources(0, SRC, DIRS, f0, t0, 1.0)
        e.set_receivers(rec_xy, rec_f)
        e.erk_step(0.0, dt, nsteps)
        v = 0.5 * dt * float(np.sum((e.traces(0) - d_obs) ** 2))
        e.close()
        return v

    med = np.asarray(mesh["medium"])
    xy = np.asarray(mesh["xy"]).reshape(-1, 2)
    bc = np.array([xy[mesh["cell_vtx"][mesh["cell_ptr"][c]:mesh["cell_ptr"][c + 1]]].mean(axis=0)
                   for c in range(len(med))])
    # cells of the region the waves reach between the source and the receivers
    near = np.where((np.abs(bc[:, 0] - 0.5) < 0.35) & (bc[:, 1] > 0.15) & (bc[:, 1] < 0.85))[0]
    rng = np.random.default_rng(5004)
    cells = list(rng.choice(near[med[near] == 0], 10, replace=False)) + \
        list(rng.choice(near[med[near] == 1], 10, replace=False))
    gmax = float(np.max(np.abs(grad)))
    checked = 0
    for c in cells:
        params = [("rho", 0), ("a", 1)] if med[c] == 0 else [("rho", 0), ("a", 1), ("b", 2)]
        for key, q in params:
            h = 1e-4 * abs(mesh[key][c])
            vals = []
            for sgn in (1, -1):
                m2 = dict(mesh)
                m2[key] = np.array(mesh[key], float, copy=True)
                m2[key][c] += sgn * h
                vals.append(J_of(m2))
            fd = (vals[0] - vals[1]) / (2 * h)
            say("cell", int(c), key, "adjoint", grad[c, q], "fd", fd)
            assert abs(grad[c, q] - fd) < 1e-5 * max(abs(fd), 1e-3 * gmax), (c, key, grad[c, q], fd)
            checked += 1
    assert checked == 50


def test_pooled_mesh_70_steps_with_source_receivers_energy():
    """Every vertex moved (all groups pooled: the pooled launch alone advances the clock), 70 steps
    in one call (graphs of 64, 4 and 2 steps), Ricker source, receivers in both media and the
    energy history, float64 against the oracle step by step; float32 state and traces."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    say("case: fully pooled mesh, 70 steps, source + receivers + energy")
    mesh = M.with_materials(M.perturbed_square(8, seed=11), perturb=0.1, seed=12)
    k, nsteps = 2, 70
    o = Oracle(mesh, k)
    src, dirs = [[0.4, 0.3]], [[0.6, -0.8]]
    rx, fld = np.array([[0.3, 0.7], [0.6, 0.2]]), np.array([0, 1], np.int32)
    o.set_point_sources(src, dirs, 10.0, 0.05, 1.0)
    U0 = np.random.default_rng(70).standard_normal(o.ndof)
    ref_U, ref_tr = U0.copy(), np.zeros((nsteps, 2, 2))
    ref_E = np.zeros(nsteps)
    e64 = Engine(mesh, k, record_energy=True)
    dt = e64.dt_cfl(0.3)
    for n in range(nsteps):
        ref_U = o.erk(ref_U, n * dt, dt, 1)
        ref_tr[n, 0, :1] = o.point_values(ref_U, *rx[0])[1][:1]
        ref_tr[n, 1, :2] = o.point_values(ref_U, *rx[1])[1][:2]
        ref_E[n] = o.energy(ref_U)
    for d, tol in (("f64", TOL64), ("f32", TOL32)):
        e = e64 if d == "f64" else Engine(mesh, k, dtype="f32", record_energy=True)
        e.set_sources(0, src, dirs, 10.0, 0.05, 1.0)
        e.set_receivers(rx, fld)
        e.set_state(U0)
        e.erk_step(0.0, dt, nsteps)
        eu, et, ee = rel(e.get_state(), ref_U), rel(e.traces(0), ref_tr), rel(e.energy_history(0), ref_E)
        say(d, "state", eu, "traces", et, "energy history", ee)
        assert eu < tol and et < tol and ee < tol
        e.close()
