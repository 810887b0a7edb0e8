"""GPU tests of the stepping driver around the stage kernel: graph replay of the step loop,
launch-shape autotuning, the CFL time step, and batched multi-mesh / multi-shot stepping,
each against the FP64 oracle."""
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


def test_graph_replay_with_receivers_and_energy():
    """75 steps = two replays of the 32-step graph plus 11 direct steps, called twice in a row so the
    cached graph is reused with a new start time; state, receiver traces and energies vs the oracle."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    say("case: graph replay 2 x 75 steps k=2")
    mesh = M.with_materials(M.unit_square(8, p_split=0.5, seed=21), perturb=0.1, seed=22)
    o = Oracle(mesh, 2)
    o.set_point_sources([[0.45, 0.3]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
    rx = np.array([[0.3, 0.8], [0.6, 0.2]])
    fld = np.array([0, 1], np.int32)
    e = Engine(mesh, 2, record_energy=True)
    e.set_sources(0, [[0.45, 0.3]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
    e.set_receivers(rx, fld)
    U = 0.05 * np.random.default_rng(4).standard_normal(o.ndof)
    e.set_state(U)
    dt = 0.4 * 0.138 / 8 / math.sqrt(3.0)
    t = 0.0
    for call in range(2):
        tr = np.zeros((75, 2, 2))
        En = np.zeros(75)
        for n in range(75):
            U = o.erk(U, t + n * dt, dt, 1)
            En[n] = o.energy(U)
            for r in range(2):
                c, vals = o.point_values(U, *rx[r])
                tr[n, r, :1 + fld[r]] = vals[:1 + fld[r]]
        e.erk_step(t, dt, 75)
        t += 75 * dt
        eu, et, ee = rel(e.get_state(), U), rel(e.traces(), tr), rel(e.energy_history(), En)
        say("call", call, "state", eu, "traces", et, "energy", ee)
        assert eu < 1e-12 and et < 1e-12 and ee < 1e-12


def test_autotune_keeps_results():
    """The autotuner picks a launch shape; stepping in any shape gives the same float64 state."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    say("case: autotune k=3 f64")
    mesh = M.with_materials(M.unit_square(20, p_split=0.5, seed=23), perturb=0.1, seed=24)
    o = Oracle(mesh, 3)
    U0 = np.random.default_rng(5).standard_normal(o.ndof)
    ref = o.erk(U0, 0.0, 1e-4, 40)
    outs = []
    for lanes in (64, 128, 256, None):
        e = Engine(mesh, 3)
        if lanes is None:
            got = e.autotune()
            say("autotune chose", got, "lanes")
            assert got in (64, 128, 256)
        else:
            e.set_launch(lanes)
        e.set_state(U0)
        e.erk_step(0.0, 1e-4, 40)
        outs.append(e.get_state())
        assert rel(outs[-1], ref) < 1e-12
    for u in outs[1:]:
        assert np.array_equal(u, outs[0])


def test_dt_cfl_matches_table():
    """hho_dt_cfl on a hybrid mesh of squares and half-square triangles (side h = 1/16, c_max =
    sqrt(3)): per shape the smaller of the paper's Table tab::ratio_geo value and 0.9 times this
    discretisation's measured limit (ERK(4), k = 1, tau^s on c_S: squares min(0.282, 0.9 x 0.3959),
    triangles min(0.265, 0.9 x 0.2410)), the triangles deciding; with tau^s on c_P the squares'
    0.9 x 0.2329 and the triangles' 0.9 x 0.1358.  Squares with hanging nodes (five vertices, four
    corners) take the square value: on a mesh of squares only, refining some of them (children of
    side h / 2 and their hanging-node neighbours) gives the children's step."""
    from paper_2505_15771_amd import Engine
    mesh = M.with_materials(M.unit_square(16, p_split=0.5, seed=25))
    for k, s, ss, cfl in ((1, 4, 1, 0.9 * 0.2410), (2, 4, 1, 0.9 * 0.1352), (3, 3, 1, 0.9 * 0.0792),
                          (1, 4, 0, 0.9 * 0.1358)):
        e = Engine(mesh, k, rk_stages=s, stab_speed=ss)
        assert abs(e.dt_cfl(0.5) - 0.5 * cfl / 16 / math.sqrt(3.0)) < 1e-15, (k, s, ss)
    refine = np.zeros((8, 8), bool)
    refine[2:4, 3:6] = True
    quads = M.with_materials(M.unit_square(8, refine=refine))
    assert abs(Engine(quads, 1).dt_cfl(1.0) - 0.282 / 16 / math.sqrt(3.0)) < 1e-15


def test_batch_of_meshes_and_shots():
    """Four meshes of different sizes and degrees (k = 1, 2, 3), float32 and float64, several shots
    each (the last with vertices moved on one half, so its stages are two launches), advanced by one
    batch (graph branches per mesh) for 70 steps; every shot vs the oracle."""
    from oracle import Oracle
    from paper_2505_15771_amd import Batch, Engine
    say("case: batch of 4 meshes")
    specs = [(6, 1, "f64", 2), (9, 2, "f32", 3), (5, 3, "f64", 1), (16, 2, "f64", 2)]
    engines, refs, dts = [], [], []
    for i, (n, k, dtype, S) in enumerate(specs):
        if i < 3:
            mesh = M.with_materials(M.unit_square(n, p_split=0.5, seed=30 + i), perturb=0.1, seed=40 + i)
        else:  # vertices moved left of x = 1/2: pooled groups beside shared-table groups
            mesh = M.with_materials(M.perturbed_square(n, seed=33, x_max=0.5), perturb=0.1, seed=43)
        e = Engine(mesh, k, dtype=dtype, n_shots=S)
        dt = e.dt_cfl(0.5)
        dts.append(dt)
        shots = []
        for sh in range(S):
            o = Oracle(mesh, k)
            xs = [[0.2 + 0.3 * sh, 0.3]]
            o.set_point_sources(xs, [[0.0, 1.0]], 10.0, 0.12, 1.0)
            e.set_sources(sh, xs, [[0.0, 1.0]], 10.0, 0.12, 1.0)
            U0 = 0.01 * np.random.default_rng(50 + 10 * i + sh).standard_normal(o.ndof)
            e.set_state(U0, shot=sh)
            shots.append(o.erk(U0, 0.1, dt, 70))
        engines.append(e)
        refs.append(shots)
    b = Batch(engines)
    b.erk_step([0.1] * len(specs), dts, 70)
    for i, e in enumerate(engines):
        tol = 1e-12 if specs[i][2] == "f64" else 1e-5
        for sh, ref in enumerate(refs[i]):
            err = rel(e.get_state(sh), ref)
            say("mesh", i, "shot", sh, err)
            assert err < tol
    b.close()


def test_full_size_batch_sampled():
    """The 16-mesh batch in the launch configuration the benchmark times (hybrid meshes of 20k-300k
    cells, k = 1, 2, 3 in turn, 4 Ricker shots each, float32 with the energy check, one batch):
    after 5 steps, sampled meshes and shots (the smallest, a middle one and the largest mesh) are
    compared with the oracle on the whole mesh."""
    from oracle import Oracle
    from paper_2505_15771_amd import Batch, Engine
    say("case: full-size 16-mesh batch, sampled vs oracle")
    specs = M.batch_meshes()
    engines, dts, meshes = [], [], []
    for i, d in enumerate(specs):
        mesh = M.with_materials(M.unit_square(d["n"], p_split=0.5, seed=d["seed"]))
        e = Engine(mesh, d["k"], dtype="f32", n_shots=4, record_energy=True)
        pos = M.shot_positions(4, 4100 + i)
        for sh in range(4):
            e.set_sources(sh, [pos[sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
            e.set_state(0.01 * np.random.default_rng(7000 + 4 * i + sh).standard_normal(e.n_dof), shot=sh)
        dts.append(e.dt_cfl(0.5))
        e.autotune()  # as the benchmark does before timing
        engines.append(e)
        meshes.append(mesh)
    b = Batch(engines)
    b.erk_step([0.1] * len(engines), dts, 5)
    for i, sh in ((0, 0), (7, 2), (15, 3)):
        o = Oracle(meshes[i], specs[i]["k"])
        pos = M.shot_positions(4, 4100 + i)
        o.set_point_sources([pos[sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
        U0 = 0.01 * np.random.default_rng(7000 + 4 * i + sh).standard_normal(o.ndof)
        ref = o.erk(U0, 0.1, dts[i], 5)
        err = rel(engines[i].get_state(sh), ref)
        say("mesh", i, "k", specs[i]["k"], "cells", engines[i].n_cells, "shot", sh, "rel L2", err)
        assert err < 1e-5
    b.close()
    for e in engines:
        e.close()


@pytest.mark.parametrize("lanes", [60, 125, 255])
def test_five_shots_every_launch_shape(lanes):
    """Five shots (lanes per workgroup 60, 125 or 255: cells of a workgroup 12, 25 or 51, so the
    last workgroup of every group is ragged) on a hanging-node hybrid mesh, k = 2, float64, with
    different initial states per shot; every shot against the oracle."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine
    say("case: 5 shots, %d lanes per workgroup" % lanes)
    mesh = M.hanging_square(9, seed=13)
    o = Oracle(mesh, 2)
    e = Engine(mesh, 2, n_shots=5)
    e.set_launch(lanes)
    dt = e.dt_cfl(0.5)
    refs = []
    for sh in range(5):
        U0 = np.random.default_rng(900 + sh).standard_normal(o.ndof)
        e.set_state(U0, shot=sh)
        refs.append(o.erk(U0, 0.0, dt, 9))
    e.erk_step(0.0, dt, 9)
    for sh in range(5):
        err = rel(e.get_state(sh), refs[sh])
        say("shot", sh, err)
        assert err < 1e-12


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_every_tuning_combination(dtype, tol, k):
    """Every launch shape with both store policies gives the oracle's state and energy (k = 3 in
    float32 keeps D_{i-1} in LDS sized by the workgroup, k = 2 in float64 combines in chunks);
    hho_get_tuning reports what hho_set_tuning set, and unknown flag bits are rejected."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine, HHOError
    mesh = M.with_materials(M.unit_square(30, p_split=0.5, seed=31), perturb=0.1, seed=32)
    o = Oracle(mesh, k)
    U0 = np.random.default_rng(950).standard_normal(o.ndof)
    e = Engine(mesh, k, dtype=dtype, record_energy=True)
    dt = e.dt_cfl(0.5)
    ref = o.erk(U0, 0.0, dt, 6)
    E_ref = o.energy(ref)
    with pytest.raises(HHOError):
        e.set_tuning(64, 2)
    for lanes in (64, 128, 256):
        for flags in range(2):
            say("case: k=%d %s, %d lanes, flags %d" % (k, dtype, lanes, flags))
            e.set_tuning(lanes, flags)
            assert e.tuning() == (lanes, flags)
            e.set_state(U0)
            e.erk_step(0.0, dt, 6)
            err = rel(e.get_state(), ref)
            dE = abs(e.energy()[0] - E_ref) / E_ref
            say("  rel L2", err, "energy", dE)
            assert err < tol
            assert dE < (1e-12 if dtype == "f64" else 1e-5)
    e.close()


def test_reserve_steps_changes_no_result():
    """hho_reserve_steps sizes the receiver and energy histories ahead of a call: a 70-step call
    after a 5-step one (graphs captured before and after the reservation) gives the state, the
    receiver traces and the energy history of an unreserved run, and of the oracle; a negative
    count is rejected."""
    from oracle import Oracle
    from paper_2505_15771_amd import Engine, HHOError
    say("case: reserve_steps, k=2 f64, 5 + 70 steps")
    mesh = M.with_materials(M.unit_square(16, p_split=0.5, seed=41), perturb=0.1, seed=42)
    o = Oracle(mesh, 2)
    U0 = np.random.default_rng(43).standard_normal(o.ndof)
    outs = []
    for reserve in (0, 70):
        e = Engine(mesh, 2, dtype="f64", record_energy=True)
        e.set_receivers([[0.3, 0.75], [0.6, 0.3]], [0, 1])
        e.set_state(U0)
        dt = e.dt_cfl(0.5)
        if reserve:
            e.reserve_steps(reserve)
            with pytest.raises(HHOError):
                e.reserve_steps(-1)
        e.erk_step(0.0, dt, 5)
        e.erk_step(5 * dt, dt, 70)
        outs.append((e.get_state(), e.traces(), e.energy_history()))
        e.close()
    ref = o.erk(U0, 0.0, dt, 75)
    for U, tr, eh in outs:
        assert rel(U, ref) < 1e-12
        assert eh.shape[0] == 70 and np.all(np.isfinite(eh))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.allclose(outs[0][2], outs[1][2], rtol=1e-13, atol=0.0)
