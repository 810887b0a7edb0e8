"""CPU checks of the benchmark's bookkeeping (no GPU): the algorithmic and the moved byte counts
of one ERK(4) step and the unknown count on a mesh small enough to count by hand, and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def _two_squares():
    return dict(xy=np.array([[0, 0], [1, 0], [2, 0], [2, 1], [1, 1], [0, 1]], float).reshape(-1),
                cell_ptr=np.array([0, 4, 8], np.int32), cell_vtx=np.array([0, 1, 4, 5, 1, 2, 3, 4], np.int32),
                medium=np.array([0, 1], np.uint8))


def test_algorithmic_bytes_two_squares():
    """Two unit squares side by side, one fluid and one solid, k = 1 (N = 3, f = 2): 9 + 15 = 24
    cell unknowns; per step 17 words per unknown per shot; in each of the 4 stages one 4-byte face
    id per cell face (8) and the material scalars (3 fluid + 4 solid), two cell ids and one
    coefficient for each of the 7 faces, and a (3f)^2 block of state words for the one
    fluid-solid face."""
    b = _bench()
    mesh = _two_squares()
    assert b._faces(mesh) == (7, 1, 1)
    for word in (4, 8):
        for shots in (1, 3):
            got, ndof = b.algorithmic_bytes_per_step(mesh, 1, word, shots)
            assert ndof == 24
            assert got == word * 17 * 24 * shots + 4 * (4 * (8 + 3 + 4) + 12 * 7 + 36 * word)


def test_moved_bytes_two_squares():
    """The same mesh with the stage kernel's own traffic: 13 words per unknown per shot and per
    stage one 4-byte link per cell face (8), the material scalars the kernel loads (3 + 6) and
    one coefficient for the single interior face."""
    b = _bench()
    mesh = _two_squares()
    for word in (4, 8):
        for shots in (1, 3):
            got, ndof = b.moved_bytes_per_step(mesh, 1, word, shots)
            assert ndof == 24
            assert got == word * 13 * 24 * shots + 4 * (4 * (8 + 9) + 4 * 1)


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_paper_bilayer_workload():
    """The granite-water bilayer of the paper's timing table: 161 x 110 squares (6762 water, 10948
    granite), 225,078 cell unknowns at k = 1, the interface on a row line, and the step counts
    that reach T_f = 0.5 s at the paper's normalised steps (800 for k = 1, 2355 for k = 3)."""
    from synth import meshes as M
    b = _bench()
    m = M.granite_water()
    med = np.asarray(m["medium"])
    assert len(med) == 17710 and int(np.sum(med == 0)) == 6762 and int(np.sum(med == 1)) == 10948
    ys = m["xy"][m["cell_vtx"], 1].reshape(-1, 4)
    y_int = -1600.0 + 68 * 2600.0 / 110
    assert np.all(np.where(med == 0, ys.min(axis=1) >= y_int - 1e-9, ys.max(axis=1) <= y_int + 1e-9))
    U = M.pressure_pulse(m, 1)
    assert U.shape == (225078,) and np.all(U[np.cumsum(np.where(med == 0, 9, 15))[med == 1] - 15] == 0)
    for k, n in ((1, 800), (3, 2355)):
        dt = b.PAPER_BILAYER[k][0] * 23.6 / 6000.0
        assert int(np.ceil(0.5 / dt - 1e-9)) == n


def test_sdirk_bytes_per_step_counts():
    """The SDIRK step's byte model on made-up sizes: matrices once per stage, 8 + i cell-vector
    words for stage i, per iteration two products with S (8-byte values, shared column lists) and
    two with the float32 preconditioner."""
    import bench
    fp = dict(n_dof=100, n_face_dof=40, nnz=400, precond_nnz=160, cell_matrix_values=1000, n_slot=80,
              shared_cols=120)
    s, it = 3, 10
    stage = sum(8.0 * 1000 + 8.0 * (8 + i) * 100 + 20 * 80 + 8.0 * 40 + 8.0 * (12 + i) * 40 for i in range(s))
    smat = 8.0 * 400 + 4.0 * 120 + 24.0 * 40
    pmat = 4.0 * 160 + 24.0 * 40
    per_it = 2 * smat + 2 * pmat + 8.0 * 22 * 40
    assert bench.sdirk_bytes_per_step(fp, s, it) == stage + it * per_it + 8.0 * (s + 4) * 100


def test_sensor_differences():
    """Relative l2 differences between two runs' traces, the second interpolated at the first's
    times: zero for the same smooth signal sampled on two grids (up to interpolation error), and
    the relative size of a known perturbation."""
    import bench
    ta, tb = np.linspace(0.01, 1.0, 100), np.linspace(0.001, 1.0, 1000)
    sig = lambda t: np.stack([np.sin(3 * t), np.cos(2 * t)], axis=1)[:, None, :]
    a, b = sig(ta), sig(tb)
    d = bench.sensor_differences(ta, a, tb, b)
    assert len(d) == 1 and d[0] < 1e-4
    d2 = bench.sensor_differences(ta, 1.01 * a, tb, b)
    assert abs(d2[0] - 0.01) < 1e-4


def test_summary_line_is_compact_json():
    """The last stdout line parses as JSON, carries the contract's keys and stays a few kB even with
    every variant and extra workload filled in (the curves of the sweeps go to stderr)."""
    b = _bench()
    head = dict(value=2.6e11, ms_per_step=2.61, device_ms_per_step=2.55, cells=1720000, shot_dofs=167000000,
                gbs=4500.0, frac=0.5625, bytes_per_step=11.4e9)
    cpu = dict(value=2.2e8, unit="DOF-stage updates/s", cores=16, kind="oracle", single_core_value=1.6e7,
               sample="meshes 0-5 of the headline workload (k=1,2,3,...; 5300000 cell unknowns), one shot, "
                      "float64, 2 RK4 steps per run, median of 3 runs after 2 warm-up steps",
               cpu="AMD EPYC 9575F 64-Core Processor")
    variants = [dict(k=k, dtype=d, shots=s, us_per_step=49.87, frac=0.452)
                for k, d, s in ((2, "f32", 1), (2, "f64", 1), (3, "f32", 1), (3, "f64", 1), (2, "f32", 8), (3, "f32", 8))]
    extras = {"adjoint_f32_1shot": dict(ms=125.6, vs_forward=3.8), "adjoint_f64_1shot": dict(ms=128.5, vs_forward=2.7),
              "adjoint_f32_8shot": dict(ms=397.0, vs_forward=4.9), "basin_f32": dict(us_per_step=245.1, frac=0.58),
              "basin_f64": dict(us_per_step=570.2, frac=0.47),
              "paper_bilayer_k1": dict(erk4_s=0.0207, sdirk34_s=3.2, paper_erk4_cpu_s=161.0),
              "paper_bilayer_k3": dict(erk4_s=0.173, sdirk34_s=4.2, paper_erk4_cpu_s=3322.0)}
    for name in ("tets_k1_f32_1shot", "tets_k2_f32_1shot", "tets_k2_f64_1shot", "tets_k2_f32_4shot",
                 "hybrid_k2_f32_1shot", "moved_k1_f32_1shot"):
        extras["cube3d_" + name] = dict(us_per_step=1216.9, frac=0.364)
    line = b.summary_line(20, 5, head, [1e-7] * 16, 9.5, cpu, variants, extras, 5200.0, None)
    assert "\n" not in line and len(line) < 3000, len(line)
    d = json.loads(line)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["steps"] == 20 and d["warmup"] == 5 and d["n_gpus"] == 1
    assert d["roofline"]["frac"] == head["frac"] and d["roofline"]["bound"] == "hbm"
    assert "workload" in d["config"] and d["cpu_baseline"]["kind"] == "oracle"
    assert abs(d["speedup_vs_f64_single_shot"] - 9.5 / 2.61) < 1e-12


def test_faces3d_counts_match_the_host_plan():
    """bench.py's three-dimensional face count (algorithmic bytes) against the library's face links."""
    import numpy as np
    import bench
    from paper_2505_15771_amd.hho import Inspect
    from synth import meshes as M
    for mesh in (M.with_materials3d(M.unit_cube(4)), M.with_materials3d(M.unit_cube(3, tets=False)),
                 M.with_materials3d(M.unit_cube(4, kind="hybrid", seed=2))):
        ins = Inspect(mesh, 1)
        L = ins.link
        n_faces, n_interior, n_interface = bench._faces3d(mesh)
        assert n_faces == ins.n_faces
        assert n_interior == int(np.sum(L >= 0)) // 2
        assert n_interface == int(np.sum((L >= 0) & (((L >> 3) & 1) == 1))) // 2
