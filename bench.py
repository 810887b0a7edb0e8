"""Benchmark of the HHO elasto-acoustic explicit Runge-Kutta path on one MI355X.

Headline workload: sixteen seeded hybrid meshes of the two-material unit square (elastic below
y = 1/2: rho = 1, cP = sqrt(3), cS = 1; acoustic above: rho = 1, c = 1), target cell counts
log-spaced from 2e4 to 3e5 (1.72 M cells in total), HHO degree k = 1, 2, 3 in turn, four Ricker
shots per mesh at seeded positions, float32 stepping with the float64 energy of every shot
recorded after every step, all meshes advanced together by one batch of captured graphs.  A step
is one classical RK4 step (four fused stage launches per mesh) of every mesh and shot; inputs are
resident in HBM before timing starts.

Reported next to it: the same workload stepped one shot at a time in float64 (the speed-up of the
batched float32 path over it), the error of the batched float32 path against the float64 oracle,
the oracle's own throughput on the host cores, and the 256 x 256 hybrid mesh stepped in float32 /
float64, one or eight shots, k = 2 and 3.  The last stdout line is one compact JSON object; the
other workloads print one JSON line each to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import meshes as M  # noqa: E402

HBM_PEAK_GBS = 8000.0

# The stage kernel's sources and the host plan that lays out its data: a measured HBM traffic figure
# is reported only while their digest matches the one it was measured with.
STAGE_SOURCES = ("kernels.hip", "stage_common.h", "device.h", "plan.cpp")


def stage_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_15771_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()
CFL_SQUARE = {1: 0.282, 2: 0.138, 3: 0.087}   # Table tab::ratio_ERK, s = 4
CFL_TRI = {1: 0.265, 2: 0.147, 3: 0.100}      # Table tab::ratio_geo, s = 4
METRIC = "HHO DOF-stage updates/s, FP64 vs FP32/batched, % of HBM roofline"


def _faces(mesh):
    """(number of faces, number of fluid-solid interface faces) of a polygon mesh: every edge
    of a cell is a face, shared by the two cells that list it."""
    vtx, ptr = np.asarray(mesh["cell_vtx"]), np.asarray(mesh["cell_ptr"])
    med = np.asarray(mesh["medium"])
    b = np.empty_like(vtx)
    owner = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    for c in range(len(ptr) - 1):
        s, e = ptr[c], ptr[c + 1]
        b[s:e] = np.roll(vtx[s:e], -1)
    keys = np.minimum(vtx, b).astype(np.int64) * (1 << 32) + np.maximum(vtx, b)
    order = np.argsort(keys, kind="stable")
    ks, ms = keys[order], med[owner[order]]
    pair = np.flatnonzero(ks[1:] == ks[:-1])
    n_faces = len(ks) - len(pair)
    n_interface = int(np.sum(ms[pair] != ms[pair + 1]))
    return n_faces, len(pair), n_interface


def algorithmic_bytes_per_step(mesh, k, word, shots):
    """Algorithmic HBM bytes of one RK4 step, the fixed amount of work that the roofline
    fraction is priced on: 17 state words per cell unknown per shot (the accumulator form of
    RK4: stage i reads U^n and the accumulator and writes the next stage state and the
    accumulator; the last stage also writes U^{n+1}), plus per stage the mesh metadata of a
    face-based layout in 4-byte words: per cell one face id per face and its material scalars (3
    fluid: 1/rho, kappa, tau; 4 solid: 1/rho, lambda, mu, tau), per face its two cell ids and one
    inverse coefficient, and per fluid-solid interface face a (3f x 3f) block in the state word.
    Returns (bytes, cell unknowns of one shot)."""
    N = (k + 1) * (k + 2) // 2
    f = k + 1
    med = np.asarray(mesh["medium"])
    nf = np.diff(mesh["cell_ptr"])
    ndof = int(np.sum(np.where(med == 0, 3, 5))) * N
    n_faces, _, n_interface = _faces(mesh)
    meta = int(np.sum(4 * nf + 4 * np.where(med == 0, 3, 4))) + 12 * n_faces + (3 * f) ** 2 * word * n_interface
    return word * 17 * ndof * shots + 4 * meta, ndof


def moved_bytes_per_step(mesh, k, word, shots):
    """Least HBM traffic of one RK4 step of this implementation's stage kernel: 13 state words
    per cell unknown per shot (stage 1 reads U^n and writes D_1; stage 2 reads D_1 and U^n and
    writes D_2 and the partial sum Q; stage 3 reads D_2 and U^n and writes D_3; stage 4 reads D_3,
    U^n and Q and writes U^{n+1}), plus per stage the per-cell metadata in 4-byte words: one face
    link per face, the material scalars the kernel loads (3 fluid: tau, kappa, 1/rho; 6 solid: tau,
    1/tau, 1/rho, lambda + 2 mu, lambda, 2 mu) and one coefficient per interior face.
    The face-trace exchange between neighbouring cells is not counted."""
    N = (k + 1) * (k + 2) // 2
    med = np.asarray(mesh["medium"])
    nf = np.diff(mesh["cell_ptr"])
    ndof = int(np.sum(np.where(med == 0, 3, 5))) * N
    meta_cells = int(np.sum(4 * nf + 4 * np.where(med == 0, 3, 6)))
    _, n_interior, _ = _faces(mesh)
    return word * 13 * ndof * shots + 4 * (meta_cells + 4 * n_interior), ndof


def _faces3d(mesh):
    """(faces, interior faces, fluid-solid interface faces) of a tetrahedron / prism / hexahedron
    mesh: a face is the vertex set of a cell's local face, shared by the cells that list it."""
    local = {4: [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)],
             6: [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
             8: [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]}
    ptr, vtx, med = np.asarray(mesh["cell_ptr"]), np.asarray(mesh["cell_vtx"]), np.asarray(mesh["medium"])
    keys, owner = [], []
    for nv, faces in local.items():
        cells = np.flatnonzero(np.diff(ptr) == nv)
        if len(cells) == 0:
            continue
        cv = vtx[ptr[cells][:, None] + np.arange(nv)[None, :]]
        for f in faces:
            kk = np.sort(cv[:, list(f)], axis=1)          # sorted vertex ids; triangles get a fourth id -1
            if len(f) == 3:
                kk = np.concatenate([kk, -np.ones((len(cells), 1), kk.dtype)], axis=1)
            keys.append(kk)
            owner.append(cells)
    keys, owner = np.concatenate(keys).astype(np.int64), np.concatenate(owner)
    order = np.lexsort(keys.T[::-1])
    ks = keys[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    pair = np.flatnonzero(same)
    n_interface = int(np.sum(med[owner[order[pair]]] != med[owner[order[pair + 1]]]))
    return len(keys) - len(pair), len(pair), n_interface


def algorithmic_bytes_per_step3d(mesh, k, word, shots):
    """The three-dimensional counterpart of algorithmic_bytes_per_step: 17 state words per cell
    unknown per shot, plus per stage one face id per cell face, the material scalars (3 fluid, 4
    solid), two cell ids and one coefficient per face, and a (4f x 4f) block per interface face
    (f = (k+1)(k+2)/2: p_F and the three components of v_F).  Returns (bytes, cell unknowns)."""
    N = (k + 1) * (k + 2) * (k + 3) // 6
    f = (k + 1) * (k + 2) // 2
    med = np.asarray(mesh["medium"])
    nv = np.diff(mesh["cell_ptr"])
    nf = np.where(nv == 4, 4, np.where(nv == 6, 5, 6))
    ndof = int(np.sum(np.where(med == 0, 4, 9))) * N
    n_faces, _, n_interface = _faces3d(mesh)
    meta = int(np.sum(4 * nf + 4 * np.where(med == 0, 3, 4))) + 12 * n_faces + (4 * f) ** 2 * word * n_interface
    return word * 17 * ndof * shots + 4 * meta, ndof


def run_3d(n, k, dtype, shots, steps, warmup, kind="tets"):
    """Two-material unit cube of n^3 cubes (each cut into six tetrahedra; or columns of hexahedra
    and triangular prisms, kind "hybrid"), solid below z = 1/2, materials perturbed by U[-10 %, 10 %]
    per cell, random states, RK4 from captured graphs; DOF-stage updates/s and the algorithmic bytes
    against the HBM peak."""
    import torch
    from paper_2505_15771_amd import Engine
    if kind == "moved":  # every interior vertex off the interface moved: every cell its own shape
        mesh = M.with_materials3d(M.unit_cube(n, jitter=0.1, seed=7000), perturb=0.1, seed=7001)
    else:
        mesh = M.with_materials3d(M.unit_cube(n, kind=kind, seed=7000), perturb=0.1, seed=7001)
    e = Engine(mesh, k, dtype=dtype, n_shots=shots)
    for sh in range(shots):
        e.set_state(M.random_state(e.n_dof, 7100 + sh), shot=sh)
    e.autotune()
    dt = (0.1 if k == 1 else 0.05) / n / M.max_wave_speed3d(mesh) * (0.6 if kind == "moved" else 1.0)
    e.reserve_steps(max(steps, warmup))  # histories sized before the graphs are captured
    e.erk_step(0.0, dt, warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    ev0.record(st)
    e.erk_step(warmup * dt, dt, steps)
    ev1.record(st)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    word = 8 if dtype == "f64" else 4
    bstep, ndof = algorithmic_bytes_per_step3d(mesh, k, word, shots)
    what = {"tets": "tetrahedra", "hybrid": "columns of hexahedra and prisms",
            "moved": "tetrahedra with moved vertices (pooled tables)"}[kind]
    out = dict(workload="unit cube %d^3 %s, two materials" % (n, what),
               cells=int(len(mesh["medium"])), k=k, dtype=dtype, shots=shots, steps=steps,
               ms_per_step=ms / steps, launch_us=ms / steps / 4 * 1e3,
               value=ndof * shots * 4 * steps / (ms * 1e-3), bytes_per_step=bstep,
               gbs=bstep * steps / (ms * 1e-3) / 1e9, tuning=e.tuning()[0],
               finite=bool(np.all(np.isfinite(e.get_state()))))
    out["frac"] = out["gbs"] / HBM_PEAK_GBS
    e.close()
    return out


def run_variant(mesh, k, dtype, shots, steps, warmup):
    import torch
    from paper_2505_15771_amd import Engine
    eng = Engine(mesh, k, dtype=dtype, n_shots=shots)
    rng = np.random.default_rng(7)
    for sh in range(shots):
        eng.set_state(1e-3 * rng.standard_normal(eng.n_dof), shot=sh)
        eng.set_sources(sh, [[0.5, 0.25 + 0.01 * sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
    eng.autotune()  # launch shape and store cache policy (outside the timed region)
    h = 1.0 / 256
    dt = 0.5 * min(CFL_SQUARE[k], CFL_TRI[k]) * h / M.max_wave_speed(mesh)
    eng.reserve_steps(max(steps, warmup))  # histories sized before the graphs are captured
    eng.erk_step(0.0, dt, warmup)
    eng.synchronize()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    eng.erk_step(warmup * dt, dt, steps)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    torch.cuda.synchronize()
    word = 8 if dtype == "f64" else 4
    bstep, ndof = algorithmic_bytes_per_step(mesh, k, word, shots)
    mstep, _ = moved_bytes_per_step(mesh, k, word, shots)
    secs = ms / 1e3
    updates = ndof * shots * 4 * steps
    launch_us = ms * 1e3 / (4 * steps)
    gbs = (bstep / 4) / (launch_us * 1e-6) / 1e9
    moved_gbs = (mstep / 4) / (launch_us * 1e-6) / 1e9
    E = eng.energy()
    lanes, flags = eng.tuning()
    eng.close()
    return dict(k=k, dtype=dtype, shots=shots, steps=steps, ms=ms, ms_per_step=ms / steps,
                value=updates / secs, launch_us=launch_us, bytes_per_launch=bstep / 4, gbs=gbs,
                frac=gbs / HBM_PEAK_GBS, moved_bytes_per_launch=mstep / 4, moved_gbs=moved_gbs,
                finite=bool(np.all(np.isfinite(E))), ndof=ndof,
                tuning=dict(lanes=lanes, nt_stores=bool(flags & 1)))


def run_adjoint(k, dtype, steps=1000, ckpt=50, shots=1):
    """The adjoint workload: 128 x 128 hybrid mesh (seed 5001), k = 2, one Ricker source per shot
    (the first at (0.5, 0.25), the others at seeded positions in the solid), 32 receivers;
    misfit gradient (summed over the shots) by hho_adjoint_step over `steps` steps with
    checkpoints every `ckpt`, against the same number of forward steps."""
    import torch
    from paper_2505_15771_amd import Engine
    mesh = M.adjoint_square(128)
    rec_xy, rec_f = M.adjoint_receivers()
    eng = Engine(mesh, k, dtype=dtype, n_shots=shots)
    pos = np.concatenate([[[0.5, 0.25]], M.shot_positions(max(shots - 1, 0), 5100)])[:shots]
    for sh in range(shots):
        eng.set_sources(sh, [pos[sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
    eng.set_receivers(rec_xy, rec_f)
    dt = eng.dt_cfl(0.5)
    d_obs = np.zeros((shots, steps, len(rec_f), 2))
    zero = np.zeros(eng.n_dof)
    eng.adjoint(0.0, dt, steps, d_obs, ckpt)  # warm-up: workspace allocation and the segment graphs
    for sh in range(shots):
        eng.set_state(zero, shot=sh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, _ = eng.adjoint(0.0, dt, steps, d_obs, ckpt)
    t_adj = time.perf_counter() - t0
    for sh in range(shots):
        eng.set_state(zero, shot=sh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.erk_step(0.0, dt, steps)
    eng.synchronize()
    t_fwd = time.perf_counter() - t0
    cells = int(len(mesh["cell_ptr"]) - 1)
    eng.close()
    return dict(workload="adjoint 128x128 hybrid, k=%d, %d steps, checkpoints every %d, %d shot%s"
                         % (k, steps, ckpt, shots, "s" if shots > 1 else ""),
                dtype=dtype, cells=cells, shots=shots, adjoint_ms=t_adj * 1e3, forward_ms=t_fwd * 1e3,
                adjoint_ms_per_shot=t_adj * 1e3 / shots, ratio=t_adj / t_fwd, finite=bool(np.isfinite(J)))


def run_basin(dtype, steps=100, warmup=5):
    """The synthetic basin (20 km x 5 km, water over a layered half-space with a Gaussian basin,
    2:1 refinement with hanging nodes, ~543k cells), k = 2, ERK(4), Ricker f0 = 2 Hz 1 km below
    the seafloor, 64 receivers of v just below the seafloor."""
    import torch
    from paper_2505_15771_amd import Engine
    mesh = M.basin()
    eng = Engine(mesh, 2, dtype=dtype)
    eng.set_sources(0, [[8000.0, -1000.0]], [[0.0, 1.0]], 2.0, 0.6, 1.0e9)
    h0 = 20000.0 / 1120
    eng.set_receivers(np.stack([np.linspace(1000.0, 19000.0, 64), np.full(64, -0.25 * h0)], axis=1),
                      np.ones(64, np.int32))
    dt = eng.dt_cfl(0.5)
    eng.autotune()
    eng.reserve_steps(max(steps, warmup))  # histories sized before the graphs are captured
    eng.erk_step(0.0, dt, warmup)
    eng.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    eng.erk_step(warmup * dt, dt, steps)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    tr = eng.traces(0)
    bstep, _ = algorithmic_bytes_per_step(mesh, 2, 8 if dtype == "f64" else 4, 1)
    gbs = bstep * steps / (ms / 1e3) / 1e9
    out = dict(workload="basin 543k cells (hanging nodes), k=2, 64 receivers", dtype=dtype, steps=steps,
               cells=int(len(mesh["cell_ptr"]) - 1), dofs=int(eng.n_dof), ms_per_step=ms / steps,
               value=eng.n_dof * 4 * steps / (ms / 1e3), gbs=gbs, frac=gbs / HBM_PEAK_GBS,
               finite=bool(np.all(np.isfinite(tr))))
    eng.close()
    return out


def run_tableaux(k=2, dtype="f32", steps=200):
    """The headline workload stepped with ERK(2), ERK(3) and ERK(4) of eq. ERK: time per step and
    DOF-stage updates/s (a stage is one fused launch in every tableau; the combine moves 5, 9 and
    13 state words per unknown per step)."""
    import torch
    from paper_2505_15771_amd import Engine
    mesh = M.hybrid_square(256)
    out = []
    for s_ in (2, 3, 4):
        e = Engine(mesh, k, rk_stages=s_, dtype=dtype)
        e.set_state(1e-3 * np.random.default_rng(7).standard_normal(e.n_dof))
        e.autotune()
        dt = e.dt_cfl(0.5)
        e.erk_step(0.0, dt, 20)
        e.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        e.erk_step(0.0, dt, steps)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        out.append(dict(stages=s_, us_per_step=ms * 1e3 / steps, us_per_stage=ms * 1e3 / (steps * s_),
                        value=e.n_dof * s_ * steps / (ms / 1e3)))
        e.close()
    return dict(workload="ERK(2/3/4) tableaux, 256x256 hybrid mesh, k=%d, %s, one shot" % (k, dtype), results=out)


def run_perturbed(k=2, dtype="f32", steps=200, n=256):
    """Meshes whose cells do not share shapes: the n x n hybrid mesh as generated, with every
    vertex moved at random (every cell its own shape class, all pooled), and with the vertices
    left of x = 1/2 moved (pooled groups beside shared-table groups); ERK(4) time per step and
    DOF-stage updates/s of each, one shot."""
    import torch
    from paper_2505_15771_amd import Engine, Inspect
    meshes = (("lattice shapes", M.with_materials(M.unit_square(n, p_split=0.5, seed=3))),
              ("all vertices moved", M.with_materials(M.perturbed_square(n, seed=3))),
              ("vertices left of x = 1/2 moved", M.with_materials(M.perturbed_square(n, seed=3, x_max=0.5))))
    out = []
    for name, mesh in meshes:
        ins = Inspect(mesh, k)
        pooled_cells = int(ins.groups[ins.pooled == 1, 4].sum())
        t0 = time.perf_counter()
        e = Engine(mesh, k, dtype=dtype)
        setup = time.perf_counter() - t0
        e.set_state(1e-3 * np.random.default_rng(7).standard_normal(e.n_dof))
        e.autotune()
        dt = 0.3 * e.dt_cfl(1.0)
        e.reserve_steps(max(steps, 20))
        e.erk_step(0.0, dt, 20)
        e.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        e.erk_step(0.0, dt, steps)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        out.append(dict(mesh=name, cells=e.n_cells, groups=int(ins.n_groups), pooled_cells=pooled_cells,
                        setup_s=setup, us_per_step=ms * 1e3 / steps, value=e.n_dof * 4 * steps / (ms / 1e3)))
        e.close()
    return dict(workload="%dx%d hybrid mesh with moved vertices, k=%d, %s, ERK(4), one shot" % (n, n, k, dtype),
                unit="DOF-stage updates/s", results=out)


def run_precision(k=2, steps=2000):
    """Float32 error of the paper-sized run: the 256 x 256 hybrid workload (Ricker source, eight
    pressure receivers at y = 0.75), `steps` steps at half the CFL step, stepped in float32 and in
    float64 on the GPU (the float64 path equals the float64 oracle to ~1e-13, see the parity
    tests); relative L2 error of the float32 state and receiver traces every 500 steps."""
    from paper_2505_15771_amd import Engine
    mesh = M.hybrid_square(256)
    src, dirs = [[0.5, 0.25]], [[0.0, 1.0]]
    rx = M.receiver_line(8, 0.75)
    engines = {}
    for dt_ in ("f64", "f32"):
        e = Engine(mesh, k, dtype=dt_)
        e.set_sources(0, src, dirs, 10.0, 0.12, 1.0)
        e.set_receivers(rx, np.zeros(8, np.int32))
        e.set_state(1e-3 * np.random.default_rng(2003).standard_normal(e.n_dof))
        engines[dt_] = e
    dt = engines["f64"].dt_cfl(0.5)
    out = []
    t = 0.0
    for block in range(steps // 500):
        tr = {}
        for dt_, e in engines.items():
            e.erk_step(t, dt, 500)
            tr[dt_] = e.traces()
        t += 500 * dt
        a, b_ = engines["f32"].get_state(), engines["f64"].get_state()
        out.append(dict(steps=500 * (block + 1), state=float(np.linalg.norm(a - b_) / np.linalg.norm(b_)),
                        traces=float(np.linalg.norm(tr["f32"] - tr["f64"]) / np.linalg.norm(tr["f64"]))))
    for e in engines.values():
        e.close()
    return dict(workload="float32 vs float64 error, 256x256 hybrid mesh, k=%d, Ricker source, %d steps" % (k, steps),
                errors=out)


PAPER_BILAYER = {1: (0.159, 161.0), 3: (0.054, 3322.0)}  # Table tab::cfl_cpu: ERK(4) dt~, CPU s
# the initial pressure pulse of the timing case (Sec. 5.2, eq. ricker_ic): centre (0, 200 m),
# lambda = c_P^f / f_c = 1500 / 10 m
PULSE_CENTER, PULSE_LAMBDA = (0.0, 200.0), 150.0
# the sensors of the timing case (Sec. 5.2): S^f records p, S^s and S^i record v (S^i at y = 0 lies
# in the granite, 7.3 m below this mesh's interface)
BILAYER_SENSORS = ([[-500.0, 200.0], [-1000.0, -500.0], [-400.0, 0.0]], [0, 1, 1])


def run_paper_bilayer(k, dtype="f64", sensors=False):
    """The paper's timed ERK(4) run (Sec. 5.2, Table tab::cfl_cpu): granite-water bilayer,
    161 x 110 squares of 23.6 m, the pressure pulse of eq. ricker_ic in the water (projected by
    the library), T_f = 0.5 s at the paper's
    normalised step dt~ = cP dt / h (0.159 for k = 1, 0.054 for k = 3).  Reports the time of
    the whole run on the GPU (state resident, graph captured by a warm-up call) and the setup
    time (plan, upload, autotuning), beside the paper's CPU seconds (hardware not stated)."""
    import torch
    from paper_2505_15771_amd import Engine
    mesh = M.granite_water()
    dtt, paper_s = PAPER_BILAYER[k]
    dt = dtt * 23.6 / 6000.0
    n = int(np.ceil(0.5 / dt - 1e-9))
    t0 = time.perf_counter()
    eng = Engine(mesh, k, dtype=dtype, record_energy=True)
    if sensors:
        eng.set_receivers(*BILAYER_SENSORS)
    eng.set_ricker_ic(PULSE_CENTER, PULSE_LAMBDA, theta=1.0, field=0)
    U0 = eng.get_state()
    eng.autotune()
    eng.synchronize()
    setup_s = time.perf_counter() - t0
    eng.erk_step(0.0, dt, 64)  # warm-up: graph capture
    eng.set_state(U0)
    E_init = float(eng.energy()[0])
    eng.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    eng.erk_step(0.0, dt, n)
    e1.record(st)
    e1.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    E = eng.energy_history()
    out = dict(workload="paper granite-water bilayer (Table tab::cfl_cpu), 17710 squares, k=%d, ERK(4), "
                        "T_f = 0.5 s" % k, dtype=dtype, k=k, steps=n, dt=dt, cell_dofs=int(eng.n_dof),
               run_s=secs, setup_s=setup_s, value=eng.n_dof * 4 * n / secs,
               paper_cpu_s=paper_s, paper_hardware="not stated", speedup_vs_paper=paper_s / secs,
               energy_ratio=float(E[-1] / E_init), finite=bool(np.all(np.isfinite(E))))
    if sensors:
        out["_traces"] = (dt * np.arange(1, n + 1), eng.traces())
    eng.close()
    return out


SDIRK_BILAYER = {"dtt": 0.398, "paper_cpu_s": {"direct": {1: 207.0, 3: 1095.0}, "iterative": {1: 281.0, 3: 1352.0}}}


def sdirk_bytes_per_step(fp, stages, iterations):
    """Algorithmic bytes of one SDIRK(s, s+1) step of the engine (float64): per stage the
    per-cell matrices once ([A^{-1}; V] and W), the cell vectors of the stage (U^n, the earlier
    Y_j, B, g, U, Y_i: 8 + i words per unknown over the stage, i earlier stages), the face-slot
    products and their indices, and the face vectors outside the iterations (about 12 words per
    face unknown); per BiCGStab iteration two products with the face matrix and two with the
    face-block preconditioner (8-byte value + 4-byte column per nonzero, row pointers, source and
    result vectors) and 22 face-vector words of the updates and dot products; the final combine
    (s + 4 words per cell unknown).  The face matrix moves 8 bytes per nonzero, its shared column
    lists 4 bytes per stored index and 8 bytes of row offsets per row; the preconditioner 4 bytes
    per nonzero and 8 per row."""
    nd, nf = fp["n_dof"], fp["n_face_dof"]
    stage = 0.0
    for i in range(stages):
        stage += 8.0 * fp["cell_matrix_values"] + 8.0 * (8 + i) * nd
        stage += (2 * 8 + 4) * fp["n_slot"] + 8.0 * nf + 8.0 * (12 + i) * nf
    smat = 8.0 * fp["nnz"] + 4.0 * fp["shared_cols"] + 8.0 * nf + 16.0 * nf
    pmat = 4.0 * fp["precond_nnz"] + 8.0 * nf + 16.0 * nf
    it = 2 * smat + 2 * pmat + 8.0 * 22 * nf
    return stage + iterations * it + 8.0 * (stages + 4) * nd


def sensor_differences(t_a, tr_a, t_b, tr_b):
    """Relative l2-in-time differences of run a's sensor traces from run b's, b interpolated
    linearly at a's times (the measure of eq. error_ricker, between two runs): one value per
    sensor, components together."""
    out = []
    for r in range(tr_a.shape[1]):
        b = np.stack([np.interp(t_a, t_b, tr_b[:, r, c]) for c in range(2)], axis=1)
        out.append(float(np.linalg.norm(tr_a[:, r, :] - b) / max(np.linalg.norm(b), 1e-300)))
    return out


def run_sdirk_bilayer(k, steps=None, tol=1e-8, erk_traces=None):
    """The paper's implicit run of Table tab::cfl_cpu (Sec. 5.2): the granite-water bilayer,
    SDIRK(3,4), mixed order k' = k + 1 with the O(1/h) Lehrenfeld-Schoberl stabilisation, normalised
    step dt~ = cP dt / h = 0.398, from the pressure pulse to T_f = 0.5 s (or `steps` steps), face
    solves by BiCGStab to the relative residual `tol`.  Reports the run time, the iterations per
    face solve, DOF-stage updates/s (cell unknowns x stages x steps / s) and the algorithmic bytes
    of the whole step per second against the HBM peak, beside the paper's CPU seconds for its
    direct and iterative solvers (hardware not stated)."""
    from paper_2505_15771_amd import SdirkEngine
    mesh = M.granite_water()
    dt = SDIRK_BILAYER["dtt"] * 23.6 / 6000.0
    n_full = int(np.ceil(0.5 / dt - 1e-9))
    n = n_full if steps is None else min(steps, n_full)
    t0 = time.perf_counter()
    eng = SdirkEngine(mesh, k, dt, stages=3, mixed=True, alpha=1, tol=tol, max_iter=5000)
    setup_s = time.perf_counter() - t0
    eng.set_ricker_ic(PULSE_CENTER, PULSE_LAMBDA, theta=1.0, field=0)
    U0 = eng.get_state()
    eng.set_receivers(*BILAYER_SENSORS)
    eng.set_state(U0)
    eng.step(0.0, 2)   # warm-up
    eng.set_state(U0)
    E0 = eng.energy()
    s0, i0, _ = eng.stats()
    t1 = time.perf_counter()
    eng.step(0.0, n)
    secs = time.perf_counter() - t1
    s1, i1, res = eng.stats()
    E1 = eng.energy()
    fp = eng.footprint()
    iters = (i1 - i0) / max(s1 - s0, 1)
    byt = sdirk_bytes_per_step(fp, 3, iters * 3)
    gbs = byt * n / secs / 1e9
    out = dict(workload="paper granite-water bilayer (Table tab::cfl_cpu), 17710 squares, k=%d, SDIRK(3,4), "
                        "mixed order, T_f = 0.5 s" % k, dtype="f64", k=k, steps=n, steps_to_t_final=n_full, dt=dt,
               cell_dofs=fp["n_dof"], face_dofs=fp["n_face_dof"], face_matrix_nnz=fp["nnz"], tol=tol,
               iterations_per_solve=iters, max_rel_residual=res, run_s=secs, ms_per_step=1e3 * secs / n,
               setup_s=setup_s, value=fp["n_dof"] * 3 * n / secs, unit="DOF-stage updates/s",
               bytes_per_step=byt, gbs=gbs, frac=gbs / HBM_PEAK_GBS,
               run_s_to_t_final=secs * n_full / n,
               paper_cpu_s=dict(direct=SDIRK_BILAYER["paper_cpu_s"]["direct"][k],
                                iterative=SDIRK_BILAYER["paper_cpu_s"]["iterative"][k]),
               paper_hardware="not stated", energy_ratio=E1 / E0)
    if erk_traces is not None and n == n_full:
        d = sensor_differences(dt * np.arange(1, n + 1), eng.traces(), *erk_traces)
        out["sensor_diff_vs_erk4"] = dict(zip(("S_f_p", "S_s_v", "S_i_v"), d))
    eng.close()
    return out


def run_cfl(k, n=32, shots=32, delta=0.01, eps=0.05):
    """Algorithm algo_CFL (Sec. 5.1) on the two-material CFL geometry with h = 1/n, ERK(4),
    T_f = 1, from a seeded random state (every mode excited): hho_cfl_search with `shots`
    simultaneous candidates, against the paper's procedure run one candidate at a time on the
    same GPU (one-shot context, hho_erk_step per candidate, stopping at the first unstable)."""
    import torch
    from paper_2505_15771_amd import Engine, Unstable
    mesh = M.with_materials(M.bilayer_vertical(n))
    e = Engine(mesh, k, n_shots=shots)
    U0 = M.random_state(np.full(1, e.n_dof), 9000 + k)
    n_start = int(np.ceil(1.0 / (0.7 * e.dt_cfl(1.0))))
    for sh in range(shots):
        e.set_state(U0, shot=sh)
    e.cfl_search(1.0, n_start, delta, eps, max_rounds=1)  # warm-up (graph capture, workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ns, nu, tried = e.cfl_search(1.0, n_start, delta, eps)
    t_batched = time.perf_counter() - t0
    e.close()
    one = Engine(mesh, k, record_energy=True)
    one.set_state(U0)
    one.erk_step(0.0, 1.0 / n_start, 40)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_ns, seq_nu = 0, 0
    for N, _ in tried:
        one.set_state(U0)
        try:
            one.erk_step(0.0, 1.0 / N, N)
        except Unstable:
            seq_nu = N
            break
        seq_ns = N
    t_seq = time.perf_counter() - t0
    one.close()
    c, h = np.sqrt(3.0), 1.0 / n
    return dict(workload="CFL* search (Algorithm algo_CFL), two-material CFL geometry h = 1/%d, k = %d, ERK(4), "
                         "random initial state, %d candidates per launch" % (n, k, shots),
                cfl_bracket=[c / nu / h if nu else None, c / ns / h if ns else None], n_stable=ns, n_unstable=nu,
                candidates=len(tried), batched_s=t_batched, one_at_a_time_s=t_seq,
                speedup=t_seq / t_batched, same_bracket=(seq_ns, seq_nu) == (ns, nu))


PAPER_RATIO_GEO = {  # Table tab::ratio_geo: CFL* (triangles, squares, hexagons) per (k, s)
    (1, 2): (0.191, 0.205, 0.264), (1, 3): (0.238, 0.253, 0.329), (1, 4): (0.265, 0.282, 0.363),
    (2, 2): (0.106, 0.099, 0.136), (2, 3): (0.133, 0.123, 0.170), (2, 4): (0.147, 0.138, 0.188),
    (3, 2): (0.072, 0.063, 0.082), (3, 3): (0.090, 0.079, 0.102), (3, 4): (0.100, 0.087, 0.115)}


def run_cfl_geometry(n=16, shots=32, delta=0.01, eps=0.05, stab_speed=0):
    """CFL* on triangles, squares and hexagons (Table tab::ratio_geo) by hho_cfl_search on the
    two-material CFL geometry: 2n x n squares of side h = 1/n, the same squares cut into triangles
    (h = side of the generating square), and regular hexagons of about the same area (h = square
    root of the hexagon area), ERK(2/3/4), k = 1..3, T_f = 1, from a seeded random state;
    CFL* = sqrt(3) dt / h at the last stable step count, with the ratios to the triangles beside
    the paper's.  stab_speed selects c^s in the solid weight (0: c_P, 1: c_S)."""
    from paper_2505_15771_amd import Engine
    X = 2 * int(round(0.5 * n * np.sqrt(2.0 * np.sqrt(3.0))))
    hexm = M.honeycomb_bilayer(X)
    meshes = (("triangles", M.with_materials(M.bilayer_vertical(n, p_split=1.0, seed=5)), 1.0 / n),
              ("squares", M.with_materials(M.bilayer_vertical(n)), 1.0 / n),
              ("hexagons", M.with_materials(hexm), hexm["h"]))
    out = dict(workload="CFL* per cell shape (Table tab::ratio_geo), two-material CFL geometry, h ~ 1/%d, "
                        "tau^s with %s" % (n, "c_P" if stab_speed == 0 else "c_S"), results=[])
    t0 = time.perf_counter()
    for k in (1, 2, 3):
        for s in (2, 3, 4):
            row = {}
            for name, mesh, h in meshes:
                e = Engine(mesh, k, rk_stages=s, n_shots=shots, stab_speed=stab_speed)
                U0 = M.random_state(np.full(1, e.n_dof), 9200 + k)
                for sh in range(shots):
                    e.set_state(U0, shot=sh)
                ns, nu, _ = e.cfl_search(1.0, int(np.ceil(1.0 / (0.5 * e.dt_cfl(1.0)))), delta, eps)
                e.close()
                row[name] = np.sqrt(3.0) / ns / h if ns else None
            paper = PAPER_RATIO_GEO[(k, s)]
            out["results"].append(dict(
                k=k, stages=s, cfl=row,
                ratio=[row[m] / row["triangles"] if row[m] and row["triangles"] else None
                       for m in ("triangles", "squares", "hexagons")],
                paper_cfl=paper, paper_ratio=[v / paper[0] for v in paper]))
    out["run_s"] = time.perf_counter() - t0
    return out


ETA_GRID = {"fluid": (0.2, 0.4, 0.6, 0.7, 0.8, 0.9, 1.0, 1.2, 1.5, 2.0),
            "solid": (0.5, 0.8, 1.0, 1.25, 1.4, 1.5, 1.6, 1.75, 2.0, 2.5, 3.0)}


def run_eta_sweep(n=16, shots=32, delta=0.02, eps=0.05, ks=(1, 2, 3)):
    """CFL* as a function of the stabilisation weight (Sec. 5.1, Figure CFL_decoupled): pure
    acoustic (rho = c = 1) and pure elastic (rho = 1, cP = sqrt 3, cS = 1) unit squares of n x n
    quads, ERK(4), Algorithm algo_CFL by hho_cfl_search (T_f = 1, `shots` candidates per launch,
    step-count decrement delta, energy criterion eps) from a seeded random state, for every eta on
    the grid; CFL* = c dt / h at the last stable step count.  The paper finds the maximisers
    eta^f = 0.8 and eta^s = 1.5."""
    from paper_2505_15771_amd import Engine
    out = dict(workload="CFL* vs stabilisation weight (Figure CFL_decoupled), unit square %dx%d quads, ERK(4)" % (n, n),
               results=[])
    t0 = time.perf_counter()
    for medium, code, c in (("fluid", M.FLUID, 1.0), ("solid", M.SOLID, np.sqrt(3.0))):
        mesh = M.with_materials(M.single_medium(n, code))
        for k in ks:
            curve = []
            for eta in ETA_GRID[medium]:
                kw = dict(eta_f=eta) if medium == "fluid" else dict(eta_s=eta)
                e = Engine(mesh, k, n_shots=shots, **kw)
                U0 = M.random_state(np.full(1, e.n_dof), 9100 + k)
                for sh in range(shots):
                    e.set_state(U0, shot=sh)
                n_start = int(np.ceil(1.0 / (0.25 * e.dt_cfl(1.0))))
                ns, nu, tried = e.cfl_search(1.0, n_start, delta, eps)
                e.close()
                curve.append(dict(eta=eta, cfl=c * n / ns if ns else None, n_stable=ns, n_unstable=nu))
            best = max((r for r in curve if r["cfl"]), key=lambda r: r["cfl"])
            out["results"].append(dict(medium=medium, k=k, curve=curve, eta_best=best["eta"], cfl_best=best["cfl"]))
    out["run_s"] = time.perf_counter() - t0
    return out


def run_batch(steps=200, warmup=4):
    """Sixteen hybrid meshes of 20k-300k cells (k = 1, 2, 3 in turn), four Ricker shots each at
    seeded positions, float32 stepping with the float64 energy check, all advanced by one batch
    (graph branches per mesh)."""
    from paper_2505_15771_amd import Batch, Engine
    engines, dts = [], []
    bstep = 0
    for i, d in enumerate(M.batch_meshes()):
        mesh = M.with_materials(M.unit_square(d["n"], p_split=0.5, seed=d["seed"]))
        bstep += algorithmic_bytes_per_step(mesh, d["k"], 4, 4)[0]
        e = Engine(mesh, d["k"], dtype="f32", n_shots=4, record_energy=True)
        pos = M.shot_positions(4, 4100 + i)
        for sh in range(4):
            e.set_sources(sh, [pos[sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
        dts.append(e.dt_cfl(0.5))
        e.autotune()
        engines.append(e)
    b = Batch(engines)
    b.erk_step([0.0] * len(engines), dts, warmup)
    t0 = time.perf_counter()
    b.erk_step([warmup * dt for dt in dts], dts, steps)
    secs = time.perf_counter() - t0
    shot_dofs = sum(e.n_dof * 4 for e in engines)
    E = [e.energy() for e in engines]
    out = dict(workload="16 hybrid meshes (%d cells in total), k = 1/2/3, 4 shots each, one batch" %
               sum(e.n_cells for e in engines), dtype="f32", steps=steps, shot_dofs=int(shot_dofs),
               ms_per_step=secs * 1e3 / steps, value=shot_dofs * 4 * steps / secs,
               gbs=bstep * steps / secs / 1e9, frac=bstep * steps / secs / 1e9 / HBM_PEAK_GBS,
               finite=bool(all(np.all(np.isfinite(x)) for x in E)))
    b.close()
    for e in engines:
        e.close()
    return out


def copy_bandwidth(mib=1024, reps=20):
    """Achievable HBM bandwidth of a plain device copy (torch's elementwise copy kernel) of
    `mib` MiB: bytes read plus bytes written per second, best of `reps` timed copies."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    st = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        dst.copy_(src)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * mib * (1 << 20) / (best * 1e-3) / 1e9




# HBM bytes of the headline batch per step from rocprofv3 FETCH_SIZE / WRITE_SIZE counters summed
# over the step's dispatches, each counter scaled by what it reads for an elementwise kernel of
# known size; valid only for the kernel and host-plan sources with this digest (else null).
MEASURED_BATCH_TRAFFIC = {
    "sources_sha256": "cd1ec4e5494d0616d238def7cbd6035d035fb10730c2bc583c911d559283bc85",
    "bytes_per_step": 14783531251,   # FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00, 512 dispatches / 8 steps
}


def batch_engines(dtype="f32", shots=4, record_energy=True, autotune=True):
    """The headline workload's engines: mesh i of M.batch_meshes() (hybrid unit square, split seed
    4000 + i, degree 1 + i mod 3, the two-material setting), `shots` Ricker shots (f0 = 10, t0 =
    0.12, vertical unit force) at the seeded positions of M.shot_positions(4, 4100 + i), dt = half
    the CFL step of eq. CFL.  Returns (engines, dts, meshes)."""
    from paper_2505_15771_amd import Engine
    engines, dts, meshes = [], [], []
    for i, d in enumerate(M.batch_meshes()):
        mesh = M.with_materials(M.unit_square(d["n"], p_split=0.5, seed=d["seed"]))
        e = Engine(mesh, d["k"], dtype=dtype, n_shots=shots, record_energy=record_energy)
        pos = M.shot_positions(4, 4100 + i)
        for sh in range(shots):
            e.set_sources(sh, [pos[sh]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
        dts.append(e.dt_cfl(0.5))
        if autotune:
            e.autotune()
        engines.append(e)
        meshes.append((mesh, d["k"]))
    return engines, dts, meshes


def run_headline(steps, warmup):
    """Time `steps` steps of the headline batch after `warmup` untimed ones.  The batch call is
    synchronous: the host clock brackets it (the whole job: energy checks included); the HIP
    events the library records on the launch stream around the graph replays give the device time
    of the stage launches, on which the roofline fraction is priced."""
    import torch
    from paper_2505_15771_amd import Batch
    t_setup = time.perf_counter()
    engines, dts, meshes = batch_engines()
    bstep = sum(algorithmic_bytes_per_step(m, k, 4, 4)[0] for m, k in meshes)
    b = Batch(engines)
    setup_s = time.perf_counter() - t_setup
    b.reserve_steps(max(steps, warmup, 1))  # histories sized for the timed call: no re-capture in it
    b.erk_step([0.0] * len(engines), dts, max(warmup, 1))  # captures the step graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.erk_step([warmup * dt for dt in dts], dts, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = b.last_time_ms()
    shot_dofs = sum(e.n_dof * 4 for e in engines)
    E = [e.energy() for e in engines]
    out = dict(steps=steps, wall_s=wall, ms_per_step=wall * 1e3 / steps, device_ms_per_step=dev_ms / steps,
               value=shot_dofs * 4 * steps / wall, shot_dofs=int(shot_dofs),
               cells=int(sum(e.n_cells for e in engines)), bytes_per_step=bstep,
               gbs=bstep * steps / (dev_ms * 1e-3) / 1e9, setup_s=setup_s,
               finite=bool(all(np.all(np.isfinite(x)) for x in E)),
               tuning=[e.tuning()[0] for e in engines])
    out["frac"] = out["gbs"] / HBM_PEAK_GBS
    return b, engines, dts, meshes, out


def run_headline_f64_single(meshes, dts, steps):
    """The headline workload stepped the plain way: float64, one shot at a time (each mesh's four
    shots one after the other), same meshes, sources and steps.  Returns ms per step of the whole
    workload (the sum over meshes of four times one shot's time per step)."""
    import torch
    from paper_2505_15771_amd import Engine
    total_ms = 0.0
    for i, ((mesh, k), dt) in enumerate(zip(meshes, dts)):
        e = Engine(mesh, k, dtype="f64", n_shots=1, record_energy=True)
        e.set_sources(0, [M.shot_positions(4, 4100 + i)[0]], [[0.0, 1.0]], 10.0, 0.12, 1.0)
        e.autotune()
        e.reserve_steps(max(steps, 4))
        e.erk_step(0.0, dt, 4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.erk_step(4 * dt, dt, steps)
        torch.cuda.synchronize()
        total_ms += 4 * (time.perf_counter() - t0) * 1e3 / steps
        e.close()
    return total_ms


def headline_error(b, engines, dts, meshes, steps=3):
    """Relative L2 error of the batched float32 path against the float64 oracle: shot 0 of every
    mesh from a seeded random state with its Ricker source, `steps` steps through the batch (the
    other shots hold zero states); returns per-mesh errors."""
    from oracle import Oracle
    errs = []
    U0s = []
    for i, e in enumerate(engines):
        U0 = 1e-3 * np.random.default_rng(6000 + i).standard_normal(e.n_dof)
        U0s.append(U0)
        e.set_state(U0, shot=0)
        for sh in range(1, 4):
            e.set_state(np.zeros(e.n_dof), shot=sh)
    b.erk_step([0.0] * len(engines), dts, steps)
    for i, ((mesh, k), e, dt) in enumerate(zip(meshes, engines, dts)):
        o = Oracle(mesh, k)
        o.set_point_sources([M.shot_positions(4, 4100 + i)[0]], [0.0, 1.0], 10.0, 0.12, 1.0)
        ref = o.erk(U0s[i], 0.0, dt, steps)
        got = e.get_state(shot=0)
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        del o
    return errs


def _cpu_model():
    """lscpu's model name, with the CPU family / model / stepping numbers and the core count
    (a virtual machine may report a generic name)."""
    info = {}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in txt.splitlines():
            if ":" in ln:
                key, val = ln.split(":", 1)
                info[key.strip()] = val.strip()
    except Exception:
        pass
    name = info.get("Model name", "unknown")
    extra = ", ".join("%s %s" % (k_.lower(), info[k_]) for k_ in ("CPU family", "Model", "Stepping", "CPU(s)")
                      if k_ in info)
    return name + (" (%s)" % extra if extra else "")


def _omp_threads(n=None):
    """Set (n given) and return the OpenMP thread count the oracle's parallel loops use."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def cpu_baseline(meshes, dts, n_meshes=6, steps=2, runs=3):
    """The float64 oracle as it stands on the host cores: one shot of the first `n_meshes` meshes of
    the headline workload (degrees 1, 2, 3, 1, 2, 3), `steps` RK4 steps per run after two warm-up
    steps, median of `runs` runs, with all cores and with one; DOF-stage updates/s of the sample."""
    from oracle import Oracle
    sample = []
    for i in range(n_meshes):
        mesh, k = meshes[i]
        o = Oracle(mesh, k)
        o.set_point_sources([M.shot_positions(4, 4100 + i)[0]], [0.0, 1.0], 10.0, 0.12, 1.0)
        sample.append((o, 1e-3 * np.random.default_rng(7000 + i).standard_normal(o.ndof), dts[i]))
    dofs = sum(o.ndof for o, _, _ in sample)
    all_cores = _omp_threads()
    res = {}
    for label, nthr in (("all", all_cores), ("one", 1)):
        used = _omp_threads(nthr)
        for o, U, dt in sample:
            o.erk(U, 0.0, dt, 2)
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            for o, U, dt in sample:
                o.erk(U, 0.0, dt, steps)
            times.append(time.perf_counter() - t0)
        res[label] = dict(value=dofs * 4 * steps / float(np.median(times)), cores=used,
                          median_s=float(np.median(times)))
        print("cpu_baseline", label, json.dumps(res[label]), file=sys.stderr, flush=True)
    _omp_threads(all_cores)
    return dict(value=res["all"]["value"], unit="DOF-stage updates/s", cores=res["all"]["cores"], kind="oracle",
                single_core_value=res["one"]["value"],
                sample="meshes 0-%d of the headline workload (k=1,2,3,...; %d cell unknowns), one shot, float64, "
                       "%d RK4 steps per run, median of %d runs after 2 warm-up steps" % (n_meshes - 1, dofs, steps, runs),
                cpu=_cpu_model())


def _log(tag, obj):
    print(tag, json.dumps(obj), file=sys.stderr, flush=True)


def summary_line(steps, warmup, head, err, f64_ms, cpu, variants, extras, copy_gbs, traffic):
    """The one JSON line of the run (kept to a few kB: curves and workloads go to stderr)."""
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "16 seeded hybrid meshes of the two-material unit square (%d cells, 2e4-3e5 "
                               "each), k=1/2/3, 4 Ricker shots per mesh, float32 batched RK4 from captured "
                               "graphs, float64 energy per shot and step" % head["cells"],
                   "shot_dofs": head["shot_dofs"], "meshes": 16, "shots_per_mesh": 4,
                   "path": "graph replays (32/16/8/4/2/1-step graphs)"},
        "roofline": {"bound": "hbm", "achieved": round(head["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["frac"], "traffic": traffic, "kernel": "stage_kernel (every launch of a step)",
                     "bytes_per_step": head["bytes_per_step"], "device_us_per_step": round(head["device_ms_per_step"] * 1e3, 1),
                     "traffic_unit": "HBM bytes per step", "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(head["gbs"] / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "rel_err_vs_oracle": None if err is None else {"max": float("%.3g" % max(err)), "mean": float("%.3g" % np.mean(err)), "steps": 3,
                                                       "what": "shot 0 of each mesh, random state + source"},
        "f64_single_shot_ms_per_step": f64_ms,
        "speedup_vs_f64_single_shot": f64_ms / head["ms_per_step"],
        "variants": {"workload": "256x256 hybrid mesh", "runs": variants},
        "extras": extras,
    }
    return json.dumps(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variants", type=int, default=1, help="also time the 256x256 hybrid-mesh variants")
    ap.add_argument("--extras", type=int, default=1, help="also run the other workloads (stderr lines)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--check", type=int, default=1, help="error of the headline against the float64 oracle")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--shots", type=int, default=1)
    ap.add_argument("--only", choices=("headline", "variant", "adjoint", "basin", "batch", "paper", "cfl",
                                       "precision", "tableaux", "sdirk", "eta", "geometry", "perturbed", "3d",
                                       "3dhybrid", "3dmoved"),
                    default=None,
                    help="run one workload alone and print its JSON line (for profiling)")
    ap.add_argument("--only-steps", type=int, default=200)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (shots and meshes would "
              "shard across GPUs without exchange, one mesh by a per-stage halo of face traces); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_mb > 0:
        # one elementwise kernel that reads and writes exactly copy_mb MiB each (negation)
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print("copy calibration: neg kernel, %d MiB read + %d MiB written" % (args.copy_mb, args.copy_mb),
              file=sys.stderr)
        del src, dst
    if args.only:
        if args.only == "headline":
            b, engines, _, _, h = run_headline(args.only_steps, 5)
            b.close()
            for e in engines:
                e.close()
            print(json.dumps(h), flush=True)
            return
        fn = {"variant": lambda: run_variant(M.hybrid_square(256), args.k, args.dtype, args.shots,
                                             args.only_steps, 5),
              "adjoint": lambda: run_adjoint(2, args.dtype, steps=args.only_steps, ckpt=50, shots=args.shots),
              "basin": lambda: run_basin(args.dtype, steps=args.only_steps),
              "batch": lambda: run_batch(steps=args.only_steps),
              "paper": lambda: [run_paper_bilayer(1), run_paper_bilayer(3)],
              "cfl": lambda: [run_cfl(k_) for k_ in (1, 2, 3)],
              "precision": lambda: run_precision(steps=args.only_steps),
              "tableaux": lambda: run_tableaux(steps=args.only_steps),
              "eta": lambda: run_eta_sweep(),
              "perturbed": lambda: run_perturbed(dtype=args.dtype, steps=args.only_steps),
              "3d": lambda: run_3d(48 if args.k == 1 else 32, args.k, args.dtype, args.shots, args.only_steps, 5),
              "3dhybrid": lambda: run_3d(48, args.k, args.dtype, args.shots, args.only_steps, 5, kind="hybrid"),
              "3dmoved": lambda: run_3d(32, args.k, args.dtype, args.shots, args.only_steps, 5, kind="moved"),
              "geometry": lambda: [run_cfl_geometry(), run_cfl_geometry(stab_speed=1)],
              "sdirk": lambda: [run_sdirk_bilayer(k_, steps=args.only_steps,
                                                  erk_traces=run_paper_bilayer(k_, sensors=True)["_traces"])
                                for k_ in (1, 3)]
              }[args.only]
        print(json.dumps(fn()), flush=True)
        return

    # ---- headline: the batched float32 workload
    b, engines, dts, meshes, head = run_headline(args.steps, args.warmup)
    _log("headline", head)
    err = headline_error(b, engines, dts, meshes) if args.check else None
    if err is not None:
        _log("headline_error", {"rel_l2_vs_oracle": err})
    b.close()
    for e in engines:
        e.close()
    f64_ms = run_headline_f64_single(meshes, dts, max(min(args.steps, 100), 10))
    _log("headline_f64_single", {"ms_per_step": f64_ms})
    cpu = cpu_baseline(meshes, dts) if args.cpu_baseline else None

    # ---- the 256 x 256 hybrid mesh, one launch per stage (float32 / float64, 1 or 8 shots)
    variants = []
    if args.variants:
        mesh = M.hybrid_square(256)
        for (k, dt_, sh) in ((2, "f32", 1), (2, "f64", 1), (3, "f32", 1), (3, "f64", 1), (2, "f32", 8),
                             (3, "f32", 8)):
            v = run_variant(mesh, k, dt_, sh, max(min(args.steps, 400), 10), 5)
            _log("variant", v)
            variants.append(dict(k=k, dtype=dt_, shots=sh, us_per_step=round(v["ms_per_step"] * 1e3, 2),
                                 frac=round(v["frac"], 3)))

    # ---- other workloads: one stderr line each, a few figures kept in the summary
    extras = {}
    if args.extras:
        for dt_, sh_ in (("f32", 1), ("f64", 1), ("f32", 8)):
            v = run_adjoint(2, dt_, shots=sh_)
            _log("workload", v)
            extras["adjoint_%s_%dshot" % (dt_, sh_)] = dict(ms=round(v["adjoint_ms"], 1),
                                                             vs_forward=round(v["ratio"], 2))
        for dt_ in ("f32", "f64"):
            v = run_basin(dt_)
            _log("workload", v)
            extras["basin_%s" % dt_] = dict(us_per_step=round(v["ms_per_step"] * 1e3, 1), frac=round(v["frac"], 3))
        for k_ in (1, 3):
            v = run_paper_bilayer(k_, sensors=True)
            erk_tr = v.pop("_traces")
            _log("workload", v)
            w = run_sdirk_bilayer(k_, erk_traces=erk_tr)
            w["erk4_run_s"] = v["run_s"]
            _log("workload", w)
            extras["paper_bilayer_k%d" % k_] = dict(erk4_s=round(v["run_s"], 4), sdirk34_s=round(w["run_s_to_t_final"], 3),
                                                    paper_erk4_cpu_s=v["paper_cpu_s"])
        for (n_, k_, dt_, sh_, kd_) in ((48, 1, "f32", 1, "tets"), (32, 2, "f32", 1, "tets"), (32, 2, "f64", 1, "tets"),
                                        (32, 2, "f32", 4, "tets"), (48, 2, "f32", 1, "hybrid"),
                                        (32, 1, "f32", 1, "moved")):
            v = run_3d(n_, k_, dt_, sh_, 200, 5, kind=kd_)
            _log("workload", v)
            extras["cube3d_%s_k%d_%s_%dshot" % (kd_, k_, dt_, sh_)] = dict(us_per_step=round(v["ms_per_step"] * 1e3, 1),
                                                                            frac=round(v["frac"], 3))
        for k_ in (1, 2, 3):
            _log("workload", run_cfl(k_))
        _log("workload", run_precision())
        _log("workload", run_tableaux())
        _log("workload", run_eta_sweep())
        for ss in (0, 1):
            _log("workload", run_cfl_geometry(stab_speed=ss))
    copy_gbs = copy_bandwidth()
    _log("copy", {"gbs": copy_gbs})

    traffic = None
    if MEASURED_BATCH_TRAFFIC["sources_sha256"] == stage_sources_digest():
        traffic = MEASURED_BATCH_TRAFFIC["bytes_per_step"]
    print(summary_line(args.steps, args.warmup, head, err, f64_ms, cpu, variants, extras, copy_gbs, traffic),
          flush=True)


if __name__ == "__main__":
    main()
