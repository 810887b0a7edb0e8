"""GPU parity of the HIP path (libhho.so through its C ABI) against the FP64 oracle.

Tolerances (relative L2 of the cell unknowns, and of energies and receiver traces):
1e-12 when stepping in float64, 1e-5 when stepping in float32 (factors formed in
float64 and rounded, energy in float64).
"""
import math
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
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def engine(mesh, k, **kw):
    from paper_2505_15771_amd import Engine
    return Engine(mesh, k, **kw)


def oracle(mesh, k, **kw):
    from oracle import Oracle
    return Oracle(mesh, k, **kw)


def test_manufactured_16x16_k1_200_steps():
    """Unit square 16 x 16 quads, interface y = 1/2, k = 1, RK4, dt = 0.5 * 0.282 * h / sqrt(3),
    200 steps from the projected manufactured solution with its separable forcing."""
    from oracle.manufactured import Manufactured
    say("case: manufactured 16x16 k=1 200 steps fp64")
    mesh = M.manufactured_square(16)
    o = oracle(mesh, 1)
    ms = Manufactured(omega=1, theta=math.sqrt(2.0), phase=float(np.random.default_rng(1001).uniform(0, 2 * np.pi)))
    U0 = o.project(*ms.fields(0.0))
    terms, om, ph = ms.forcing_terms()
    g = np.stack([o.load_vector(*tm) for tm in terms])
    o.set_dense_load(g, om, ph)
    dt = 0.5 * 0.282 * (1.0 / 16) / math.sqrt(3.0)
    ref = o.erk(U0, 0.0, dt, 200)
    e = engine(mesh, 1)
    e.set_loads(g, om, ph)
    e.set_state(U0)
    e.erk_step(0.0, dt, 200)
    got = e.get_state()
    err = rel(got, ref)
    say("rel L2 =", err)
    assert err < TOL64


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("s", [2, 3, 4])
def test_random_state_hanging_hybrid(k, s):
    """Hybrid mesh with 2:1 hanging nodes (pentagons, quadrilateral triangles) and the
    interface, perturbed materials, random state: ERK(s) steps match the oracle."""
    say("case: hanging hybrid k=%d s=%d fp64" % (k, s))
    mesh = M.with_materials(M.unit_square(10, p_split=0.5, seed=7,
                                          refine=np.random.default_rng(8).random((10, 10)) < 0.3),
                            perturb=0.1, seed=9)
    o = oracle(mesh, k)
    U0 = np.random.default_rng(k * 10 + s).standard_normal(o.ndof)
    dt = 0.3 * 0.087 * 0.05 / math.sqrt(3.0)
    ref = o.erk(U0, 0.0, dt, 7, s=s)
    e = engine(mesh, k, rk_stages=s)
    e.set_state(U0)
    e.erk_step(0.0, dt, 7)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < TOL64


@pytest.mark.parametrize("eta_f,eta_s,stab_speed", [(0.3, 3.0, 0), (2.0, 0.5, 1), (0.8, 1.5, 1)])
@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", 1e-5)])
def test_stabilisation_weights_and_speed(eta_f, eta_s, stab_speed, dtype, tol):
    """The stabilisation weights eta^f, eta^s (the paper's sweep of Sec. 5.1) and the solid
    stabilisation speed (c_P or c_S) change tau and every coefficient derived from it on the
    host; ERK(3) steps on a hanging-node hybrid mesh match the oracle built with the same values."""
    say("case: eta_f=%g eta_s=%g stab_speed=%d %s" % (eta_f, eta_s, stab_speed, dtype))
    mesh = M.with_materials(M.unit_square(10, p_split=0.5, seed=17,
                                          refine=np.random.default_rng(18).random((10, 10)) < 0.3),
                            perturb=0.1, seed=19)
    o = oracle(mesh, 2, eta_f=eta_f, eta_s=eta_s, stab_speed=stab_speed)
    U0 = np.random.default_rng(77).standard_normal(o.ndof)
    dt = 0.2 * 0.087 * 0.05 / math.sqrt(3.0)
    ref = o.erk(U0, 0.0, dt, 6, s=3)
    e = engine(mesh, 2, rk_stages=3, eta_f=eta_f, eta_s=eta_s, stab_speed=stab_speed, dtype=dtype)
    e.set_state(U0)
    e.erk_step(0.0, dt, 6)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < tol


@pytest.mark.parametrize("k", [1, 2, 3])
def test_float32_stepping(k):
    """float32 matvecs and accumulation against the float64 oracle."""
    say("case: fp32 k=%d" % k)
    mesh = M.with_materials(M.unit_square(12, p_split=0.5, seed=3), perturb=0.1, seed=4)
    o = oracle(mesh, k)
    U0 = o.project([lambda x, y: np.sin(3 * x) * np.cos(2 * y), lambda x, y: x * y, lambda x, y: np.cos(x)],
                   [lambda x, y: np.sin(2 * y), lambda x, y: x - y, lambda x, y: x * x, lambda x, y: y,
                    lambda x, y: np.sin(x + y)])
    dt = 0.4 * 0.087 / 12 / math.sqrt(3.0)
    ref = o.erk(U0, 0.0, dt, 50)
    e = engine(mesh, k, dtype="f32")
    e.set_state(U0)
    e.erk_step(0.0, dt, 50)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < TOL32


def test_multishot_sources_receivers_energy():
    """Three shots (a lane count that is not a power of two) with different initial states and
    Ricker point sources; receivers record p in the fluid and v in the solid after every step;
    energies per step; all against the oracle shot by shot."""
    say("case: 3 shots, sources, receivers, energy")
    k = 2
    mesh = M.with_materials(M.unit_square(8, p_split=0.5, seed=11), perturb=0.1, seed=12)
    rx = np.array([[0.31, 0.77], [0.62, 0.91], [0.45, 0.21], [0.83, 0.33]])
    fld = np.array([0, 0, 1, 1], np.int32)
    srcs = [np.array([[0.5, 0.25]]), np.array([[0.3, 0.7]]), np.array([[0.71, 0.12], [0.2, 0.3]])]
    dirs = [np.array([[0.0, 1.0]]), np.array([[1.0, 0.0]]), np.array([[0.6, -0.8], [1.0, 0.0]])]
    dt = 0.5 * 0.138 / 8 / math.sqrt(3.0)
    nsteps = 30
    e = engine(mesh, k, n_shots=3, record_energy=True)
    e.set_receivers(rx, fld)
    refs = []
    for sh in range(3):
        o = oracle(mesh, k)
        U0 = 0.1 * np.random.default_rng(50 + sh).standard_normal(o.ndof)
        o.set_point_sources(srcs[sh], dirs[sh], 10.0, 0.12, 1.0 + sh)
        e.set_sources(sh, srcs[sh], dirs[sh], 10.0, 0.12, 1.0 + sh)
        e.set_state(U0, shot=sh)
        U = U0.copy()
        tr = np.zeros((nsteps, 4, 2))
        En = np.zeros(nsteps)
        for n in range(nsteps):
            U = o.erk(U, n * dt, dt, 1)
            En[n] = o.energy(U)
            for r in range(4):
                c, vals = o.point_values(U, *rx[r])
                tr[n, r, :(1 if fld[r] == 0 else 2)] = vals[:1] if fld[r] == 0 else vals[:2]
        refs.append((U, tr, En))
    e.erk_step(0.0, dt, nsteps)
    E_now = e.energy()
    for sh in range(3):
        U, tr, En = refs[sh]
        err_u = rel(e.get_state(sh), U)
        err_t = rel(e.traces(sh), tr)
        err_e = rel(e.energy_history(sh), En)
        say("shot", sh, "state", err_u, "traces", err_t, "energy", err_e)
        assert err_u < TOL64 and err_t < TOL64 and err_e < TOL64
        assert abs(E_now[sh] - En[-1]) < TOL64 * En[-1]


def test_single_cell_and_zero_steps():
    """Degenerate inputs: one fluid triangle (all faces on the boundary), zero steps."""
    say("case: single cell")
    mesh = M.with_materials(dict(xy=np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
                                 cell_ptr=np.array([0, 3], np.int32), cell_vtx=np.array([0, 1, 2], np.int32),
                                 medium=np.array([0], np.uint8)))
    o = oracle(mesh, 3)
    U0 = np.random.default_rng(2).standard_normal(o.ndof)
    e = engine(mesh, 3)
    e.set_state(U0)
    e.erk_step(0.0, 1e-3, 0)
    assert rel(e.get_state(), U0) == 0.0
    e.erk_step(0.0, 1e-3, 5)
    assert rel(e.get_state(), o.erk(U0, 0.0, 1e-3, 5)) < TOL64


def test_device_pointer_state():
    """State handed over as float64 torch cuda tensors (device pointers through the C ABI)."""
    import torch
    say("case: device pointers")
    mesh = M.with_materials(M.unit_square(6, p_split=0.5, seed=1))
    o = oracle(mesh, 2)
    U0 = np.random.default_rng(3).standard_normal(o.ndof)
    e = engine(mesh, 2)
    e.set_state(torch.tensor(U0, device="cuda:0"))
    e.erk_step(0.0, 1e-3, 3)
    out = torch.zeros(o.ndof, dtype=torch.float64, device="cuda:0")
    e.get_state(out=out)
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), o.erk(U0, 0.0, 1e-3, 3)) < TOL64


def test_unstable_time_step_is_reported():
    """Energy criterion of Algorithm algo_CFL: a time step far above the CFL limit makes the
    lossless run blow up and hho_erk_step returns HHO_ERR_UNSTABLE."""
    from paper_2505_15771_amd import Unstable
    say("case: unstable dt")
    mesh = M.manufactured_square(8)
    e = engine(mesh, 1, record_energy=True)
    e.set_state(np.random.default_rng(5).standard_normal(e.n_dof))
    with pytest.raises(Unstable):
        e.erk_step(0.0, 3.0 * 0.282 / 8 / math.sqrt(3.0), 200)


@pytest.mark.parametrize("k,dtype", [(2, "f64"), (2, "f32"), (3, "f64")])
def test_full_size_hybrid_256(k, dtype):
    """The 256 x 256 hybrid workload (random quads / split triangles, materials +-10 %)
    in the launch configuration the benchmark times: a few RK4 steps from a smooth state,
    compared with the oracle on the whole mesh."""
    say("case: full-size hybrid 256 k=%d %s" % (k, dtype))
    mesh = M.hybrid_square(256)
    o = oracle(mesh, k)
    U0 = np.random.default_rng(2002).standard_normal(o.ndof)
    cmax = M.max_wave_speed(mesh)
    cfl = {1: 0.265, 2: 0.138, 3: 0.087}[k]
    dt = 0.5 * cfl * (1.0 / 256) / cmax
    ref = o.erk(U0, 0.0, dt, 3)
    e = engine(mesh, k, dtype=dtype)
    e.set_state(U0)
    say("tuning", e.autotune(), e.tuning())  # as the benchmark does before timing
    e.erk_step(0.0, dt, 3)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < (TOL64 if dtype == "f64" else TOL32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_basin(dtype):
    """The synthetic basin at full size (543k cells: triangles, quadrilaterals and 2:1 hanging-node
    polygons, water over a layered half-space, physical units), k = 2, ERK(4) at half the CFL step,
    two steps from a random state, on the whole mesh against the oracle."""
    say("case: full-size basin k=2 %s" % dtype)
    mesh = M.basin()
    o = oracle(mesh, 2)
    U0 = np.random.default_rng(3001).standard_normal(o.ndof)
    e = engine(mesh, 2, dtype=dtype)
    dt = e.dt_cfl(0.5)
    ref = o.erk(U0, 0.0, dt, 2)
    e.set_state(U0)
    say("tuning", e.autotune(), e.tuning())  # as the benchmark does before timing
    e.erk_step(0.0, dt, 2)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < (TOL64 if dtype == "f64" else TOL32)


def test_full_size_float32_error_growth():
    """The 256 x 256 hybrid workload, k = 2, with its Ricker point source and receivers, stepped
    200 steps in float32 at half the CFL step: the relative L2 error against the float64 oracle
    (state and receiver traces) is reported every 50 steps and stays below 1e-5."""
    say("case: full-size hybrid 256 k=2 f32, 200 steps, error growth")
    mesh = M.hybrid_square(256)
    o = oracle(mesh, 2)
    src, dirs = [[0.5, 0.25]], [[0.0, 1.0]]
    o.set_point_sources(src, dirs, 10.0, 0.12, 1.0)
    rx = M.receiver_line(8, 0.75)
    U = 1e-3 * np.random.default_rng(2003).standard_normal(o.ndof)
    e = engine(mesh, 2, dtype="f32")
    e.set_sources(0, src, dirs, 10.0, 0.12, 1.0)
    e.set_receivers(rx, np.zeros(8, np.int32))
    e.set_state(U)
    e.autotune()  # as the benchmark does before timing
    dt = e.dt_cfl(0.5)
    t = 0.0
    for block in range(4):
        tr = np.zeros((50, 8, 2))
        for n in range(50):
            U = o.erk(U, t + n * dt, dt, 1)
            for r in range(8):
                tr[n, r, 0] = o.point_values(U, *rx[r])[1][0]
        e.erk_step(t, dt, 50)
        t += 50 * dt
        eu, et = rel(e.get_state(), U), rel(e.traces(), tr)
        say("steps", 50 * (block + 1), "state", eu, "traces", et)
        assert eu < TOL32 and et < TOL32


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", 1e-5)])
def test_mirrored_mesh(dtype, tol):
    """The mirror-symmetric hybrid mesh of the oracle's symmetry pin (random cuts on one side,
    reflected on the other, so every face is seen in both orientations): ERK(4) steps from a
    random state match the oracle, and from mirror-symmetric data the GPU state stays symmetric
    (compared through the oracle's point evaluation at mirrored points)."""
    from test_oracle_pins import _mirrored_hybrid
    say("case: mirrored hybrid mesh %s" % dtype)
    mesh = _mirrored_hybrid()
    o = oracle(mesh, 2)
    e = engine(mesh, 2, dtype=dtype)
    U0 = np.random.default_rng(31).standard_normal(o.ndof)
    e.set_state(U0)
    e.erk_step(0.0, 0.002, 12)
    err = rel(e.get_state(), o.erk(U0, 0.0, 0.002, 12))
    say("rel L2 =", err)
    assert err < tol
    g = lambda x, y: np.exp(-20 * (x - 0.5) ** 2) * np.sin(np.pi * y)
    odd = lambda x, y: (x - 0.5) * np.exp(-10 * (x - 0.5) ** 2) * np.cos(2 * y)
    S0 = o.project([g, odd, lambda x, y: g(x, y) * y],
                   [odd, g, lambda x, y: g(x, y) * (1 + y), lambda x, y: np.cos(3 * y) * g(x, y), odd])
    e.set_state(S0)
    e.erk_step(0.0, 0.002, 12)
    V = e.get_state()
    parity = {0: [1, -1, 1], 1: [-1, 1, 1, 1, -1]}
    worst, scale = 0.0, 0.0
    for x, y in np.random.default_rng(8).uniform(0.02, 0.98, (100, 2)):
        if abs(x - 0.5) < 1e-3 or abs(y - 0.5) < 1e-3:
            continue
        c1, a = o.point_values(V, x, y)
        _, b = o.point_values(V, 1.0 - x, y)
        worst = max(worst, float(np.max(np.abs(a - np.array(parity[int(o.medium[c1])]) * b))))
        scale = max(scale, float(np.max(np.abs(a))))
    say("symmetry defect", worst / scale)
    assert worst <= (1e-12 if dtype == "f64" else 1e-5) * scale
    e.close()


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", 1e-5)])
def test_honeycomb_mesh(k, dtype, tol):
    """Regular hexagons (six faces per cell) with pentagons and quadrilaterals where the domain
    boundary and the fluid-solid interface x = 0 cut them: ERK(4) from a random state against the
    oracle."""
    say("case: honeycomb k=%d %s" % (k, dtype))
    mesh = M.with_materials(M.honeycomb_bilayer(8), perturb=0.1, seed=41)
    o = oracle(mesh, k)
    e = engine(mesh, k, dtype=dtype)
    U0 = np.random.default_rng(40 + k).standard_normal(o.ndof)
    dt = 0.3 * e.dt_cfl(1.0)
    e.set_state(U0)
    e.erk_step(0.0, dt, 10)
    err = rel(e.get_state(), o.erk(U0, 0.0, dt, 10))
    say("rel L2 =", err)
    assert err < tol


@pytest.mark.parametrize("k", [1, 2, 3])
def test_partly_perturbed_mesh(k):
    """Vertices moved left of x = 1/2 only: the cells there each have their own shape and go to
    pooled groups (several workgroups each, ragged tails), the lattice cells on the right keep
    groups with shared class tables, so every stage runs both launches over real work.  Two
    shots with Ricker point sources in both halves, receivers in both halves and the energy
    recorded at every step, float64 against the oracle; float32 stepping of the state."""
    say("case: partly perturbed mesh k=%d" % k)
    mesh = M.with_materials(M.perturbed_square(32, seed=5, x_max=0.5), perturb=0.1, seed=6)
    from paper_2505_15771_amd import Inspect
    ins = Inspect(mesh, k)
    assert ins.pooled.any() and not ins.pooled.all()
    rx = np.array([[0.21, 0.77], [0.81, 0.62], [0.33, 0.18], [0.74, 0.41]])
    fld = np.array([0, 0, 1, 1], np.int32)
    srcs = [np.array([[0.23, 0.31], [0.7, 0.8]]), np.array([[0.41, 0.66]])]
    dirs = [np.array([[0.6, -0.8], [1.0, 0.0]]), np.array([[1.0, 0.0]])]
    nsteps = 20
    e = engine(mesh, k, n_shots=2, record_energy=True)
    dt = 0.3 * e.dt_cfl(1.0)
    e.set_receivers(rx, fld)
    e32 = engine(mesh, k, n_shots=2, dtype="f32")
    refs = []
    for sh in range(2):
        o = oracle(mesh, k)
        U0 = 0.1 * np.random.default_rng(70 + sh).standard_normal(o.ndof)
        o.set_point_sources(srcs[sh], dirs[sh], 10.0, 0.05, 1.0 + sh)
        for eng in (e, e32):
            eng.set_sources(sh, srcs[sh], dirs[sh], 10.0, 0.05, 1.0 + sh)
            eng.set_state(U0, shot=sh)
        U = U0.copy()
        tr = np.zeros((nsteps, 4, 2))
        En = np.zeros(nsteps)
        for n in range(nsteps):
            U = o.erk(U, n * dt, dt, 1)
            En[n] = o.energy(U)
            for r in range(4):
                c, vals = o.point_values(U, *rx[r])
                tr[n, r, :(1 if fld[r] == 0 else 2)] = vals[:1] if fld[r] == 0 else vals[:2]
        refs.append((U, tr, En))
    e.erk_step(0.0, dt, nsteps)
    e32.erk_step(0.0, dt, nsteps)
    for sh in range(2):
        U, tr, En = refs[sh]
        err_u = rel(e.get_state(sh), U)
        err_t = rel(e.traces(sh), tr)
        err_e = rel(e.energy_history(sh), En)
        err32 = rel(e32.get_state(sh), U)
        say("shot", sh, "state", err_u, "traces", err_t, "energy", err_e, "float32 state", err32)
        assert err_u < TOL64 and err_t < TOL64 and err_e < TOL64
        assert err32 < 1e-5


@pytest.mark.parametrize("k", [1, 2, 3])
def test_perturbed_vertices_mesh(k):
    """Every vertex moved at random (no two cells share a shape: more than 64 classes, all of them
    pooled, every lane reading its own class table): ERK(4) from a random state against the
    oracle, float64 and float32 stepping."""
    say("case: perturbed-vertex mesh k=%d" % k)
    mesh = M.with_materials(M.perturbed_square(8, seed=11), perturb=0.1, seed=12)
    o = oracle(mesh, k)
    e = engine(mesh, k)
    U0 = np.random.default_rng(50 + k).standard_normal(o.ndof)
    dt = 0.3 * e.dt_cfl(1.0)
    e.set_state(U0)
    e.erk_step(0.0, dt, 8)
    ref = o.erk(U0, 0.0, dt, 8)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < TOL64
    e32 = engine(mesh, k, dtype="f32")
    e32.set_state(U0)
    e32.erk_step(0.0, dt, 8)
    err32 = rel(e32.get_state(), ref)
    say("rel L2 (float32) =", err32)
    assert err32 < 1e-5
    # only the pooled launch runs on such a mesh, so it also advances the clock: a Ricker source
    # and receivers after every step depend on it
    nsteps, src, dirs = 12, [[0.4, 0.3]], [[0.6, -0.8]]
    rx, fld = np.array([[0.3, 0.7], [0.6, 0.2]]), np.array([0, 1], np.int32)
    o.set_point_sources(src, dirs, 10.0, 0.05, 1.0)
    e.set_sources(0, src, dirs, 10.0, 0.05, 1.0)
    e.set_receivers(rx, fld)
    e.set_state(U0)
    e.erk_step(0.0, dt, nsteps)
    U, tr = U0.copy(), np.zeros((nsteps, 2, 2))
    for n in range(nsteps):
        U = o.erk(U, n * dt, dt, 1)
        tr[n, 0, :1] = o.point_values(U, *rx[0])[1][:1]
        tr[n, 1, :2] = o.point_values(U, *rx[1])[1][:2]
    err_u, err_t = rel(e.get_state(), U), rel(e.traces(0), tr)
    say("with source: state", err_u, "traces", err_t)
    assert err_u < TOL64 and err_t < TOL64
