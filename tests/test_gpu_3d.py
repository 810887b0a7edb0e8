"""GPU parity of the three-dimensional HIP path (hho_setup3d through the C ABI) against the
three-dimensional FP64 oracle (oracle/oracle3d.py): tetrahedra, parallelepiped hexahedra, sheared
columns of hexahedra and triangular prisms, and tetrahedra with moved vertices (pooled class tables), two materials with the fluid-solid
interface, k = 1 and 2, ERK(2/3/4), several shots, a batch that mixes a two- and a
three-dimensional context, and a larger mesh checked through properties that hold at any size.

Tolerances (relative L2 of the cell unknowns and of energies): 1e-12 stepping in float64, 1e-5
stepping in float32.
"""
import sys

import numpy as np
import pytest

from synth import meshes as M

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
SHEAR = [[1.0, 0.2, 0.1], [0.0, 1.0, 0.3], [0.0, 0.0, 1.0]]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_ORACLES = {}


def oracle3d(mesh, k, key=None):
    """The oracle of a mesh (cached under `key` across the float64 / float32 cases)."""
    if key is not None and (key, k) in _ORACLES:
        return _ORACLES[(key, k)]
    from oracle.oracle3d import Oracle3D
    cells = [tuple(int(v) for v in mesh["cell_vtx"][mesh["cell_ptr"][c]:mesh["cell_ptr"][c + 1]])
             for c in range(len(mesh["medium"]))]
    o = Oracle3D(dict(xyz=mesh["xyz"], cells=cells, medium=mesh["medium"], rho=mesh["rho"], a=mesh["a"],
                      b=mesh["b"]), k)
    if key is not None:
        _ORACLES[(key, k)] = o
    return o


def dt_for(mesh, n, k):
    """A step well inside the stability limit: 0.1 (k = 1) or 0.05 (k = 2) times h / c_max."""
    return (0.1 if k == 1 else 0.05) / n / M.max_wave_speed3d(mesh)


MESHES = {
    "tets": lambda: (M.with_materials3d(M.unit_cube(4), perturb=0.1, seed=21), 4),
    "hexes": lambda: (M.with_materials3d(M.unit_cube(4, tets=False, shear=SHEAR), perturb=0.1, seed=22), 4),
    "tets-moved": lambda: (M.with_materials3d(M.unit_cube(4, jitter=0.25, seed=23), perturb=0.1, seed=24), 4),
    "hexes-prisms": lambda: (M.with_materials3d(M.unit_cube(4, kind="hybrid", seed=25, shear=SHEAR), perturb=0.1,
                                                seed=26), 4),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("case", sorted(MESHES))
def test_3d_parity_random_state(case, k, dtype):
    from paper_2505_15771_amd import Engine
    mesh, n = MESHES[case]()
    say("case: 3d %s k=%d %s, 40 RK4 steps" % (case, k, dtype))
    o = oracle3d(mesh, k, key=case)
    U0 = np.random.default_rng(31).standard_normal(o.ndof)
    dt = dt_for(mesh, n, k)
    ref = o.erk(U0, dt, 40)
    e = Engine(mesh, k, dtype=dtype, record_energy=True)
    assert e.n_dof == o.ndof
    e.set_state(U0)
    e.erk_step(0.0, dt, 40)  # one 32-step graph and one 8-step graph
    err = rel(e.get_state(), ref)
    tol = TOL64 if dtype == "f64" else TOL32
    say("rel L2 =", err)
    assert err < tol
    # energies: the float64 energy of the final state, and a non-increasing history (no sources)
    E = e.energy()[0]
    assert abs(E - o.energy(ref)) < tol * o.energy(ref)
    H = e.energy_history()
    assert len(H) == 40 and np.all(np.diff(H) <= 1e-12 * H[0]) and H[-1] < o.energy(U0)
    e.close()


@pytest.mark.parametrize("stages", [2, 3])
def test_3d_tableaux(stages):
    from oracle.oracle import ERK_TABLEAUX
    from paper_2505_15771_amd import Engine
    mesh, n = MESHES["tets"]()
    k = 2
    say("case: 3d tets k=2 ERK(%d) 12 steps f64" % stages)
    o = oracle3d(mesh, k)
    U0 = np.random.default_rng(32).standard_normal(o.ndof)
    dt = 0.5 * dt_for(mesh, n, k)
    assert stages in ERK_TABLEAUX
    ref = o.erk(U0, dt, 12, s=stages)
    e = Engine(mesh, k, rk_stages=stages)
    e.set_state(U0)
    e.erk_step(0.0, dt, 12)
    err = rel(e.get_state(), ref)
    say("rel L2 =", err)
    assert err < TOL64


def test_3d_shots_and_ragged_groups():
    """Three shots from different states on 6^3 cubes (1296 tetrahedra: groups of 108 cells, two
    64-lane blocks each with a ragged tail), float64 and float32, 70 steps (two 32-step graphs, a
    4-step and a 2-step graph)."""
    from paper_2505_15771_amd import Engine
    n, k = 6, 1
    mesh = M.with_materials3d(M.unit_cube(n), rho_f=1.2, c_f=1.4, rho_s=2.0, lam=1.5, mu=0.8)
    say("case: 3d 6^3 tets k=1, 3 shots, 70 steps")
    o = oracle3d(mesh, k)
    rng = np.random.default_rng(33)
    U0 = [rng.standard_normal(o.ndof) for _ in range(3)]
    dt = dt_for(mesh, n, k)
    refs = [o.erk(u, dt, 70) for u in U0]
    for dtype, tol in (("f64", TOL64), ("f32", TOL32)):
        e = Engine(mesh, k, dtype=dtype, n_shots=3)
        for sh, u in enumerate(U0):
            e.set_state(u, shot=sh)
        e.erk_step(0.0, dt, 70)
        for sh in range(3):
            err = rel(e.get_state(shot=sh), refs[sh])
            say(dtype, "shot", sh, "rel L2 =", err)
            assert err < tol
        e.close()


def test_3d_batch_with_a_two_dimensional_context():
    """hho_batch_erk_step over a 2D hybrid-mesh context and a 3D hexahedron context (36 steps)."""
    from oracle import Oracle
    from paper_2505_15771_amd import Batch, Engine
    say("case: batch of a 2D and a 3D context, 36 steps")
    m2 = M.with_materials(M.unit_square(6, p_split=0.5, seed=3), perturb=0.1, seed=2)
    m3, n3 = MESHES["hexes"]()
    o2, o3 = Oracle(m2, 2), oracle3d(m3, 2)
    U2 = np.random.default_rng(34).standard_normal(o2.ndof)
    U3 = np.random.default_rng(35).standard_normal(o3.ndof)
    dt2 = 0.3 * 0.138 / 6 / np.sqrt(3.0)
    dt3 = dt_for(m3, n3, 2)
    r2, r3 = o2.erk(U2, 0.0, dt2, 36), o3.erk(U3, dt3, 36)
    e2, e3 = Engine(m2, 2, record_energy=True), Engine(m3, 2, record_energy=True)
    e2.set_state(U2)
    e3.set_state(U3)
    b = Batch([e2, e3])
    b.erk_step([0.0, 0.0], [dt2, dt3], 36)
    err2, err3 = rel(e2.get_state(), r2), rel(e3.get_state(), r3)
    say("rel L2 2D =", err2, "3D =", err3)
    assert err2 < TOL64 and err3 < TOL64
    b.close()


def test_3d_full_size_properties():
    """24^3 cubes cut into 82,944 tetrahedra, k = 2: float32 against float64 stepping after 20 steps
    (the oracle is too slow at this size), the energy never increasing without sources, and the
    float64 energy of the two runs agreeing."""
    from paper_2505_15771_amd import Engine
    n, k = 24, 2
    mesh = M.with_materials3d(M.unit_cube(n), perturb=0.1, seed=25)
    say("case: 3d 24^3 tets k=2 20 steps f64 vs f32")
    e64 = Engine(mesh, k, dtype="f64", record_energy=True)
    U0 = np.random.default_rng(36).standard_normal(e64.n_dof)
    dt = dt_for(mesh, n, k)
    e64.set_state(U0)
    e64.erk_step(0.0, dt, 20)
    a = e64.get_state()
    H = e64.energy_history()
    e32 = Engine(mesh, k, dtype="f32", record_energy=True)
    e32.set_state(U0)
    e32.erk_step(0.0, dt, 20)
    b = e32.get_state()
    err = rel(b, a)
    say("f32 vs f64 rel L2 =", err, "energy", H[0], H[-1])
    assert err < TOL32
    assert np.all(np.diff(H) <= 1e-12 * H[0])
    assert abs(e32.energy()[0] - H[-1]) < TOL32 * H[-1]


def test_3d_rejects_two_dimensional_calls():
    """Separable loads, the adjoint, the tabulated CFL step and the Ricker initial field are
    two-dimensional only: ARG on a three-dimensional context."""
    from paper_2505_15771_amd import Engine
    from paper_2505_15771_amd.hho import HHOError
    mesh, _ = MESHES["tets"]()
    e = Engine(mesh, 1)
    for call in (lambda: e.set_loads(np.zeros((1, e.n_dof)), [1.0], [0.0]),
                 lambda: e.adjoint(0.0, 1e-3, 2),
                 lambda: e.dt_cfl(0.5),
                 lambda: e.set_ricker_ic((0.5, 0.5), 0.1)):
        with pytest.raises(HHOError) as ex:
            call()
        assert ex.value.code == 1


@pytest.mark.parametrize("case,dtype", [("tets", "f64"), ("tets", "f32"), ("hexes-prisms", "f64")])
def test_3d_ricker_sources_and_receivers(case, dtype):
    """Two shots on 4^3 cubes (tetrahedra, or sheared hexahedron / prism columns), k = 2: shot 0 a
    Ricker point force in the solid, shot 1 a Ricker pressure source in the fluid; two receivers per
    medium recording p or (v_x, v_y, v_z) after every step; 60 steps from rest against the oracle
    driven by the same point loads."""
    from oracle.oracle3d import ricker
    from paper_2505_15771_amd import Engine
    mesh, n = MESHES[case]()
    k = 2
    say("case: 3d %s k=2 %s, Ricker sources in both media, 4 receivers, 60 steps" % (case, dtype))
    o = oracle3d(mesh, k, key=case)
    dt = dt_for(mesh, n, k)
    f0, t0, amp = 10.0, 0.12, 1.0
    src = [(np.array([0.41, 0.36, 0.29]), np.array([0.3, -0.2, 1.0])),
           (np.array([0.62, 0.53, 0.77]), np.array([1.0, 0.0, 0.0]))]
    rec = np.array([[0.31, 0.71, 0.74], [0.79, 0.22, 0.61], [0.28, 0.33, 0.21], [0.68, 0.57, 0.41]])
    fld = [0, 0, 1, 1]
    e = Engine(mesh, k, dtype=dtype, n_shots=2)
    for sh, (x, d) in enumerate(src):
        e.set_sources(sh, [x], [d], f0, t0, amp)
    e.set_receivers(rec, fld)
    e.erk_step(0.0, dt, 60)
    tol = TOL64 if dtype == "f64" else TOL32
    for sh, (x, d) in enumerate(src):
        F = o.point_load(x, d)
        traces = np.zeros((60, 4, 3))

        def record(step, U):
            for r in range(4):
                v = o.point_values(U, rec[r])
                traces[step, r, :len(v)] = v
        ref = o.erk(np.zeros(o.ndof), dt, 60, load=lambda t: amp * ricker(t, f0, t0) * F, record=record)
        err = rel(e.get_state(shot=sh), ref)
        terr = rel(e.traces(shot=sh), traces)
        say(dtype, "shot", sh, "state rel L2 =", err, "traces rel L2 =", terr)
        assert err < tol and terr < tol
