"""CPU tests of the library's host side and C ABI surface (no GPU needed).

* libhho.so loads and exports every symbol declared in include/*.h;
* the host plan (shape classes, class tables, links, coefficients) drives a NumPy
  model of the stage kernel that reproduces the FP64 oracle's semi-discrete operator
  (eq. ex_solve) on meshes with triangles, quads, hanging-node polygons and the
  fluid-solid interface;
* invalid meshes and parameters are rejected with the documented status codes.
"""
import os
import re

import numpy as np
import pytest

from synth import meshes as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_15771_amd import hho
    return hho.load_library()


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names.update(re.findall(r"^\s*(?:[A-Za-z_][\w \*]*?[\s\*])(hho_\w+)\s*\(", src, re.M))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "hho_setup" in names and "hho_erk_step" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_2505_15771_amd.hho import EXPORTS
    assert set(names) == set(EXPORTS)


CASES = {
    "quads_interface": lambda: M.with_materials(M.unit_square(6), perturb=0.1, seed=1),
    "hybrid_interface": lambda: M.with_materials(M.unit_square(6, p_split=0.5, seed=3), perturb=0.1, seed=2),
    "hanging_interface": lambda: M.hanging_square(6, seed=5),
    "perturbed_vertices": lambda: M.with_materials(M.perturbed_square(8, seed=6), perturb=0.1, seed=7),
    "hexagons": lambda: M.with_materials(M.honeycomb_bilayer(6), perturb=0.1, seed=8),
    "partly_perturbed": lambda: M.with_materials(M.perturbed_square(16, seed=9, x_max=0.5), perturb=0.1, seed=10),
}


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("case", list(CASES))
def test_plan_reproduces_oracle_operator(k, case):
    from oracle import Oracle
    from paper_2505_15771_amd import Inspect
    import kernel_model
    mesh = CASES[case]()
    ins = Inspect(mesh, k)
    o = Oracle(mesh, k)
    assert ins.n_faces == o.nfaces
    U = np.random.default_rng(k).standard_normal(o.ndof)
    got = kernel_model.rhs(ins, mesh, U)
    ref = o.rhs(U)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_small_classes_are_pooled():
    """On a mesh with more than 64 shape classes, cells whose shape occurs fewer than 32 times go
    to pooled groups (one per medium and face-count bucket) whose lanes find their own class
    tables; shapes that repeat keep groups of their own, and meshes with few classes (hanging
    nodes, cut cells) are not pooled.  With every vertex moved every group is pooled and the
    internal cells are padded per pooled group only."""
    from paper_2505_15771_amd import Inspect
    ins = Inspect(M.with_materials(M.perturbed_square(8, seed=2)), 2)
    assert ins.pooled.all() and ins.n_groups <= 4
    assert ins.n_ic <= ins.n_cells + ins.n_groups * 256
    tab_cells = {int(ins.ic_tab[ic]) for ic in ins.ic_of_cell}
    assert len(tab_cells) == ins.n_cells          # one table per cell
    part = Inspect(M.with_materials(M.perturbed_square(16, seed=2, x_max=0.5)), 2)
    assert part.pooled.any() and not part.pooled.all()
    shared = part.groups[part.pooled == 0]
    for tab in set(shared[:, 2]):                  # lattice shapes right of x = 1/2, both media
        assert shared[shared[:, 2] == tab, 4].sum() >= 32
    big = Inspect(M.with_materials(M.unit_square(16)), 2)
    assert not big.pooled.any()
    assert not Inspect(M.hanging_square(8, seed=3), 2).pooled.any()


def test_shape_classes_are_shared():
    from paper_2505_15771_amd import Inspect
    ins = Inspect(M.with_materials(M.unit_square(16, p_split=0.5, seed=1)), 2)
    # squares and the four half-square triangles, in each medium
    assert ins.n_groups <= 10
    assert ins.n_cells == int(np.sum(ins.groups[:, 4]))


def test_rejects_bad_input():
    from paper_2505_15771_amd import Inspect, HHOError
    mesh = M.with_materials(M.unit_square(3))
    with pytest.raises(HHOError) as e:
        Inspect(mesh, 4)
    assert e.value.code == 1
    bad = dict(mesh)
    vtx = bad["cell_vtx"].copy()
    s, t = bad["cell_ptr"][0], bad["cell_ptr"][1]
    vtx[s:t] = vtx[s:t][::-1]  # clockwise cell
    bad["cell_vtx"] = vtx
    with pytest.raises(HHOError) as e:
        Inspect(bad, 1)
    assert e.value.code == 2
    neg = dict(mesh)
    neg["rho"] = -np.asarray(mesh["rho"])
    with pytest.raises(HHOError) as e:
        Inspect(neg, 1)
    assert e.value.code == 1


@pytest.mark.parametrize("k", [1, 2, 3])
def test_plan_adjoint_operator(k):
    """The transpose of the condensed operator in the form the adjoint stage kernel computes it,
    L^T x = D R_c(D M^{-1} x) (D flips the dual unknowns, R_c reverses the interface coupling),
    built from the host plan, equals the oracle's explicitly transposed operator."""
    from oracle import Oracle
    from paper_2505_15771_amd import Inspect
    import kernel_model
    mesh = M.hanging_square(6, seed=5)
    ins = Inspect(mesh, k)
    o = Oracle(mesh, k)
    x = np.random.default_rng(k).standard_normal(o.ndof)
    got = kernel_model.rhs(ins, mesh, x, adjoint=True)
    ref = o.rhs_T(x)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("stab_speed", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_plan_gradient_terms(k, stab_speed):
    """The per-stage parameter derivatives in the form the adjoint stage kernel computes them
    (stored forward face values, adjoint face values of z, the plan's material-derivative
    coefficients) equal the oracle's gradient terms, on a mesh with hanging nodes and the
    fluid-solid interface, for both stabilisation speeds."""
    from oracle import Oracle
    from paper_2505_15771_amd import Inspect
    import kernel_model
    mesh = M.hanging_square(6, seed=5)
    ins = Inspect(mesh, k, stab_speed=stab_speed)
    o = Oracle(mesh, k, stab_speed=stab_speed)
    rng = np.random.default_rng(10 + k)
    Y, kk, mu = (rng.standard_normal(o.ndof) for _ in range(3))
    ref = np.zeros((o.nc, 3))
    o.grad_terms(Y, kk, mu, ref)
    got = kernel_model.grad_terms(ins, mesh, Y, kk, mu)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("s", [2, 3, 4])
def test_erk_increment_form_reproduces_tableau(s):
    """The stage combine as the kernel performs it (increments D_i, the partial sum Q, the last
    stage's combination), driven by the host's coefficients, applied to the linear system
    y' = A y: one step equals the Taylor polynomial sum_{j<=s} (dt A)^j / j! y (the stability
    polynomial of the tableaux of eq. ERK, all of order s), and the stage nodes are the tableau's."""
    from math import factorial
    from paper_2505_15771_amd.hho import erk_coefficients
    co = erk_coefficients(s)
    rng = np.random.default_rng(s)
    A = rng.standard_normal((5, 5))
    U = rng.standard_normal(5)
    dt = 0.1
    D_prev, Q = None, None
    for i in range(s):
        c, cY, ck, cb, qa, qb, cd, qw, qr = co[i]
        Y = U if i == 0 else U + D_prev
        k = A @ Y
        if i < s - 1:
            D = (cY * D_prev if i > 0 else 0.0) + ck * dt * k
            if qw:
                Q = qa * D_prev + qb * D
            D_prev = D
        else:
            Unew = U + ((Q if qr else 0.0) + cd * D_prev + cb * dt * k)
    ref = sum(np.linalg.matrix_power(dt * A, j) @ U / factorial(j) for j in range(s + 1))
    assert np.linalg.norm(Unew - ref) < 1e-14 * np.linalg.norm(ref)
    nodes = {2: [0, 0.5], 3: [0, 0.5, 1.0], 4: [0, 0.5, 0.5, 1.0]}[s]
    assert np.allclose(co[:, 0], nodes)


def _cfl_test_mesh(shape, k):
    n = {1: 5, 2: 4, 3: 3}[k]
    if shape in ("quads", "triangles", "hybrid"):
        return M.with_materials(M.bilayer_vertical(n, p_split={"quads": 0.0, "triangles": 1.0, "hybrid": 0.5}[shape],
                                                   seed=3))
    if shape == "hanging":
        return M.hanging_square(n + 1, seed=5, frac=0.35)
    if shape == "hexagons":
        return M.with_materials(M.honeycomb_bilayer(2 * n))
    return M.with_materials(M.perturbed_square(n + 1, seed=4))


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("shape", ["quads", "triangles", "hybrid", "hanging", "hexagons", "perturbed"])
def test_cfl_step_is_stable(k, shape):
    """hho_dt_cfl at factor 1 (eq. CFL with the CFL* of Table tab::ratio_geo, lowered where this
    discretisation's own limit is smaller) against the spectrum of the condensed operator L (the
    oracle's dense matrix): every eigenvalue lambda satisfies |R_s(dt lambda)| <= 1 for the
    amplification polynomial R_s(z) = sum_{j<=s} z^j / j! of ERK(s), s = 2, 3, 4, on squares,
    triangles, hybrid meshes, squares and triangles with hanging nodes, hexagons, and quads and
    triangles with moved vertices."""
    from math import factorial
    from oracle import Oracle
    from paper_2505_15771_amd import Inspect
    mesh = _cfl_test_mesh(shape, k)
    ins = Inspect(mesh, k)
    lam = np.linalg.eigvals(Oracle(mesh, k).dense_operator())
    assert np.max(lam.real) < 1e-10 * np.max(np.abs(lam))  # dissipative semi-discretisation
    for s_ in (2, 3, 4):
        z = ins.dt_cfl[s_] * lam
        R = sum(z ** j / factorial(j) for j in range(s_ + 1))
        assert np.max(np.abs(R)) <= 1.0 + 1e-12, (s_, float(np.max(np.abs(R))))
