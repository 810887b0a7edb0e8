"""Pins of the SDIRK oracle (oracle/implicit.py): the implicit time stepping of Sec. 4.1 over the
mixed-order (k' = k + 1, Lehrenfeld-Schoberl) and equal-order HHO operators of Sec. 3.3.

Each pin ties the oracle to something other than itself: the independent explicit-path oracle
(equal order), polynomial consistency of the reconstructions, the skew-plus-dissipative structure
of the operator, the order conditions of the tableaux, the stability function of the scheme, and
convergence to an exact standing wave.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from oracle.implicit import (ImplicitOracle, sdirk_tableau, printed_sdirk2_tableau, domain_diameter,
                             FLUID, SOLID)
import synth.meshes as M


def _coupled(n=3, seed=11, refine=True):
    ref = None
    if refine:
        ref = np.zeros((n, n), bool)
        ref[0, 1] = True
    m = M.unit_square(n, p_split=0.5, seed=seed, refine=ref)
    return M.with_materials(m, perturb=0.1, seed=seed + 1)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("stab_speed", [0, 1])
def test_equal_order_matches_explicit_oracle(k, stab_speed):
    """With k' = k and alpha = 0 the assembled operator, condensed by a dense Schur complement,
    equals the explicit-path oracle's condensed operator (its own quadrature of the same forms,
    face by face condensation): two independent writings of eq. HHO1 / HHO2."""
    m = _coupled()
    io = ImplicitOracle(m, k, mixed=False, alpha=0, eta_f=0.8, eta_s=1.5, stab_speed=stab_speed)
    ref = Oracle(m, k, 0.8, 1.5, stab_speed).dense_operator()
    L = io.dense_operator()
    assert np.abs(L - ref).max() <= 1e-10 * np.abs(ref).max()


def _interior_cells(io):
    tag = io.ftag
    out = []
    for c in range(io.nc):
        faces = io.geo.cell_ops(c)["faces"]
        if all(tag[f] not in (3, 4) for f in faces):
            out.append(c)
    return out


def _face_projection(io, f, fn):
    fx, fy, fw = io._face_quad(f)
    psi = io._face_basis(f, fx, fy)
    return (psi * fw) @ fn(fx, fy)


@pytest.mark.parametrize("k", [1, 2])
def test_mixed_order_polynomial_consistency_fluid(k):
    """For a polynomial p of degree k + 1 with face values Pi^k_F p: the stabilisation of
    Lehrenfeld-Schoberl vanishes (p rows and face rows of K X are zero when m = 0) and
    -b_T(p; r) = -(grad p, r)_T on every cell away from the Dirichlet boundary."""
    m = M.with_materials(M.single_medium(4, M.FLUID, p_split=0.5, seed=5), perturb=0.1, seed=6)
    io = ImplicitOracle(m, k, mixed=True, alpha=1)
    rng = np.random.default_rng(7)
    cf = rng.standard_normal((k + 2, k + 2))
    p = lambda x, y: sum(cf[a, b] * x ** a * y ** b for a in range(k + 2) for b in range(k + 2 - a))
    px = lambda x, y: sum(a * cf[a, b] * x ** (a - 1) * y ** b for a in range(1, k + 2) for b in range(k + 2 - a))
    py = lambda x, y: sum(b * cf[a, b] * x ** a * y ** (b - 1) for a in range(k + 2) for b in range(1, k + 2 - a))
    z = lambda x, y: 0 * x
    X = np.zeros(io.ntot)
    X[:io.ndof] = io.project([p, z, z], [z] * 5)
    for f in range(len(io.ftag)):
        if io.ftag[f] in (3, 4):
            continue
        X[io.foff[f]:io.foff[f] + io.nf] = _face_projection(io, f, p)
    KX = io.K @ X
    G = io.project([z, px, py], [z] * 5)          # (d_c p, phi_a)_T in the orthonormal basis
    Np, N = io.Np, io.N
    for c in _interior_cells(io):
        o = io.off[c]
        assert np.abs(KX[o:o + Np]).max() < 1e-11
        np.testing.assert_allclose(KX[o + Np:o + Np + 2 * N], -G[o + Np:o + Np + 2 * N], atol=1e-11)
    interior_faces = [f for f in range(len(io.ftag))
                      if io.ftag[f] == 0 and all(io.fc[f, s] in set(_interior_cells(io)) for s in range(2))]
    for f in interior_faces:
        assert np.abs(KX[io.foff[f]:io.foff[f] + io.nf]).max() < 1e-11


@pytest.mark.parametrize("k", [1, 2])
def test_mixed_order_polynomial_consistency_solid(k):
    """Solid: for v of degree k + 1 (componentwise) with face values Pi^k_F v and s = 0, the v rows
    and face rows vanish and -h_T(v; b) = -(grad_sym v, b)_T on interior cells; a rigid motion
    gives zero on every row of interior cells."""
    m = M.with_materials(M.single_medium(4, M.SOLID, p_split=0.5, seed=8), perturb=0.1, seed=9)
    io = ImplicitOracle(m, k, mixed=True, alpha=1)
    rng = np.random.default_rng(10)
    cx, cy = rng.standard_normal((2, k + 2, k + 2))
    poly = lambda cf: (lambda x, y: sum(cf[a, b] * x ** a * y ** b for a in range(k + 2) for b in range(k + 2 - a)))
    dx = lambda cf: (lambda x, y: sum(a * cf[a, b] * x ** (a - 1) * y ** b for a in range(1, k + 2) for b in range(k + 2 - a)))
    dy = lambda cf: (lambda x, y: sum(b * cf[a, b] * x ** a * y ** (b - 1) for a in range(k + 2) for b in range(1, k + 2 - a)))
    z = lambda x, y: 0 * x
    r2 = 1.0 / math.sqrt(2.0)
    cases = [(poly(cx), poly(cy), dx(cx), dy(cy), lambda x, y: r2 * (dy(cx)(x, y) + dx(cy)(x, y))),
             (lambda x, y: 0.3 - 0.7 * y, lambda x, y: -0.2 + 0.7 * x, z, z, z)]   # rigid motion
    Np, N = io.Np, io.N
    for vx, vy, exx, eyy, exy in cases:
        X = np.zeros(io.ntot)
        X[:io.ndof] = io.project([z] * 3, [vx, vy, z, z, z])
        for f in range(len(io.ftag)):
            if io.ftag[f] in (3, 4):
                continue
            X[io.foff[f]:io.foff[f] + io.nf] = _face_projection(io, f, vx)
            X[io.foff[f] + io.nf:io.foff[f] + 2 * io.nf] = _face_projection(io, f, vy)
        KX = io.K @ X
        G = io.project([z] * 3, [z, z, exx, eyy, exy])
        for c in _interior_cells(io):
            o = io.off[c]
            assert np.abs(KX[o:o + 2 * Np]).max() < 1e-11
            np.testing.assert_allclose(KX[o + 2 * Np:o + 2 * Np + 3 * N], -G[o + 2 * Np:o + 2 * Np + 3 * N],
                                       atol=1e-11)


@pytest.mark.parametrize("mixed", [True, False])
def test_operator_is_skew_plus_dissipation(mixed):
    """K + K^T is the (symmetric positive semi-definite) stabilisation: it has no entries on the
    dual unknowns, and the gradient, coupling and interface blocks cancel in it."""
    m = _coupled()
    io = ImplicitOracle(m, 1, mixed=mixed, alpha=1)
    K = io.K.toarray()
    Sy = K + K.T
    dual = np.zeros(io.ntot, bool)
    for c in range(io.nc):
        o = io.off[c]
        if io.medium[c] == FLUID:
            dual[o + io.Np:o + io.Np + 2 * io.N] = True
        else:
            dual[o + 2 * io.Np:o + 2 * io.Np + 3 * io.N] = True
    assert np.abs(Sy[dual]).max() < 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(Sy)
    assert ev.min() > -1e-11 * ev.max() and ev.max() > 0
    assert np.abs(K - K.T).max() > 1e-2 * np.abs(K).max()    # a genuine skew part remains


def _order_conditions(A, b, c):
    e = np.ones(len(b))
    return {
        1: [b @ e - 1],
        2: [b @ c - 0.5],
        3: [b @ c ** 2 - 1 / 3, b @ A @ c - 1 / 6],
        4: [b @ c ** 3 - 1 / 4, b @ (c * (A @ c)) - 1 / 8, b @ A @ c ** 2 - 1 / 12, b @ A @ A @ c - 1 / 24],
    }


@pytest.mark.parametrize("s", [1, 2, 3])
def test_sdirk_tableaux_order_and_stability(s):
    """SDIRK(s, s+1): singly diagonal, c = A 1, order conditions up to order s + 1 (and not
    beyond), algebraically stable (b >= 0 and b_i a_ij + b_j a_ji - b_i b_j positive
    semi-definite), hence A-stable."""
    A, b, c = sdirk_tableau(s)
    assert np.allclose(np.diag(A), A[0, 0]) and np.allclose(np.triu(A, 1), 0)
    assert np.allclose(A.sum(axis=1), c)
    oc = _order_conditions(A, b, c)
    for p in range(1, s + 2):
        assert np.abs(oc[p]).max() < 1e-14, (p, oc[p])
    if s + 2 <= 4:
        assert np.abs(oc[s + 2]).max() > 1e-3
    Mm = b[:, None] * A + (b[:, None] * A).T - np.outer(b, b)
    assert (b >= 0).all() and np.linalg.eigvalsh(Mm).min() > -1e-14
    for y in np.logspace(-2, 3, 50):
        z = 1j * y
        R = 1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))
        assert abs(R) <= 1 + 1e-13


def test_printed_two_stage_tableau_is_second_order_only():
    """Reading of eq. SDIRK: the two-stage tableau as printed (a* = 1/4) meets the order 1 and 2
    conditions but not the order 3 ones; the oracle's SDIRK(2,3) uses a* = (3 + sqrt 3)/6."""
    A, b, c = printed_sdirk2_tableau()
    oc = _order_conditions(A, b, c)
    assert max(abs(x) for x in oc[1] + oc[2]) < 1e-15
    assert abs(oc[3][0]) > 1e-2


def _stability_matrix_function(L, dt, A, b):
    """R(dt L) with R(z) = P(z) / (1 - a* z)^s, P the numerator polynomial fitted exactly at
    s + 1 points from R(z) = 1 + z b^T (I - z A)^{-1} 1."""
    s = len(b)
    ast = A[0, 0]
    zs = -np.arange(1, s + 2, dtype=float)
    Rz = [1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s)) for z in zs]
    Pz = [r * (1 - ast * z) ** s for r, z in zip(Rz, zs)]
    coef = np.linalg.solve(np.vander(zs, s + 1, increasing=True), Pz)
    Z = dt * L
    n = len(L)
    P = np.zeros_like(Z)
    Zp = np.eye(n)
    for q in range(s + 1):
        P += coef[q] * Zp
        Zp = Zp @ Z
    Q = np.linalg.matrix_power(np.eye(n) - ast * Z, s)
    return np.linalg.solve(Q, P)


@pytest.mark.parametrize("s", [1, 2, 3])
@pytest.mark.parametrize("mixed", [True, False])
def test_sdirk_step_equals_stability_function(s, mixed):
    """One SDIRK step of the uncondensed stage systems equals R(dt L) U with L the densely
    condensed operator and R the scheme's stability function (no sources)."""
    m = _coupled(n=2, seed=21, refine=False)
    io = ImplicitOracle(m, 1, mixed=mixed, alpha=1)
    L = io.dense_operator()
    rng = np.random.default_rng(s)
    U0 = rng.standard_normal(io.ndof)
    dt = 0.05
    U1 = io.sdirk(U0, 0.0, dt, 1, s=s)
    A, b, _ = sdirk_tableau(s)
    ref = _stability_matrix_function(L, dt, A, b) @ U0
    assert np.linalg.norm(U1 - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_energy_never_grows_at_large_steps(s):
    """Algebraically stable scheme over a dissipative operator: the energy cannot grow, at a step
    many times the explicit stability limit, and it decays."""
    m = _coupled(n=4, seed=31)
    io = ImplicitOracle(m, 1, mixed=True, alpha=1)
    rng = np.random.default_rng(32)
    U0 = rng.standard_normal(io.ndof)
    _, E = io.sdirk(U0, 0.0, 0.2, 12, s=s, energies=True)
    E = np.concatenate([[io.energy(U0)], E])
    assert (np.diff(E) <= 1e-13 * E[:-1]).all()
    assert E[-1] < 0.9 * E[0]


@pytest.mark.parametrize("k", [1, 2])
def test_mixed_order_standing_wave_convergence(k):
    """One medium (acoustic, triangles), the standing wave p = cos(sqrt2 pi t) sin(pi x) sin(pi y)
    from its projection, SDIRK(3,4) with a time step small enough for the spatial error to
    dominate: the energy-norm error of the cell unknowns at T = 0.25 falls at rate >= k + 0.7."""
    w = math.sqrt(2.0) * math.pi
    def fields(t):
        a, b = math.cos(w * t), math.sin(w * t) / w * math.pi
        fl = [lambda x, y: a * np.sin(np.pi * x) * np.sin(np.pi * y),
              lambda x, y: b * np.cos(np.pi * x) * np.sin(np.pi * y),
              lambda x, y: b * np.sin(np.pi * x) * np.cos(np.pi * y)]
        return fl, [lambda x, y: 0 * x] * 5
    errs = []
    for n in (4, 8, 16):
        io = ImplicitOracle(M.with_materials(M.single_medium(n, M.FLUID, p_split=1.0, seed=2)), k)
        U0 = io.project(*fields(0.0))
        T = 0.25
        ns = 2 * n
        U = io.sdirk(U0, 0.0, T / ns, ns, s=3)
        Ue = io.project(*fields(T))
        errs.append(math.sqrt(io.mass_dot(U - Ue, U - Ue) / io.mass_dot(Ue, Ue)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 0.7, (errs, rates)   # measured 2.09 (k = 1), 3.12 (k = 2)


def test_domain_diameter():
    """l_Omega = diam(Omega): sqrt(2) for the unit square, sqrt(5) for the (-1, 1) x (0, 1)
    bilayer, whatever the cell shapes."""
    assert abs(domain_diameter(M.unit_square(3, p_split=0.5, seed=1)) - math.sqrt(2)) < 1e-15
    assert abs(domain_diameter(M.bilayer_vertical(2, p_split=0.5, seed=1)) - math.sqrt(5)) < 1e-15
