"""Pins of the 3D oracle (oracle/oracle3d.py): the method of Sec. 3 written out for tetrahedra and
parallelepiped hexahedra, checked against what the mathematics fixes.

* unknown counts per cell and face, and the 3D face shares of Table tab::DOFS;
* the skew part of the assembled form cancels: X . A X equals the stabilisation energy
  sum eta tau_T |u_T - u_F|^2_F integrated separately (any cell and face values, both media,
  the fluid-solid interface), so the signs of every reconstruction and coupling term are fixed;
* polynomial consistency: for p in P^k and v in P^k(R^3) with face values their traces, the
  reconstruction rows return (grad p, r)_T and (grad_sym v, b)_T and the stabilisation vanishes;
  rigid motions give no stress;
* the face block is block-diagonal (one block per face: the condensation of eq. ex_solve is
  face-local), and its inverse gives the condensed operator;
* one ERK(s) step equals the Taylor polynomial of the dense operator; undriven energy does not grow;
* an acoustic standing wave in the unit cube converges at a rate near k + 1.
"""
import math

import numpy as np
import pytest

from oracle.oracle3d import FLUID, SOLID, SYM, Oracle3D, cube_mesh


def _stab_energy_by_quadrature(o, X):
    """sum over cells T and their faces F of eta tau_T |u_T - u_F|^2_F, u the primal fields
    (p in the fluid, v in the solid), boundary faces with u_F = 0."""
    nT, N, f = o.ndof, o.N, o.f
    e = 0.0
    for c in range(o.nc):
        et = o.tau(c)
        comps = [0] if o.medium[c] == FLUID else [0, 1, 2]
        for F in o.cell_faces[c]:
            XF, WF = o.face_quad(F)
            phi, _ = o.cell_basis(c, XF)
            psi = o.face_basis(F, XF)
            for comp in comps:
                uT = phi @ X[o.off[c] + comp * N: o.off[c] + (comp + 1) * N]
                if len(o.face_cells[F]) == 2:
                    base = nT + (o.fp[F] if o.medium[c] == FLUID else o.fv[F] + comp * f)
                    uF = psi @ X[base: base + f]
                else:
                    uF = 0.0
                e += et * float(np.sum(WF * (uT - uF) ** 2))
    return e


def test_dof_counts_and_face_shares():
    """N = (k+1)(k+2)(k+3)/6 cell and f = (k+1)(k+2)/2 face functions; 4 (fluid) and 9 (solid)
    fields per cell, 1 / 3 / 4 per fluid / solid / interface face.  With four faces per
    tetrahedron each shared by two cells, the face share of the unknowns is 3 / (2k + 9)
    (acoustic) and 2 / (k + 5) (elastic): 27 / 23 / 20 % and 33 / 29 / 25 % for k = 1, 2, 3, the
    3D rows of Table tab::DOFS; on a 6^3-cube tetrahedral mesh the share of interior faces
    approaches them from below."""
    table = {(1, FLUID): 0.27, (2, FLUID): 0.23, (3, FLUID): 0.20, (1, SOLID): 0.33, (2, SOLID): 0.29,
             (3, SOLID): 0.25}
    for k in (1, 2, 3):
        o = Oracle3D(cube_mesh(1, medium_of=lambda x, y, z: FLUID), k)
        N, f = (k + 1) * (k + 2) * (k + 3) // 6, (k + 1) * (k + 2) // 2
        assert (o.N, o.f) == (N, f)
        assert o.ndof == 6 * 4 * N
        for med, ncell, nface in ((FLUID, 4, 1), (SOLID, 9, 3)):
            share = 2 * nface * f / (2 * nface * f + ncell * N)
            assert share == pytest.approx(3 / (2 * k + 9) if med == FLUID else 2 / (k + 5), rel=1e-14)
            assert round(100 * share) == round(100 * table[(k, med)])
    o = Oracle3D(cube_mesh(6, medium_of=lambda x, y, z: FLUID), 1)
    share = o.nfdof / (o.nfdof + o.ndof)
    assert 0.20 < share < 3 / 11
    m = cube_mesh(2)
    o = Oracle3D(m, 1)
    itf = sum(1 for F, fc in enumerate(o.face_cells) if len(fc) == 2 and len({o.medium[c] for c in fc}) == 2)
    assert itf == 2 * 2 * 2 and o.nfdof == o.f * (o.fp >= 0).sum() + 3 * o.f * (o.fv >= 0).sum()


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("kind", ["tets", "hexes", "prisms"])
def test_skew_part_cancels(k, kind):
    """X . A X = stabilisation energy for random cell and face values, on a two-material mesh
    (solid below z = 1/2) with materials varying per cell."""
    m = cube_mesh(2, tets=kind == "tets", prisms=kind == "prisms")
    rng = np.random.default_rng(k)
    m["rho"] = m["rho"] * (1 + 0.2 * rng.random(len(m["rho"])))
    m["a"] = m["a"] * (1 + 0.2 * rng.random(len(m["a"])))
    m["b"] = m["b"] * (1 + 0.2 * rng.random(len(m["b"])))
    o = Oracle3D(m, k)
    X = rng.standard_normal(o.ndof + o.nfdof)
    lhs = float(X @ (o.A @ X))
    rhs = _stab_energy_by_quadrature(o, X)
    assert abs(lhs - rhs) < 1e-12 * rhs
    # at the condensed face values: U . K_eff U = stabilisation energy >= 0
    U = X[:o.ndof]
    assert abs(U @ o.keff(U) - o.stab_energy(U)) < 1e-12 * abs(U @ o.keff(U))


class _Poly:
    """Random polynomial of total degree <= k in (x, y, z) with its gradient."""

    def __init__(self, k, rng):
        self.e = [(a, b, c) for a in range(k + 1) for b in range(k + 1) for c in range(k + 1) if a + b + c <= k]
        self.w = rng.standard_normal(len(self.e))

    def __call__(self, x, y, z):
        return sum(w * x ** a * y ** b * z ** c for w, (a, b, c) in zip(self.w, self.e))

    def grad(self, x, y, z):
        g = [0 * x, 0 * x, 0 * x]
        for w, (a, b, c) in zip(self.w, self.e):
            if a:
                g[0] = g[0] + w * a * x ** (a - 1) * y ** b * z ** c
            if b:
                g[1] = g[1] + w * b * x ** a * y ** (b - 1) * z ** c
            if c:
                g[2] = g[2] + w * c * x ** a * y ** b * z ** (c - 1)
        return g


def _with_traces(o, U, fluid_fn, solid_fns):
    X = np.concatenate([U, np.zeros(o.nfdof)])
    for F, fc in enumerate(o.face_cells):
        if len(fc) < 2:
            continue
        if o.fp[F] >= 0:
            X[o.ndof + o.fp[F]: o.ndof + o.fp[F] + o.f] = o.face_project(F, fluid_fn)
        if o.fv[F] >= 0:
            for comp in range(3):
                X[o.ndof + o.fv[F] + comp * o.f: o.ndof + o.fv[F] + (comp + 1) * o.f] = o.face_project(F, solid_fns[comp])
    return X


@pytest.mark.parametrize("k,prisms", [(1, False), (2, False), (3, False), (2, True)])
def test_polynomial_consistency(k, prisms):
    """Interior cells only see polynomial traces: for p in P^k (fluid) and v in P^k(R^3) (solid)
    with face values their traces, the m rows of A X are -(grad p, r)_T and the s rows
    -(grad_sym v, b)_T for every interior cell, and the stabilisation energy of the interior
    faces vanishes; a rigid motion v = a + w x x gives zero s rows."""
    rng = np.random.default_rng(10 + k)
    p = _Poly(k, rng)
    vs = [_Poly(k, rng) for _ in range(3)]
    zero = lambda x, y, z: 0 * x
    for med in (FLUID, SOLID):
        o = Oracle3D(cube_mesh(3, medium_of=lambda x, y, z, m_=med: m_, prisms=prisms), k)
        U = o.project([p, zero, zero, zero], [vs[0], vs[1], vs[2]] + [zero] * 6)
        X = _with_traces(o, U, p, vs)
        R = o.A @ X
        N = o.N
        checked = 0
        for c in range(o.nc):
            if any(len(o.face_cells[F]) < 2 for F in o.cell_faces[c]):
                continue
            Xq, W = o.cell_quad(c, k + 3)
            phi, _ = o.cell_basis(c, Xq)
            x, y, z = Xq.T
            # m = 0 and s = 0 here, so the p and v rows hold only the stabilisation: zero
            prim = slice(o.off[c], o.off[c] + (N if med == FLUID else 3 * N))
            assert np.abs(R[prim]).max() < 1e-11 * (1 + np.abs(U[prim]).max())
            if med == FLUID:
                g = p.grad(x, y, z)
                for d in range(3):
                    ref = -(phi * W[:, None]).T @ g[d]
                    got = R[o.off[c] + (1 + d) * N: o.off[c] + (2 + d) * N]
                    assert np.abs(got - ref).max() < 1e-11 * (1 + np.abs(ref).max())
            else:
                G = [v.grad(x, y, z) for v in vs]
                for dd, (i, j) in enumerate(SYM):
                    e = G[i][i] if i == j else (G[i][j] + G[j][i]) / math.sqrt(2.0)
                    ref = -(phi * W[:, None]).T @ e
                    got = R[o.off[c] + (3 + dd) * N: o.off[c] + (4 + dd) * N]
                    assert np.abs(got - ref).max() < 1e-11 * (1 + np.abs(ref).max())
            checked += 1
        assert checked > 0
    # rigid motion a + w x x: grad_sym = 0 -> s rows vanish on interior cells
    o = Oracle3D(cube_mesh(3, medium_of=lambda x, y, z: SOLID), k)
    a, w = rng.standard_normal(3), rng.standard_normal(3)
    rig = [lambda x, y, z: a[0] + w[1] * z - w[2] * y, lambda x, y, z: a[1] + w[2] * x - w[0] * z,
           lambda x, y, z: a[2] + w[0] * y - w[1] * x]
    U = o.project([zero] * 4, rig + [zero] * 6)
    X = _with_traces(o, U, zero, rig)
    R = o.A @ X
    for c in range(o.nc):
        if all(len(o.face_cells[F]) == 2 for F in o.cell_faces[c]):
            assert np.abs(R[o.off[c] + 3 * o.N: o.off[c + 1]]).max() < 1e-11


def test_face_block_is_block_diagonal():
    """No face unknown couples to another face's unknowns (eq. ex_solve: K_F is block-diagonal),
    including the interface faces, where p_F and v_F couple to each other only."""
    o = Oracle3D(cube_mesh(2), 2)
    face_of = np.zeros(o.nfdof, int)
    for F in range(o.nfaces):
        if o.fp[F] >= 0:
            face_of[o.fp[F]: o.fp[F] + o.f] = F
        if o.fv[F] >= 0:
            face_of[o.fv[F]: o.fv[F] + 3 * o.f] = F
    C = o.AFF.tocoo()
    nz = np.abs(C.data) > 0
    assert np.all(face_of[C.row[nz]] == face_of[C.col[nz]])


@pytest.mark.parametrize("s", [2, 3, 4])
def test_erk_step_is_taylor_polynomial(s):
    from math import factorial
    o = Oracle3D(cube_mesh(1), 1)
    L = o.dense_operator()
    U = np.random.default_rng(s).standard_normal(o.ndof)
    dt = 0.01
    ref, term = U.copy(), U.copy()
    for j in range(1, s + 1):
        term = dt * L @ term
        ref = ref + term / factorial(j)
    got = o.erk(U, dt, 1, s=s)
    assert np.linalg.norm(got - ref) < 1e-13 * np.linalg.norm(ref)


def test_energy_does_not_grow():
    """Undriven two-material run at a step well inside the spectral limit: the energy decreases
    (the stabilisation dissipates, the rest is skew)."""
    o = Oracle3D(cube_mesh(2), 1)
    lam = np.linalg.eigvals(o.dense_operator())
    dt = 1.0 / np.abs(lam).max()
    U = np.random.default_rng(3).standard_normal(o.ndof)
    E = [o.energy(U)]
    for _ in range(10):
        U = o.erk(U, dt, 1)
        E.append(o.energy(U))
    assert all(E[i + 1] <= E[i] * (1 + 1e-14) for i in range(10))


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_acoustic_standing_wave_converges(k):
    """p = cos(w t) sin(pi x) sin(pi y) sin(pi z), m = sin(w t) grad(sin sin sin) / (rho w),
    w = sqrt(3) pi c, in the unit cube of acoustic medium (rho = 1, c = 1; p = 0 on the boundary):
    the energy-norm error of (p, m) at T = 0.2 decreases at a rate above k + 0.5 between 2^3 and
    4^3 cubes of six tetrahedra (measured 1.82 at k = 1, 3.10 at k = 2; 2.10 at k = 1 from 4^3 to
    8^3)."""
    w = math.sqrt(3.0) * math.pi
    S = lambda x, y, z: np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    dS = [lambda x, y, z: np.pi * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z),
          lambda x, y, z: np.pi * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z),
          lambda x, y, z: np.pi * np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z)]
    zero = lambda x, y, z: 0 * x

    def fields(t):
        return ([lambda x, y, z: np.cos(w * t) * S(x, y, z)] +
                [lambda x, y, z, d=d: np.sin(w * t) / w * dS[d](x, y, z) for d in range(3)], [zero] * 9)

    T = 0.2
    errs = []
    for n in (2, 4):
        o = Oracle3D(cube_mesh(n, medium_of=lambda x, y, z: FLUID), k)
        nsteps = 4 * n * k * (k + 1)
        U = o.erk(o.project(*fields(0.0)), T / nsteps, nsteps)
        ref = o.project(*fields(T))
        d = U - ref
        errs.append(math.sqrt(float(d @ (o.M @ d))))
    rate = math.log(errs[0] / errs[1], 2)
    assert rate > k + 0.5, (errs, rate)


# ------------------------------------------------------------------ point sources and receivers
def _poly_fields(k, rng):
    """Random polynomial fields of degree k: 4 fluid (p, m) and 9 solid (v, s) callables."""
    def one():
        cf = rng.standard_normal((k + 1, k + 1, k + 1))
        def f(x, y, z):
            out = np.zeros_like(x)
            for a in range(k + 1):
                for b in range(k + 1 - a):
                    for c in range(k + 1 - a - b):
                        out = out + cf[a, b, c] * x ** a * y ** b * z ** c
            return out
        return f
    return [one() for _ in range(4)], [one() for _ in range(9)]


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("kind", ["tets", "hexes", "prisms"])
def test_point_load_and_point_values_reproduce_polynomials(kind, k):
    """Point evaluation is exact on polynomial fields: for U the projection of fields of degree k,
    F . U = d . u(x) for the point-force load F, and the receiver values are u(x), in either medium."""
    o = Oracle3D(cube_mesh(2, tets=kind == "tets", prisms=kind == "prisms"), k)
    rng = np.random.default_rng(41)
    ff, sf = _poly_fields(k, rng)
    U = o.project(ff, sf)
    for x, expect_medium in (([0.31, 0.42, 0.23], SOLID), ([0.62, 0.27, 0.81], FLUID)):
        x = np.array(x)
        assert o.medium[o.locate(x)] == expect_medium
        d = rng.standard_normal(3)
        F = o.point_load(x, d)
        fields = ff if expect_medium == FLUID else sf
        u = np.array([f(*x[:, None])[0] for f in fields[:(1 if expect_medium == FLUID else 3)]])
        ref = d[0] * u[0] if expect_medium == FLUID else float(d @ u)
        assert abs(F @ U - ref) < 1e-11 * max(1.0, abs(ref))
        assert np.allclose(o.point_values(U, x), u, rtol=1e-11, atol=1e-11)


def test_forced_erk_is_fourth_order():
    """ERK(4) with a time-dependent load (a point force times sin(omega t)) against the exact solution
    of U' = L U + M^{-1} F(t), from the matrix exponential of the system augmented with the
    oscillator (a, b)' = (omega b, -omega a): the error falls by about 2^4 when dt halves."""
    from scipy.linalg import expm
    o = Oracle3D(cube_mesh(1, tets=True), 1)
    L = o.dense_operator()
    f = o.point_load(np.array([0.3, 0.6, 0.2]), np.array([0.2, -0.4, 1.0]))
    g = o._M_lu.solve(f)
    om = 9.0
    n = o.ndof
    Aug = np.zeros((n + 2, n + 2))
    Aug[:n, :n] = L
    Aug[:n, n] = g            # the load enters as sin(omega t) = a
    Aug[n, n + 1] = om        # a' = omega b
    Aug[n + 1, n] = -om       # b' = -omega a
    U0 = np.random.default_rng(42).standard_normal(n)
    T = 0.2
    exact = (expm(T * Aug) @ np.concatenate([U0, [0.0, 1.0]]))[:n]
    errs = []
    for steps in (20, 40):
        dt = T / steps
        U = o.erk(U0, dt, steps, load=lambda t: math.sin(om * t) * f)
        errs.append(np.linalg.norm(U - exact) / np.linalg.norm(exact))
    assert errs[0] / errs[1] > 12.0, errs


def test_ricker_time_factor_3d():
    """The Ricker factor of the 3D oracle: maximum 1 at t0, zeros at t0 +- 1/(sqrt 2 pi f0), zero
    time integral (trapezoidal rule on a fine grid)."""
    from oracle.oracle3d import ricker
    f0, t0 = 10.0, 0.12
    assert ricker(t0, f0, t0) == 1.0
    tz = 1.0 / (math.sqrt(2.0) * math.pi * f0)
    assert abs(ricker(t0 + tz, f0, t0)) < 1e-15 and abs(ricker(t0 - tz, f0, t0)) < 1e-15
    t = np.linspace(t0 - 1.0, t0 + 1.0, 200001)
    r = np.array([ricker(x, f0, t0) for x in t])
    assert abs(np.trapezoid(r, t)) < 1e-9 and r.max() <= 1.0
