"""Plain float64 oracle of the HHO elasto-acoustic semi-discretisation in three dimensions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper states its method for d = 2 and
3 (Sec. 2-3; Table tab::DOFS counts the 3D unknowns) and names 3D as the next step (Sec. 6).
This module writes the same method out for tetrahedra, triangular prisms with parallelogram sides
and parallelepiped hexahedra, as plainly as possible: every local form of eq. HHO1 / HHO2 with the
reconstructions eq. rec_a / rec_e and the least-squares stabilisation eq. stab is integrated by
quadrature and assembled into one global sparse matrix on the cell and face unknowns; the face
unknowns are eliminated as in eq. ex_solve (their block is block-diagonal, one block per face),
and the explicit Runge-Kutta tableaux of eq. ERK advance the cell unknowns.

Readings (the same as the 2D oracle's):
  * the weak-form signs of eq. HHO1 / HHO2;
  * tau^f = eta^f / (rho c) and tau^s = eta^s rho c_S (0.8 and 1.5), least squares (alpha = 0);
  * homogeneous Dirichlet boundary faces carry no unknowns but enter the stabilisation;
  * n_Gamma points from the solid into the fluid;
  * compliance of d-dimensional isotropic elasticity, C^{-1} s = (s - lambda / (3 lambda + 2 mu)
    tr(s) I) / (2 mu); symmetric tensors in the Frobenius-orthonormal basis e_i e_i (i = 1..3),
    (e_i e_j + e_j e_i) / sqrt 2 (ij = 12, 13, 23).

Unknowns.  Cell basis: the scaled monomials of degree <= k in (x - x_T) / h_T, orthonormalised
in L2(T) by the inverse Cholesky factor of their Gram matrix (N = (k+1)(k+2)(k+3)/6 functions).
Face basis: the scaled monomials of degree <= k in the coordinates of a face frame fixed by the
face's global vertex ids (so both cells see one basis), orthonormalised in L2(F)
(f = (k+1)(k+2)/2 functions).  Cell layout: fluid [p | m_x | m_y | m_z], solid
[v_x | v_y | v_z | s_1 .. s_6], N values each.  Face unknowns: p_F (fluid faces), v_F (x, y, z;
solid faces), both on interface faces.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FLUID, SOLID = 0, 1
R2 = 1.0 / math.sqrt(2.0)
# symmetric-tensor basis: index pairs (i, j) of E_1 .. E_6
SYM = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))

TET_FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
# hexahedron: vertices 0-3 counter-clockwise at the bottom, 4-7 above them
HEX_FACES = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))
HEX_TETS = ((0, 1, 2, 6), (0, 2, 3, 6), (0, 3, 7, 6), (0, 7, 4, 6), (0, 4, 5, 6), (0, 5, 1, 6))
# triangular prism: vertices 0-2 around the bottom triangle, 3-5 above them (parallelogram sides)
PRISM_FACES = ((0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5))
PRISM_TETS = ((0, 1, 2, 3), (1, 2, 3, 4), (2, 3, 4, 5))
LOCAL_FACES = {4: TET_FACES, 6: PRISM_FACES, 8: HEX_FACES}
CELL_TETS = {6: PRISM_TETS, 8: HEX_TETS}


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def exponents(k, dim):
    """Graded exponents of the monomials of degree <= k in dim variables."""
    out = []
    for d in range(k + 1):
        if dim == 2:
            out += [(a, d - a) for a in range(d, -1, -1)]
        else:
            for a in range(d, -1, -1):
                out += [(a, b, d - a - b) for b in range(d - a, -1, -1)]
    return np.array(out)


def tet_rule(P, n):
    """Conical-product rule on the tetrahedron with vertices P[0..3]: exact to degree 2n - 3."""
    x, w = gauss01(n)
    a = x[:, None, None]
    b = (1 - a) * x[None, :, None]
    c = (1 - a) * (1 - x[None, :, None]) * x[None, None, :]
    jac = (1 - a) ** 2 * (1 - x[None, :, None])
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :] * jac).reshape(-1)
    a, b, c = (np.broadcast_to(t, (n, n, n)).reshape(-1) for t in (a, b, c))
    D = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)
    X = P[0][None, :] + np.stack([a, b, c], axis=1) @ D.T
    return X, W * abs(np.linalg.det(D))


def tri_rule(P, n):
    x, w = gauss01(n)
    a = x[:, None]
    b = (1 - a) * x[None, :]
    W = (w[:, None] * w[None, :] * (1 - a)).reshape(-1)
    a, b = (np.broadcast_to(t, (n, n)).reshape(-1) for t in (a, b))
    X = P[0][None, :] + a[:, None] * (P[1] - P[0])[None, :] + b[:, None] * (P[2] - P[0])[None, :]
    return X, W * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))


def quad_rule(P, n):
    """Parallelogram P[0], P[1], P[2] = P[1] + P[3] - P[0], P[3]."""
    x, w = gauss01(n)
    s, t = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w).reshape(-1)
    X = P[0][None, :] + s.reshape(-1)[:, None] * (P[1] - P[0])[None, :] + t.reshape(-1)[:, None] * (P[3] - P[0])[None, :]
    return X, W * np.linalg.norm(np.cross(P[1] - P[0], P[3] - P[0]))


def _orthonormal(V, W):
    """Coefficients C (lower) with phi = C m orthonormal in the weighted inner product of the
    monomial values V [q, n]: C = L^{-1}, G = L L^T the Gram matrix."""
    G = (V * W[:, None]).T @ V
    L = np.linalg.cholesky(G)
    return np.linalg.inv(L)


class Oracle3D:
    """mesh: dict with xyz [n_vertices, 3], cells (list of vertex-id tuples: 4 = tetrahedron,
    6 = triangular prism, 8 = parallelepiped hexahedron), medium [n_cells], rho, a (fluid c, solid
    lambda), b (solid mu)."""

    def __init__(self, mesh, k, eta_f=0.8, eta_s=1.5):
        self.k = k
        self.xyz = np.asarray(mesh["xyz"], float)
        self.cells = [tuple(int(v) for v in c) for c in mesh["cells"]]
        self.medium = np.asarray(mesh["medium"], int)
        self.rho = np.asarray(mesh["rho"], float)
        self.pa = np.asarray(mesh["a"], float)
        self.pb = np.asarray(mesh["b"], float)
        self.eta_f, self.eta_s = eta_f, eta_s
        self.nc = len(self.cells)
        self.ec = exponents(k, 3)
        self.ef = exponents(k, 2)
        self.N, self.f = len(self.ec), len(self.ef)
        self.nq_cell = k + 3
        self.nq_face = k + 2
        self._faces()
        self._geometry()
        self._offsets()
        self._assemble()

    # ------------------------------------------------------------------ topology and geometry
    def _faces(self):
        keys = {}
        self.cell_faces = []
        for c, vs in enumerate(self.cells):
            loc = LOCAL_FACES[len(vs)]
            fl = []
            for lf in loc:
                fv = tuple(vs[i] for i in lf)
                key = tuple(sorted(fv))
                if key not in keys:
                    keys[key] = len(keys)
                    self._fverts = getattr(self, "_fverts", []) + [fv]
                fl.append(keys[key])
            self.cell_faces.append(fl)
        self.nfaces = len(keys)
        self.face_cells = [[] for _ in range(self.nfaces)]
        for c, fl in enumerate(self.cell_faces):
            for F in fl:
                self.face_cells[F].append(c)
        if any(len(fc) > 2 for fc in self.face_cells):
            raise ValueError("a face is shared by more than two cells")

    def _cell_tets(self, c):
        vs = self.cells[c]
        P = self.xyz[list(vs)]
        return [P] if len(vs) == 4 else [P[list(t)] for t in CELL_TETS[len(vs)]]

    def cell_quad(self, c, n=None):
        n = n or self.nq_cell
        X, W = zip(*[tet_rule(T, n) for T in self._cell_tets(c)])
        return np.concatenate(X), np.concatenate(W)

    def face_quad(self, F, n=None):
        n = n or self.nq_face
        P = self.xyz[list(self._fverts[F])]
        return tri_rule(P, n) if len(P) == 3 else quad_rule(P, n)

    def _geometry(self):
        self.vol = np.zeros(self.nc)
        self.bary = np.zeros((self.nc, 3))
        self.hT = np.zeros(self.nc)
        for c in range(self.nc):
            X, W = self.cell_quad(c, 2)
            self.vol[c] = W.sum()
            self.bary[c] = (W[:, None] * X).sum(0) / W.sum()
            P = self.xyz[list(self.cells[c])]
            self.hT[c] = max(np.linalg.norm(p - q) for p in P for q in P)
        # face frames from the global vertex ids: origin and tangents from the lowest ids
        self.fcent = np.zeros((self.nfaces, 3))
        self.farea = np.zeros(self.nfaces)
        self.fnorm = np.zeros((self.nfaces, 3))
        self.ft = np.zeros((self.nfaces, 2, 3))
        self.fh = np.zeros(self.nfaces)
        for F in range(self.nfaces):
            X, W = self.face_quad(F, 2)
            self.farea[F] = W.sum()
            self.fcent[F] = (W[:, None] * X).sum(0) / W.sum()
            ids = sorted(self._fverts[F])
            a, b, cc = self.xyz[ids[0]], self.xyz[ids[1]], self.xyz[ids[2]]
            n = np.cross(b - a, cc - a)
            n /= np.linalg.norm(n)
            t1 = (b - a) / np.linalg.norm(b - a)
            self.fnorm[F] = n
            self.ft[F] = (t1, np.cross(n, t1))
            P = self.xyz[list(self._fverts[F])]
            self.fh[F] = max(np.linalg.norm(p - q) for p in P for q in P)
        # orthonormalisation of the cell and face bases
        self.cC = [None] * self.nc
        for c in range(self.nc):
            X, W = self.cell_quad(c)
            self.cC[c] = _orthonormal(self._cmono(c, X), W)
        self.fC = [None] * self.nfaces
        for F in range(self.nfaces):
            X, W = self.face_quad(F)
            self.fC[F] = _orthonormal(self._fmono(F, X), W)

    def _cmono(self, c, X):
        Y = (X - self.bary[c]) / self.hT[c]
        e = self.ec
        return Y[:, 0:1] ** e[:, 0] * Y[:, 1:2] ** e[:, 1] * Y[:, 2:3] ** e[:, 2]

    def _cmono_grad(self, c, X):
        Y = (X - self.bary[c]) / self.hT[c]
        e = self.ec
        g = []
        for d in range(3):
            ed = e.copy()
            coef = ed[:, d].astype(float)
            ed[:, d] = np.maximum(ed[:, d] - 1, 0)
            g.append(coef * Y[:, 0:1] ** ed[:, 0] * Y[:, 1:2] ** ed[:, 1] * Y[:, 2:3] ** ed[:, 2] / self.hT[c])
        return np.stack(g)  # [3, q, N]

    def _fmono(self, F, X):
        Y = X - self.fcent[F]
        s = (Y @ self.ft[F, 0]) / self.fh[F]
        t = (Y @ self.ft[F, 1]) / self.fh[F]
        e = self.ef
        return s[:, None] ** e[:, 0] * t[:, None] ** e[:, 1]

    def cell_basis(self, c, X):
        """Values [q, N] and gradients [3, q, N] of cell c's basis at points X [q, 3]."""
        C = self.cC[c]
        return self._cmono(c, X) @ C.T, self._cmono_grad(c, X) @ C.T

    def face_basis(self, F, X):
        return self._fmono(F, X) @ self.fC[F].T

    # ------------------------------------------------------------------ unknowns
    def ncomp(self, c):
        return 4 if self.medium[c] == FLUID else 9

    def _offsets(self):
        N, f = self.N, self.f
        self.off = np.zeros(self.nc + 1, int)
        for c in range(self.nc):
            self.off[c + 1] = self.off[c] + self.ncomp(c) * N
        self.ndof = int(self.off[-1])
        # face unknowns: p_F on faces touching a fluid cell, v_F on faces touching a solid cell
        # (interior faces only)
        self.fp = -np.ones(self.nfaces, int)
        self.fv = -np.ones(self.nfaces, int)
        nfd = 0
        for F, fc in enumerate(self.face_cells):
            if len(fc) < 2:
                continue
            if any(self.medium[c] == FLUID for c in fc):
                self.fp[F] = nfd
                nfd += f
            if any(self.medium[c] == SOLID for c in fc):
                self.fv[F] = nfd
                nfd += 3 * f
        self.nfdof = nfd

    def tau(self, c):
        """eta tau_T: fluid eta^f / (rho c), solid eta^s rho c_S."""
        if self.medium[c] == FLUID:
            return self.eta_f / (self.rho[c] * self.pa[c])
        return self.eta_s * self.rho[c] * math.sqrt(self.pb[c] / self.rho[c])

    def compliance(self, c):
        """C^{-1} in the symmetric-tensor basis (6 x 6)."""
        lam, mu = self.pa[c], self.pb[c]
        A = np.zeros((6, 6))
        t = lam / (3 * lam + 2 * mu)
        for i in range(3):
            for j in range(3):
                A[i, j] = ((1.0 if i == j else 0.0) - t) / (2 * mu)
        for i in range(3, 6):
            A[i, i] = 1.0 / (2 * mu)
        return A

    # ------------------------------------------------------------------ assembly
    def _assemble(self):
        N, f = self.N, self.f
        nT = self.ndof
        rows, cols, vals = [], [], []
        mrows, mcols, mvals = [], [], []

        def put(r, c, B):
            rr, cc = np.meshgrid(r, c, indexing="ij")
            rows.append(rr.reshape(-1))
            cols.append(cc.reshape(-1))
            vals.append(np.asarray(B).reshape(-1))

        def T(c, comp):  # cell unknowns of component comp
            return self.off[c] + comp * N + np.arange(N)

        def FP(F):
            return nT + self.fp[F] + np.arange(f)

        def FV(F, comp):
            return nT + self.fv[F] + comp * f + np.arange(f)

        for c in range(self.nc):
            X, W = self.cell_quad(c)
            phi, dphi = self.cell_basis(c, X)
            M0 = (phi * W[:, None]).T @ phi
            # D[d][a, b] = (d_d phi_b, phi_a)_T
            D = [(phi * W[:, None]).T @ dphi[d] for d in range(3)]
            et = self.tau(c)
            if self.medium[c] == FLUID:
                kap = self.rho[c] * self.pa[c] ** 2
                for i, blk in enumerate([M0 / kap] + [self.rho[c] * M0] * 3):
                    rr, cc = np.meshgrid(T(c, i), T(c, i), indexing="ij")
                    mrows.append(rr.reshape(-1)); mcols.append(cc.reshape(-1)); mvals.append(blk.reshape(-1))
                for d in range(3):
                    put(T(c, 1 + d), T(c, 0), -D[d])        # m rows: -(grad p_T, r)
                    put(T(c, 0), T(c, 1 + d), D[d].T)       # p rows: (grad q, m)
            else:
                for i in range(3):
                    rr, cc = np.meshgrid(T(c, i), T(c, i), indexing="ij")
                    mrows.append(rr.reshape(-1)); mcols.append(cc.reshape(-1)); mvals.append((self.rho[c] * M0).reshape(-1))
                A = self.compliance(c)
                for i in range(6):
                    for j in range(6):
                        if A[i, j] != 0.0:
                            rr, cc = np.meshgrid(T(c, 3 + i), T(c, 3 + j), indexing="ij")
                            mrows.append(rr.reshape(-1)); mcols.append(cc.reshape(-1))
                            mvals.append((A[i, j] * M0).reshape(-1))
                # (grad_sym (phi e_comp) : E_d, phi) as -(...) in the s rows and +(...)^T in the v rows
                for dd, (i, j) in enumerate(SYM):
                    for comp in range(3):
                        G = np.zeros((N, N))
                        if i == j:
                            if comp == i:
                                G = D[i]
                        else:
                            if comp == i:
                                G = G + R2 * D[j]
                            if comp == j:
                                G = G + R2 * D[i]
                        if np.any(G):
                            put(T(c, 3 + dd), T(c, comp), -G)
                            put(T(c, comp), T(c, 3 + dd), G.T)
            # faces of the cell
            for F in self.cell_faces[c]:
                XF, WF = self.face_quad(F)
                phiF, _ = self.cell_basis(c, XF)
                psi = self.face_basis(F, XF)
                n = self.fnorm[F] * (1.0 if np.dot(self.fcent[F] - self.bary[c], self.fnorm[F]) > 0 else -1.0)
                E = (phiF * WF[:, None]).T @ phiF      # (phi_b, phi_a)_F
                G = (phiF * WF[:, None]).T @ psi       # (phi_a, psi_b)_F  [N, f]
                MF = (psi * WF[:, None]).T @ psi
                interior = len(self.face_cells[F]) == 2
                if self.medium[c] == FLUID:
                    for d in range(3):
                        put(T(c, 1 + d), T(c, 0), n[d] * E)       # m rows: +(p_T, r.n)
                        put(T(c, 0), T(c, 1 + d), -n[d] * E)      # p rows: -(q, m.n)
                    put(T(c, 0), T(c, 0), et * E)                 # stabilisation
                    if interior:
                        for d in range(3):
                            put(T(c, 1 + d), FP(F), -n[d] * G)    # m rows: -(p_F, r.n)
                            put(FP(F), T(c, 1 + d), n[d] * G.T)   # face rows: (q_F, m.n)
                        put(T(c, 0), FP(F), -et * G)
                        put(FP(F), T(c, 0), -et * G.T)
                        put(FP(F), FP(F), et * MF)
                        other = [o for o in self.face_cells[F] if o != c][0]
                        if self.medium[other] == SOLID:           # n_Gamma = -n (into this fluid cell)
                            for d in range(3):
                                put(FP(F), FV(F, d), -n[d] * MF)
                else:
                    for dd, (i, j) in enumerate(SYM):
                        for comp in range(3):
                            En = (n[j] if comp == i else 0.0) if i == j else \
                                R2 * ((n[j] if comp == i else 0.0) + (n[i] if comp == j else 0.0))
                            if En != 0.0:
                                put(T(c, 3 + dd), T(c, comp), En * E)       # s rows: +(v_T, b n)
                                put(T(c, comp), T(c, 3 + dd), -En * E)      # v rows: -(w, s n)
                                if interior:
                                    put(T(c, 3 + dd), FV(F, comp), -En * G)    # s rows: -(v_F, b n)
                                    put(FV(F, comp), T(c, 3 + dd), En * G.T)   # face rows: (w_F, s n)
                    for comp in range(3):
                        put(T(c, comp), T(c, comp), et * E)
                        if interior:
                            put(T(c, comp), FV(F, comp), -et * G)
                            put(FV(F, comp), T(c, comp), -et * G.T)
                            put(FV(F, comp), FV(F, comp), et * MF)
                    if interior:
                        other = [o for o in self.face_cells[F] if o != c][0]
                        if self.medium[other] == FLUID:           # n_Gamma = n (out of this solid cell)
                            for d in range(3):
                                put(FV(F, d), FP(F), -n[d] * MF)
        ntot = nT + self.nfdof
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ntot, ntot))
        self.A = A
        self.M = sp.csr_matrix((np.concatenate(mvals), (np.concatenate(mrows), np.concatenate(mcols))), shape=(nT, nT))
        self.ATT, self.ATF = A[:nT, :nT], A[:nT, nT:]
        self.AFT, self.AFF = A[nT:, :nT], A[nT:, nT:]
        self._AFF_lu = spla.splu(sp.csc_matrix(self.AFF)) if self.nfdof else None
        self._M_lu = spla.splu(sp.csc_matrix(self.M))

    # ------------------------------------------------------------------ points: sources, receivers
    def locate(self, x):
        """Lowest-id cell whose closed cell holds the point x: barycentric coordinates of x in the
        cell's tetrahedra (the tetrahedron itself, or the six of a hexahedron) all >= -1e-12."""
        x = np.asarray(x, float)
        for c in range(self.nc):
            for P in self._cell_tets(c):
                D = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)
                lam = np.linalg.solve(D, x - P[0])
                if lam.min() >= -1e-12 and lam.sum() <= 1.0 + 1e-12:
                    return c
        raise ValueError("point outside the mesh")

    def point_load(self, x, direction):
        """Load vector of eq. rhs for the point force d delta(. - x): phi_a(x) d on the v rows of
        the solid cell holding x, phi_a(x) d_x on the p rows of a fluid cell."""
        c = self.locate(x)
        phi, _ = self.cell_basis(c, np.asarray(x, float)[None, :])
        F = np.zeros(self.ndof)
        N = self.N
        if self.medium[c] == FLUID:
            F[self.off[c]: self.off[c] + N] = direction[0] * phi[0]
        else:
            for comp in range(3):
                F[self.off[c] + comp * N: self.off[c] + (comp + 1) * N] = direction[comp] * phi[0]
        return F

    def point_values(self, U, x):
        """(p,) in a fluid cell or (v_x, v_y, v_z) in a solid cell: the cell polynomials at x."""
        c = self.locate(x)
        phi, _ = self.cell_basis(c, np.asarray(x, float)[None, :])
        N = self.N
        comps = 1 if self.medium[c] == FLUID else 3
        return np.array([phi[0] @ U[self.off[c] + i * N: self.off[c] + (i + 1) * N] for i in range(comps)])

    # ------------------------------------------------------------------ dynamics
    def face_values(self, U):
        """U_F = -A_FF^{-1} A_FT U_T (eq. ex_solve, first line)."""
        if not self.nfdof:
            return np.zeros(0)
        return -self._AFF_lu.solve(self.AFT @ U)

    def keff(self, U):
        return self.ATT @ U + (self.ATF @ self.face_values(U) if self.nfdof else 0.0)

    def rhs(self, U, F=None):
        """k = M^{-1} (F - K_eff U) (eq. ex_solve, second line)."""
        r = -self.keff(U)
        if F is not None:
            r = r + F
        return self._M_lu.solve(r)

    def erk(self, U, dt, nsteps, s=4, load=None, t0=0.0, record=None):
        """n steps of ERK(s) (eq. ERK) from time t0; load(t) gives the load vector F(t) of eq. rhs
        at the stage times t_n + c_i dt; record(n, U) is called after every step."""
        from .oracle import ERK_TABLEAUX
        A, b, c = ERK_TABLEAUX[s]
        U = np.array(U, float, copy=True)
        for n in range(nsteps):
            tn = t0 + n * dt
            ks = []
            for i in range(s):
                Y = U + dt * sum(A[i, j] * ks[j] for j in range(i)) if i else U
                ks.append(self.rhs(Y, None if load is None else load(tn + c[i] * dt)))
            U = U + dt * sum(b[i] * ks[i] for i in range(s))
            if record is not None:
                record(n, U)
        return U

    def energy(self, U):
        return 0.5 * float(U @ (self.M @ U))

    def stab_energy(self, U):
        """sum over cells and faces of eta tau_T |u_T - u_F|^2_F at the face values of U."""
        X = np.concatenate([U, self.face_values(U)])
        return 0.5 * float(X @ ((self.A + self.A.T) @ X))

    def dense_operator(self):
        """L = -M^{-1} K_eff as a dense matrix (tiny meshes)."""
        Kd = self.ATT.toarray()
        if self.nfdof:
            Kd = Kd - self.ATF.toarray() @ np.linalg.solve(self.AFF.toarray(), self.AFT.toarray())
        return -np.linalg.solve(self.M.toarray(), Kd)

    # ------------------------------------------------------------------ projections
    def project(self, fluid_fns, solid_fns):
        """L2 projection of (p, m_x, m_y, m_z) / (v_x, v_y, v_z, s_1 .. s_6) given as callables
        f(x, y, z) onto the cell bases."""
        U = np.zeros(self.ndof)
        N = self.N
        for c in range(self.nc):
            X, W = self.cell_quad(c, self.k + 5)
            phi, _ = self.cell_basis(c, X)
            M0 = (phi * W[:, None]).T @ phi
            fns = fluid_fns if self.medium[c] == FLUID else solid_fns
            for i, fn in enumerate(fns):
                U[self.off[c] + i * N: self.off[c] + (i + 1) * N] = np.linalg.solve(
                    M0, (phi * W[:, None]).T @ fn(X[:, 0], X[:, 1], X[:, 2]))
        return U

    def face_project(self, F, fn):
        X, W = self.face_quad(F, self.k + 4)
        psi = self.face_basis(F, X)
        MF = (psi * W[:, None]).T @ psi
        return np.linalg.solve(MF, (psi * W[:, None]).T @ fn(X[:, 0], X[:, 1], X[:, 2]))


def ricker(t, f0, t0):
    """Ricker wavelet (1 - 2 a^2) exp(-a^2), a = pi f0 (t - t0): the time factor of the point
    sources (the same convention as the two-dimensional oracle)."""
    a = math.pi * f0 * (t - t0)
    return (1.0 - 2.0 * a * a) * math.exp(-a * a)


def cube_mesh(n, tets=True, medium_of=None, materials=None, L=1.0, prisms=False):
    """n^3 cubes of side L / n on [0, L]^3, each split into six tetrahedra around its main diagonal
    (or kept as hexahedra, or with prisms cut into two triangular prisms along the diagonal of its
    base); medium_of(x, y, z) of the cell centre gives 0 (fluid) / 1 (solid)
    (default: solid below z = L / 2); materials (rho_f, c_f, rho_s, lambda, mu), default
    rho = 1, c = 1 in the fluid and rho = 1, lambda = mu = 1 (c_P = sqrt 3, c_S = 1) in the solid."""
    g = np.linspace(0.0, L, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    vid = lambda i, j, l: (i * (n + 1) + j) * (n + 1) + l
    cells = []
    for i in range(n):
        for j in range(n):
            for l in range(n):
                h = (vid(i, j, l), vid(i + 1, j, l), vid(i + 1, j + 1, l), vid(i, j + 1, l),
                     vid(i, j, l + 1), vid(i + 1, j, l + 1), vid(i + 1, j + 1, l + 1), vid(i, j + 1, l + 1))
                if prisms:
                    cells += [(h[0], h[1], h[2], h[4], h[5], h[6]), (h[0], h[2], h[3], h[4], h[6], h[7])]
                elif tets:
                    cells += [tuple(h[t] for t in tt) for tt in HEX_TETS]
                else:
                    cells.append(h)
    medium_of = medium_of or (lambda x, y, z: SOLID if z < 0.5 * L else FLUID)
    cent = np.array([xyz[list(c)].mean(0) for c in cells])
    med = np.array([medium_of(*p) for p in cent], int)
    rf, cf, rs, lam, mu = materials or (1.0, 1.0, 1.0, 1.0, 1.0)
    rho = np.where(med == FLUID, rf, rs)
    a = np.where(med == FLUID, cf, lam)
    b = np.where(med == FLUID, 0.0, mu)
    # orient every tetrahedron positively
    cells = [c if len(c) != 4 or np.linalg.det(np.stack([xyz[c[1]] - xyz[c[0]], xyz[c[2]] - xyz[c[0]],
                                                             xyz[c[3]] - xyz[c[0]]])) > 0 else (c[0], c[2], c[1], c[3])
             for c in cells]
    return dict(xyz=xyz, cells=cells, medium=med, rho=rho, a=a, b=b)
