"""SDIRK(s, s+1) time stepping of the HHO elasto-acoustic semi-discretisation (Sec. 4.1), with the
cell degree k' = k + 1 and the Lehrenfeld-Schoberl stabilisation of Sec. 3.3 (mixed order) or
k' = k with the plain least-squares one (equal order).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain and global: the local forms of
eq. HHO1 / HHO2 with the reconstructions eq. rec_a / rec_e and eq. stab are integrated by
quadrature cell by cell and assembled into one sparse matrix K over all cell and face unknowns
(the ordering of eq. compact_AR: cells first, then faces), the cell mass matrix M beside it; an
SDIRK step is eq. SDIRK_compact as printed, every stage solving the full (uncondensed) system
[[M + a* dt K_T, a* dt K_TF], [a* dt K_FT, a* dt K_F]] U^{n,i} = B^{n,i} with a sparse LU factored
once, the right-hand sides formed by applying K to the earlier stages.  No static condensation,
no blocking.

The geometry, the face list and tags and the cell quadrature points come from the explicit-path
oracle (``Oracle``); the bases, the local forms and the assembly are written here.

Bases: on each cell the graded monomials ((x - x_T)/h_T)^a ((y - y_T)/h_T)^b of degree <= k'
(degree-major, decreasing power of x), orthonormalised in L2(T) by the Cholesky factor of their
Gram matrix; the dual unknowns (m, s) use the first dim P^k(T) of them (the same functions as the
degree-k orthonormal basis).  Faces: orthonormal Legendre polynomials of degree <= k along the
face, from its lower to its higher vertex id.  Symmetric tensors: E1 = e1e1, E2 = e2e2,
E3 = (e1e2 + e2e1)/sqrt(2).

Unknown layout per cell: fluid [p (N') | m_x (N) | m_y (N)], solid [v_x (N') | v_y (N') | s_1 |
s_2 | s_3 (N each)], N' = dim P^{k'}, N = dim P^k; cells in input order.  Faces: fluid f, solid
2f ([v_x | v_y]), interface 3f ([p | v_x | v_y]) unknowns, f = k + 1; boundary faces carry none
(homogeneous Dirichlet data).

Readings (the paper leaves them open):
  * stabilisation weights: tau^f = eta^f / (rho c) and tau^s = eta^s rho c^s (c^s = c_P, or c_S
    with stab_speed = 1), times (h_T / l_Omega)^(-alpha); l_Omega = diam(Omega), by default the
    largest distance between two boundary vertices; eta^f = eta^s = 1 unless given (the weights
    0.8 / 1.5 of Sec. 5.1 are stated for the explicit schemes);
  * SDIRK(1,2) is the implicit midpoint rule; SDIRK(2,3) takes a* = (3 + sqrt(3))/6 (the printed
    two-stage tableau, a* = 1/4, c = (1/4, 3/4), satisfies the order conditions up to order 2
    only); SDIRK(3,4) is the printed tableau with nu and xi;
  * the last stage only inverts the mass matrix on the cell rows (the text of Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .oracle import Oracle

T_INT_F, T_INT_S, T_GAMMA, T_BND_F, T_BND_S = 0, 1, 2, 3, 4
FLUID, SOLID = 0, 1


def sdirk_tableau(s):
    """(A, b, c) of SDIRK(s, s+1), s = 1, 2, 3 (eq. SDIRK; readings in the module docstring)."""
    if s == 1:
        return np.array([[0.5]]), np.array([1.0]), np.array([0.5])
    if s == 2:
        g = (3.0 + math.sqrt(3.0)) / 6.0
        return np.array([[g, 0.0], [1.0 - 2.0 * g, g]]), np.array([0.5, 0.5]), np.array([g, 1.0 - g])
    if s == 3:
        nu = math.cos(math.pi / 18.0) / math.sqrt(3.0) + 0.5
        xi = 1.0 / (6.0 * (2.0 * nu - 1.0) ** 2)
        A = np.array([[nu, 0, 0], [0.5 - nu, nu, 0], [2 * nu, 1 - 4 * nu, nu]])
        return A, np.array([xi, 1 - 2 * xi, xi]), np.array([nu, 0.5, 1 - nu])
    raise ValueError("SDIRK stages must be 1, 2 or 3")


def printed_sdirk2_tableau():
    """The two-stage tableau as the paper prints it (a* = 1/4)."""
    return np.array([[0.25, 0.0], [0.5, 0.25]]), np.array([0.5, 0.5]), np.array([0.25, 0.75])


def _exps(k):
    return [(a, d - a) for d in range(k + 1) for a in range(d, -1, -1)]


def _eten(al, c, d):
    if al == 0:
        return 1.0 if (c == 0 and d == 0) else 0.0
    if al == 1:
        return 1.0 if (c == 1 and d == 1) else 0.0
    return 1.0 / math.sqrt(2.0) if c != d else 0.0


def _ricker(t, f0, t0):
    a = math.pi * f0 * (t - t0)
    return (1.0 - 2.0 * a * a) * math.exp(-a * a)


def domain_diameter(mesh):
    """Largest distance between two vertices lying on boundary edges (= diam of the polygonal
    domain, attained at boundary vertices)."""
    ptr, vtx, xy = mesh["cell_ptr"], mesh["cell_vtx"], np.asarray(mesh["xy"], float)
    cnt = {}
    for c in range(len(ptr) - 1):
        vs = vtx[ptr[c]:ptr[c + 1]]
        for i in range(len(vs)):
            e = (min(vs[i], vs[(i + 1) % len(vs)]), max(vs[i], vs[(i + 1) % len(vs)]))
            cnt[e] = cnt.get(e, 0) + 1
    bv = sorted({v for e, n in cnt.items() if n == 1 for v in e})
    P = xy[bv]
    best = 0.0
    for i in range(len(P)):
        d = np.sqrt(((P[i + 1:] - P[i]) ** 2).sum(axis=1))
        if len(d):
            best = max(best, float(d.max()))
    return best


class ImplicitOracle:
    """Global FP64 assembly of M and K, SDIRK stepping by sparse LU of the full stage system."""

    def __init__(self, mesh, k, mixed=True, alpha=1, eta_f=1.0, eta_s=1.0, stab_speed=1, ell=None):
        self.mesh, self.k, self.mixed, self.alpha = mesh, k, mixed, alpha
        self.kp = k + 1 if mixed else k
        self.N = (k + 1) * (k + 2) // 2
        self.Np = (self.kp + 1) * (self.kp + 2) // 2
        self.nf = k + 1
        self.geo = Oracle(mesh, k, eta_f, eta_s, stab_speed)
        g = self.geo.cell_geom()
        self.bary, self.h = g["bary"], g["h"]
        self.nc = self.geo.nc
        self.medium = np.asarray(mesh["medium"], np.uint8)
        self.ell = float(ell) if ell else domain_diameter(mesh)
        rho, pa, pb = (np.asarray(mesh[x], float) for x in ("rho", "a", "b"))
        self.rho = rho
        tau = np.zeros(self.nc)
        self.cinv = np.zeros((self.nc, 3, 3))
        for c in range(self.nc):
            scale = (self.ell / self.h[c]) ** alpha
            if self.medium[c] == FLUID:
                tau[c] = eta_f / (rho[c] * pa[c]) * scale
            else:
                lam, mu = pa[c], pb[c]
                cs = math.sqrt((lam + 2 * mu) / rho[c]) if stab_speed == 0 else math.sqrt(mu / rho[c])
                tau[c] = eta_s * rho[c] * cs * scale
                for al in range(3):
                    for be in range(3):
                        X = np.array([[_eten(be, 0, 0), _eten(be, 0, 1)], [_eten(be, 1, 0), _eten(be, 1, 1)]])
                        Y = (X - lam / (2 * (lam + mu)) * np.trace(X) * np.eye(2)) / (2 * mu)
                        Ea = np.array([[_eten(al, 0, 0), _eten(al, 0, 1)], [_eten(al, 1, 0), _eten(al, 1, 1)]])
                        self.cinv[c, al, be] = float((Y * Ea).sum())
        self.tau = tau
        # unknown offsets
        sizes = np.where(self.medium == FLUID, self.Np + 2 * self.N, 2 * self.Np + 3 * self.N)
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.ndof = int(self.off[-1])
        fv, fc, tag = self.geo.face_info()
        self.fv, self.fc, self.ftag = fv, fc, tag
        w = np.array([1, 2, 3, 0, 0])[tag]
        self.foff = np.concatenate([[0], np.cumsum(w * self.nf)]).astype(np.int64) + self.ndof
        self.nface_dofs = int(self.foff[-1] - self.ndof)
        self.ntot = self.ndof + self.nface_dofs
        self.sources = []
        self._assemble()

    # ---------------------------------------------------------------- bases
    def _cell_basis(self, c, x, y):
        """Orthonormal degree-k' basis of cell c and its gradient at points (x, y) -> [Np, n]."""
        C = self._coef[c]
        h, (xT, yT) = self.h[c], self.bary[c]
        X, Y = (np.asarray(x) - xT) / h, (np.asarray(y) - yT) / h
        mu = np.array([X ** a * Y ** b for a, b in _exps(self.kp)])
        mx = np.array([a * X ** max(a - 1, 0) * Y ** b / h if a else 0 * X for a, b in _exps(self.kp)])
        my = np.array([b * X ** a * Y ** max(b - 1, 0) / h if b else 0 * X for a, b in _exps(self.kp)])
        return C @ mu, C @ mx, C @ my

    def _face_basis(self, f, x, y):
        a, b = self.fv[f]
        xy = np.asarray(self.mesh["xy"], float)
        P0, P1 = xy[a], xy[b]
        L = float(np.hypot(*(P1 - P0)))
        t = ((np.asarray(x) - P0[0]) * (P1[0] - P0[0]) + (np.asarray(y) - P0[1]) * (P1[1] - P0[1])) / L ** 2
        xi = 2.0 * t - 1.0
        return np.array([math.sqrt((2 * i + 1) / L) * np.polynomial.legendre.Legendre.basis(i)(xi)
                         for i in range(self.nf)])

    def _face_quad(self, f):
        a, b = self.fv[f]
        xy = np.asarray(self.mesh["xy"], float)
        P0, P1 = xy[a], xy[b]
        L = float(np.hypot(*(P1 - P0)))
        gx, gw = np.polynomial.legendre.leggauss(self.kp + 2)
        t = 0.5 * (1 + gx)
        return P0[0] + t * (P1[0] - P0[0]), P0[1] + t * (P1[1] - P0[1]), 0.5 * gw * L

    # ---------------------------------------------------------------- assembly
    def _assemble(self):
        nq = self.kp + 3
        px, py, pw, pc = self.geo.quad_points(nq)
        ptr = np.asarray(self.mesh["cell_ptr"])
        self._coef = []
        N, Np, nf = self.N, self.Np, self.nf
        rows, cols, vals = [], [], []
        mrows, mcols, mvals = [], [], []

        def put(r, cidx, block):
            rr, cc = np.meshgrid(r, cidx, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(np.asarray(block, float).ravel())

        def putm(r, cidx, block):
            rr, cc = np.meshgrid(r, cidx, indexing="ij")
            mrows.append(rr.ravel())
            mcols.append(cc.ravel())
            mvals.append(np.asarray(block, float).ravel())

        q0 = 0
        for c in range(self.nc):
            nqc = (ptr[c + 1] - ptr[c]) * nq * nq
            sl = slice(q0, q0 + nqc)
            q0 += nqc
            x, y, w = px[sl], py[sl], pw[sl]
            h, (xT, yT) = self.h[c], self.bary[c]
            X, Y = (x - xT) / h, (y - yT) / h
            mu = np.array([X ** a * Y ** b for a, b in _exps(self.kp)])
            Gm = (mu * w) @ mu.T
            Lc = np.linalg.cholesky(Gm)
            self._coef.append(np.linalg.inv(Lc))
            ph, phx, phy = self._cell_basis(c, x, y)
            M0p = (ph * w) @ ph.T                     # (phi'_a, phi'_b)_T
            M0 = M0p[:N, :N]
            Dd = [(ph[:N] * w) @ g.T for g in (phx, phy)]   # D_c[a][b] = (d_c phi'_b, phi_a)_T
            o = int(self.off[c])
            ops = self.geo.cell_ops(c)
            faces, nrm = ops["faces"], ops["n"]
            tau = self.tau[c]
            if self.medium[c] == FLUID:
                ip, im = o + np.arange(Np), [o + Np + cc * N + np.arange(N) for cc in range(2)]
                kap = self.rho[c] * float(self.mesh["a"][c]) ** 2
                putm(ip, ip, M0p / kap)
                for cc in range(2):
                    putm(im[cc], im[cc], self.rho[c] * M0)
                    # m rows: -b_T(p; r): -(d_c p_T, r) + (p_T - p_F, r n_c)_dT
                    put(im[cc], ip, -Dd[cc])
                    # p rows: b_T(q; m) = (d_c q_T, m_c) - (q_T, m . n)_dT
                    put(ip, im[cc], Dd[cc].T)
            else:
                iv = [o + cc * Np + np.arange(Np) for cc in range(2)]
                isg = [o + 2 * Np + al * N + np.arange(N) for al in range(3)]
                for cc in range(2):
                    putm(iv[cc], iv[cc], self.rho[c] * M0p)
                for al in range(3):
                    for be in range(3):
                        putm(isg[al], isg[be], self.cinv[c, al, be] * M0)
                for al in range(3):
                    for cc in range(2):
                        for d in range(2):
                            e = _eten(al, cc, d)
                            if e == 0.0:
                                continue
                            # s rows: -(grad_sym v_T, b)_T ; v rows: +(grad_sym w_T, s)_T
                            put(isg[al], iv[cc], -e * Dd[d])
                            put(iv[cc], isg[al], e * Dd[d].T)
            for j, f in enumerate(faces):
                fx, fy, fw = self._face_quad(f)
                phf, _, _ = self._cell_basis(c, fx, fy)
                psi = self._face_basis(f, fx, fy)
                Ep = (phf[:N] * fw) @ phf.T            # (phi'_b, phi_a)_F, a < N
                Gp = (phf * fw) @ psi.T                # (phi'_a, psi_i)_F
                Gd = Gp[:N]                            # (phi_a, psi_i)_F
                Pp = Gp @ Gp.T                         # (Pi phi'_b, Pi phi'_a)_F
                MF = (psi * fw) @ psi.T
                n = nrm[j]
                tagf = self.ftag[f]
                bnd = tagf in (T_BND_F, T_BND_S)
                if self.medium[c] == FLUID:
                    ipF = None if bnd else self.foff[f] + np.arange(nf)
                    for cc in range(2):
                        put(im[cc], ip, n[cc] * Ep)
                        put(ip, im[cc], -n[cc] * Ep.T)
                        if ipF is not None:
                            put(im[cc], ipF, -n[cc] * Gd)
                            put(ipF, im[cc], n[cc] * Gd.T)
                    put(ip, ip, tau * Pp)
                    if ipF is not None:
                        put(ip, ipF, -tau * Gp)
                        put(ipF, ip, -tau * Gp.T)
                        put(ipF, ipF, tau * MF)
                else:
                    base = self.foff[f] + (nf if tagf == T_GAMMA else 0)
                    ivF = None if bnd else [base + cc * nf + np.arange(nf) for cc in range(2)]
                    for al in range(3):
                        for cc in range(2):
                            en = _eten(al, cc, 0) * n[0] + _eten(al, cc, 1) * n[1]
                            if en == 0.0:
                                continue
                            put(isg[al], iv[cc], en * Ep)
                            put(iv[cc], isg[al], -en * Ep.T)
                            if ivF is not None:
                                put(isg[al], ivF[cc], -en * Gd)
                                put(ivF[cc], isg[al], en * Gd.T)
                    for cc in range(2):
                        put(iv[cc], iv[cc], tau * Pp)
                        if ivF is not None:
                            put(iv[cc], ivF[cc], -tau * Gp)
                            put(ivF[cc], iv[cc], -tau * Gp.T)
                            put(ivF[cc], ivF[cc], tau * MF)
                    if tagf == T_GAMMA:
                        # coupling: fluid face rows +(v_F . n_G, q_F), solid face rows -(p_F n_G, w_F),
                        # n_G = outward normal of the solid cell
                        ipF = self.foff[f] + np.arange(nf)
                        for cc in range(2):
                            put(ipF, ivF[cc], n[cc] * MF)
                            put(ivF[cc], ipF, -n[cc] * MF.T)
        nt = self.ntot
        self.K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nt, nt))
        self.M = sp.csr_matrix((np.concatenate(mvals), (np.concatenate(mrows), np.concatenate(mcols))),
                               shape=(self.ndof, self.ndof))
        self.Mfull = sp.block_diag([self.M, sp.csr_matrix((self.nface_dofs, self.nface_dofs))], format="csr")

    # ---------------------------------------------------------------- loads
    def set_point_sources(self, xy, direction, f0, t0, amp):
        """Point forces with a Ricker time factor: F_a = amp R(t) phi'_a(x_s) d (solid v rows) or
        amp R(t) d_x phi'_a(x_s) (fluid p rows), in the cell with the lowest id holding x_s."""
        xy = np.asarray(xy, float).reshape(-1, 2)
        n = len(xy)
        d = np.broadcast_to(np.asarray(direction, float), (n, 2))
        f0, t0, amp = (np.broadcast_to(np.asarray(v, float), (n,)) for v in (f0, t0, amp))
        self.sources = []
        for s in range(n):
            c = self.geo.locate(*xy[s])
            if c < 0:
                continue
            ph, _, _ = self._cell_basis(c, np.array([xy[s, 0]]), np.array([xy[s, 1]]))
            g = np.zeros(self.ndof)
            o = int(self.off[c])
            if self.medium[c] == FLUID:
                g[o:o + self.Np] = d[s, 0] * ph[:, 0]
            else:
                for cc in range(2):
                    g[o + cc * self.Np:o + (cc + 1) * self.Np] = d[s, cc] * ph[:, 0]
            self.sources.append((g, float(f0[s]), float(t0[s]), float(amp[s])))

    def load(self, t):
        """Cell load vector F_T(t) (eq. rhs, load-vector reading)."""
        F = np.zeros(self.ndof)
        for g, f0, t0, amp in self.sources:
            F += amp * _ricker(t, f0, t0) * g
        return F

    # ---------------------------------------------------------------- projections / diagnostics
    def project(self, fluid_fns, solid_fns, nq=None):
        """L2 projection of (p, m_x, m_y) / (v_x, v_y, s_1, s_2, s_3) onto the cell bases (nq
        points per direction of each fan triangle; default k' + 6, exact for polynomial data)."""
        nq = nq or self.kp + 6
        px, py, pw, pc = self.geo.quad_points(nq)
        ptr = np.asarray(self.mesh["cell_ptr"])
        U = np.zeros(self.ndof)
        q0 = 0
        for c in range(self.nc):
            nqc = (ptr[c + 1] - ptr[c]) * nq * nq
            x, y, w = px[q0:q0 + nqc], py[q0:q0 + nqc], pw[q0:q0 + nqc]
            q0 += nqc
            ph, _, _ = self._cell_basis(c, x, y)
            Mp = (ph * w) @ ph.T
            o = int(self.off[c])
            if self.medium[c] == FLUID:
                blocks = [(fluid_fns[0], self.Np)] + [(fn, self.N) for fn in fluid_fns[1:]]
            else:
                blocks = [(fn, self.Np) for fn in solid_fns[:2]] + [(fn, self.N) for fn in solid_fns[2:]]
            for fn, n in blocks:
                rhs = (ph[:n] * w) @ fn(x, y)
                U[o:o + n] = np.linalg.solve(Mp[:n, :n], rhs)
                o += n
        return U

    def point_values(self, U, x, y):
        """(cell, values) of the cell polynomials of U at (x, y) in the lowest-id cell holding it:
        fluid (p, m_x, m_y), solid (v_x, v_y, s_1, s_2, s_3)."""
        c = self.geo.locate(x, y)
        if c < 0:
            raise ValueError("point outside the mesh")
        ph, _, _ = self._cell_basis(c, np.array([x]), np.array([y]))
        ph = ph[:, 0]
        o = int(self.off[c])
        sizes = [self.Np, self.N, self.N] if self.medium[c] == FLUID else [self.Np, self.Np] + [self.N] * 3
        vals = []
        for n in sizes:
            vals.append(float(ph[:n] @ U[o:o + n]))
            o += n
        return c, np.array(vals)

    def energy(self, U):
        """Half the mass-weighted squared norm of the cell unknowns (Sec. 5.1)."""
        return 0.5 * float(U @ (self.M @ U))

    def mass_dot(self, U, V):
        return float(U @ (self.M @ V))

    def dense_operator(self):
        """L = -M^{-1} (K_T - K_TF K_F^{-1} K_FT), dense (tiny meshes)."""
        K = self.K.toarray()
        nd = self.ndof
        KT, KTF, KFT, KF = K[:nd, :nd], K[:nd, nd:], K[nd:, :nd], K[nd:, nd:]
        Keff = KT - KTF @ np.linalg.solve(KF, KFT) if self.nface_dofs else KT
        return -np.linalg.solve(self.M.toarray(), Keff)

    # ---------------------------------------------------------------- SDIRK
    def sdirk(self, U, t0, dt, nsteps, s=3, energies=False, tableau=None):
        """n steps of SDIRK(s, s+1) (eq. SDIRK_compact) from time t0; returns U (and the energy
        after every step)."""
        A, b, c = tableau if tableau is not None else sdirk_tableau(s)
        s = len(b)
        ast = A[0, 0]
        nd = self.ndof
        lu = spla.splu((self.Mfull + ast * dt * self.K).tocsc())
        U = np.array(U, float, copy=True)
        E = []
        for n in range(nsteps):
            t = t0 + n * dt
            X0 = np.concatenate([U, np.zeros(self.nface_dofs)])
            MX0 = self.Mfull @ X0
            Fj, KX = [], []
            for i in range(s):
                Fi = np.concatenate([self.load(t + c[i] * dt), np.zeros(self.nface_dofs)])
                B = MX0 + ast * dt * Fi
                for j in range(i):
                    B += dt * A[i, j] * (Fj[j] - KX[j])
                X = lu.solve(B)
                Fj.append(Fi)
                KX.append(self.K @ X)
            R = self.M @ U
            for j in range(s):
                R += dt * b[j] * (Fj[j][:nd] - KX[j][:nd])
            U = spla.spsolve(self.M.tocsc(), R)
            if energies:
                E.append(self.energy(U))
        return (U, np.array(E)) if energies else U
