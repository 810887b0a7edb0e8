"""NumPy model of the fused stage kernels' arithmetic, driven by the host plan that
libhho.so exports through include/hho_inspect.h (no GPU needed).

Used by the CPU tests to check the library's host side (shape classes, class tables,
face links, face-solve coefficients, materials, gradient coefficients, the orientation
convention between neighbouring cells) against the FP64 oracle before any kernel runs.
It follows the same algebra as kernels.hip and adjoint.hip: own trace contribution
r_T = tau G^T u - G^T (flux . n), neighbour contribution read in the neighbour's face basis
(mode i flips sign as (-1)^i), face solve, cell residual, inverse mass; for the adjoint the
transformed state z = D M^{-1} mu, the face solve with the interface coupling reversed, and
the per-cell parameter derivatives.
"""
import numpy as np

R2 = 1.0 / np.sqrt(2.0)


_DEG = (0, 1, 1, 2, 2, 2, 3, 3, 3, 3)


def _unpack_pooled(t, off, N, F, nF):
    """Dense B_x, B_y, S, G, normals from a pooled (packed) table: the entries of B_x and B_y with
    deg(b) < deg(r), the upper triangle of S, the entries of G_j with i <= deg(a), the normals."""
    pos = off
    B = []
    for _ in range(2):
        M = np.zeros((N, N))
        for r in range(N):
            for b in range(N):
                if _DEG[b] < _DEG[r]:
                    M[r, b] = t[pos]
                    pos += 1
        B.append(M)
    Sm = np.zeros((N, N))
    for r in range(N):
        for b in range(r, N):
            Sm[r, b] = Sm[b, r] = t[pos]
            pos += 1
    G = np.zeros((nF, N, F))
    for j in range(nF):
        for a in range(N):
            for i in range(F):
                if i <= _DEG[a]:
                    G[j, a, i] = t[pos]
                    pos += 1
    nrm = t[pos:pos + 2 * nF].reshape(nF, 2)
    return B[0], B[1], Sm, G, nrm


def _cell_tables(ins, g, ic):
    """Class tables of internal cell ic in group g (a pooled group's cells each have their own,
    packed)."""
    N, F = ins.N, ins.F
    med, nF, off = int(ins.groups[g, 0]), int(ins.groups[g, 1]), int(ins.ic_tab[ic])
    t = ins.tables
    if ins.pooled[g]:
        return (med, nF) + _unpack_pooled(t, off, N, F, nF)
    Bx = t[off:off + N * N].reshape(N, N)
    By = t[off + N * N:off + 2 * N * N].reshape(N, N)
    Sm = t[off + 2 * N * N:off + 3 * N * N].reshape(N, N)
    G = t[off + 3 * N * N:off + 3 * N * N + nF * N * F].reshape(nF, N, F)
    nrm = t[off + 3 * N * N + nF * N * F:off + 3 * N * N + nF * N * F + 2 * nF].reshape(nF, 2)
    return med, nF, Bx, By, Sm, G, nrm


class _Layout:
    def __init__(self, ins, mesh):
        self.med_in = np.asarray(mesh["medium"])
        self.nb = np.where(self.med_in == 0, 3, 5)
        self.ext_off = np.concatenate([[0], np.cumsum(self.nb * ins.N)])
        self.cell_of_ic = -np.ones(ins.n_ic, int)
        self.cell_of_ic[ins.ic_of_cell] = np.arange(len(self.med_in))
        self.group_of_ic = -np.ones(ins.n_ic, int)
        for g in range(ins.n_groups):
            b, n = ins.groups[g, 3], ins.groups[g, 4]
            self.group_of_ic[b:b + n] = g

    def split(self, ins, U):
        """external vector -> {ic: [rows, N]}"""
        return {ins.ic_of_cell[c]: U[self.ext_off[c]:self.ext_off[c + 1]].reshape(self.nb[c], ins.N).copy()
                for c in range(len(self.med_in))}


def _dual_inv_mass(ins, ic, med, u):
    """z = D M^{-1} u for one cell (D flips the sign of the dual unknowns m, s)."""
    irho, stiff, lam, tmu = ins.mat[0, ic], ins.mat[1, ic], ins.mat[3, ic], ins.mat[4, ic]
    if med == 0:
        return np.stack([stiff * u[0], -irho * u[1], -irho * u[2]])
    return np.stack([irho * u[0], irho * u[1], -(stiff * u[2] + lam * u[3]), -(lam * u[2] + stiff * u[3]),
                     -tmu * u[4]])


def _face_values(ins, lay, state, adjoint):
    """Face values per (ic, j), in the cell's own face orientation: [1, F] (fluid) or [2, F]
    (solid), from the cell states; adjoint=True reverses the interface coupling."""
    tau, itau = ins.mat[2], ins.mat[5]
    tr = {}
    for ic, u in state.items():
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, lay.group_of_ic[ic], ic)
        for j in range(nF):
            nx, ny = nrm[j]
            if med == 0:
                q = tau[ic] * u[0] - (nx * u[1] + ny * u[2])
                tr[(ic, j)] = (G[j].T @ q)[None, :]
            else:
                qx = tau[ic] * u[0] - (nx * u[2] + R2 * ny * u[4])
                qy = tau[ic] * u[1] - (R2 * nx * u[4] + ny * u[3])
                tr[(ic, j)] = np.stack([G[j].T @ qx, G[j].T @ qy])
    sg = np.array([(-1.0) ** i for i in range(ins.F)])
    sc = -1.0 if adjoint else 1.0
    fv = {}
    for ic in state:
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, lay.group_of_ic[ic], ic)
        for j in range(nF):
            lk = int(ins.link[j, ic])
            if lk < 0:
                continue
            icn, iface, jn = lk >> 4, (lk >> 3) & 1, lk & 7
            nx, ny = nrm[j]
            cc = ins.c0[j, ic]
            own, nbr = tr[(ic, j)], tr[(icn, jn)] * sg[None, :]
            if med == 0:
                if not iface:
                    pF = (own[0] + nbr[0]) * cc
                else:
                    pF = (own[0] + sc * (nx * nbr[0] + ny * nbr[1]) * itau[icn]) * cc
                fv[(ic, j)] = pF[None, :]
            else:
                if not iface:
                    vFx, vFy = (own[0] + nbr[0]) * cc, (own[1] + nbr[1]) * cc
                else:
                    pF = (nbr[0] - sc * (nx * own[0] + ny * own[1]) * itau[ic]) * cc
                    vFx, vFy = (own[0] + sc * nx * pF) * itau[ic], (own[1] + sc * ny * pF) * itau[ic]
                fv[(ic, j)] = np.stack([vFx, vFy])
    return fv


def rhs(ins, mesh, U, adjoint=False):
    """k = M^{-1}(-K_eff U) for the external state U (no loads).

    adjoint=True models the adjoint stage instead: L^T x = D R_c(D M^{-1} x), where D flips the
    sign of the dual unknowns (m, s) and R_c = -K_eff with the interface coupling reversed."""
    lay = _Layout(ins, mesh)
    state = lay.split(ins, U)
    if adjoint:
        state = {ic: _dual_inv_mass(ins, ic, lay.med_in[lay.cell_of_ic[ic]], u) for ic, u in state.items()}
    fv = _face_values(ins, lay, state, adjoint)
    tau = ins.mat[2]
    out = np.zeros_like(U)
    for ic, u in state.items():
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, lay.group_of_ic[ic], ic)
        t = tau[ic]
        if med == 0:
            p, mx, my = u
            rmx, rmy = Bx @ p, By @ p
            rp = -(Bx.T @ mx + By.T @ my + t * Sm @ p)
        else:
            vx, vy, s1, s2, s3 = u
            rs1, rs2, rs3 = Bx @ vx, By @ vy, R2 * (By @ vx + Bx @ vy)
            rvx = -(Bx.T @ s1 + R2 * By.T @ s3 + t * Sm @ vx)
            rvy = -(By.T @ s2 + R2 * Bx.T @ s3 + t * Sm @ vy)
        for j in range(nF):
            if (ic, j) not in fv:
                continue
            nx, ny = nrm[j]
            if med == 0:
                w = G[j] @ fv[(ic, j)][0]
                rmx += nx * w
                rmy += ny * w
                rp += t * w
            else:
                wx, wy = G[j] @ fv[(ic, j)][0], G[j] @ fv[(ic, j)][1]
                rs1 += nx * wx
                rs2 += ny * wy
                rs3 += R2 * (ny * wx + nx * wy)
                rvx += t * wx
                rvy += t * wy
        c = lay.cell_of_ic[ic]
        irho, stiff, lam, tmu = ins.mat[0, ic], ins.mat[1, ic], ins.mat[3, ic], ins.mat[4, ic]
        if adjoint:
            k = np.concatenate([rp, -rmx, -rmy]) if med == 0 else np.concatenate([rvx, rvy, -rs1, -rs2, -rs3])
        elif med == 0:
            k = np.concatenate([stiff * rp, irho * rmx, irho * rmy])
        else:
            k = np.concatenate([irho * rvx, irho * rvy, stiff * rs1 + lam * rs2, lam * rs1 + stiff * rs2,
                                tmu * rs3])
        out[lay.ext_off[c]:lay.ext_off[c + 1]] = k
    return out


def grad_terms(ins, mesh, Y, k, mu):
    """Per-cell parameter derivatives of one stage as the adjoint stage kernel forms them:
    grad[c] = -[w^T (dM/dtheta) k + (dtau/dtheta) sum_F (Y_T - Y_F, w_T - W_F)_F] with
    w = D z, z = D M^{-1} mu, Y_F the forward face values of Y and W_F the adjoint face values
    of z; the face mass of the orthonormal face basis is the identity and S = sum_F E_F."""
    lay = _Layout(ins, mesh)
    ys, ks = lay.split(ins, Y), lay.split(ins, k)
    zs = {ic: _dual_inv_mass(ins, ic, lay.med_in[lay.cell_of_ic[ic]], u)
          for ic, u in lay.split(ins, mu).items()}
    fy = _face_values(ins, lay, ys, False)
    fz = _face_values(ins, lay, zs, True)
    gm = ins.gm
    grad = np.zeros((len(lay.med_in), 3))
    for ic, z in zs.items():
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, lay.group_of_ic[ic], ic)
        y, kk = ys[ic], ks[ic]
        nc = 1 if med == 0 else 2
        w = z.copy()
        w[nc:] *= -1.0
        stab = 0.0
        for c in range(nc):
            stab += y[c] @ Sm @ w[c]
            for j in range(nF):
                if (ic, j) not in fy:
                    continue
                YF, WF = fy[(ic, j)][c], fz[(ic, j)][c]
                stab -= y[c] @ G[j] @ WF + w[c] @ G[j] @ YF - YF @ WF
        g = np.zeros(3)
        if med == 0:
            wk_p, wk_m = w[0] @ kk[0], w[1] @ kk[1] + w[2] @ kk[2]
            g[0] = -(gm[0, ic] * wk_p + wk_m + gm[2, ic] * stab)
            g[1] = -(gm[1, ic] * wk_p + gm[3, ic] * stab)
        else:
            P = np.array([[w[2 + a] @ kk[2 + b] for b in range(3)] for a in range(3)])
            g[0] = -(w[0] @ kk[0] + w[1] @ kk[1] + gm[0, ic] * stab)
            g[1] = -(gm[3, ic] * P[:2, :2].sum() + gm[1, ic] * stab)
            g[2] = -(gm[4, ic] * (P[0, 0] + P[1, 1]) + gm[5, ic] * (P[0, 1] + P[1, 0]) + gm[6, ic] * P[2, 2]
                     + gm[2, ic] * stab)
        grad[lay.cell_of_ic[ic]] = g
    return grad
