"""NumPy model of the fused stage kernel's arithmetic, driven by the host plan that
libhho.so exports through include/hho_inspect.h (no GPU needed).

Used by the CPU tests to check the library's host side (shape classes, class tables,
face links, face-solve coefficients, materials, the orientation convention between
neighbouring cells) against the FP64 oracle before any kernel runs.  It follows the
same algebra as kernels.hip: own trace contribution r_T = tau G^T u - G^T (flux . n),
neighbour contribution read in the neighbour's face basis (mode i flips sign as
(-1)^i), face solve, cell residual, inverse mass.
"""
import numpy as np

R2 = 1.0 / np.sqrt(2.0)


def _cell_tables(ins, g):
    N, F = ins.N, ins.F
    med, nF, off = int(ins.groups[g, 0]), int(ins.groups[g, 1]), int(ins.groups[g, 2])
    t = ins.tables
    Bx = t[off:off + N * N].reshape(N, N)
    By = t[off + N * N:off + 2 * N * N].reshape(N, N)
    Sm = t[off + 2 * N * N:off + 3 * N * N].reshape(N, N)
    G = t[off + 3 * N * N:off + 3 * N * N + nF * N * F].reshape(nF, N, F)
    nrm = t[off + 3 * N * N + nF * N * F:off + 3 * N * N + nF * N * F + 2 * nF].reshape(nF, 2)
    return med, nF, Bx, By, Sm, G, nrm


def rhs(ins, mesh, U, adjoint=False):
    """k = M^{-1}(-K_eff U) for the external state U (no loads).

    adjoint=True models the adjoint stage instead: L^T x = D R_c(D M^{-1} x), where D flips the
    sign of the dual unknowns (m, s) and R_c = -K_eff with the interface coupling reversed."""
    N, F = ins.N, ins.F
    med_in = np.asarray(mesh["medium"])
    nb = np.where(med_in == 0, 3, 5)
    ext_off = np.concatenate([[0], np.cumsum(nb * N)])
    cell_of_ic = -np.ones(ins.n_ic, int)
    cell_of_ic[ins.ic_of_cell] = np.arange(len(med_in))
    group_of_ic = -np.ones(ins.n_ic, int)
    for g in range(ins.n_groups):
        b, n = ins.groups[g, 3], ins.groups[g, 4]
        group_of_ic[b:b + n] = g
    state = {}
    for c in range(len(med_in)):
        u = U[ext_off[c]:ext_off[c + 1]].reshape(nb[c], N).copy()
        if adjoint:
            ic = ins.ic_of_cell[c]
            irho, stiff, lam, tmu = ins.mat[0, ic], ins.mat[1, ic], ins.mat[3, ic], ins.mat[4, ic]
            if med_in[c] == 0:
                u = np.stack([stiff * u[0], -irho * u[1], -irho * u[2]])
            else:
                u = np.stack([irho * u[0], irho * u[1], -(stiff * u[2] + lam * u[3]), -(lam * u[2] + stiff * u[3]),
                              -tmu * u[4]])
        state[ins.ic_of_cell[c]] = u
    tau = ins.mat[2]
    itau = ins.mat[5]
    # trace contributions of every cell and face
    tr = {}
    for ic, u in state.items():
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, group_of_ic[ic])
        for j in range(nF):
            nx, ny = nrm[j]
            if med == 0:
                q = tau[ic] * u[0] - (nx * u[1] + ny * u[2])
                tr[(ic, j)] = (G[j].T @ q)[None, :]
            else:
                qx = tau[ic] * u[0] - (nx * u[2] + R2 * ny * u[4])
                qy = tau[ic] * u[1] - (R2 * nx * u[4] + ny * u[3])
                tr[(ic, j)] = np.stack([G[j].T @ qx, G[j].T @ qy])
    sg = np.array([(-1.0) ** i for i in range(F)])
    out = np.zeros_like(U)
    for ic, u in state.items():
        med, nF, Bx, By, Sm, G, nrm = _cell_tables(ins, group_of_ic[ic])
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
            lk = int(ins.link[j, ic])
            if lk < 0:
                continue
            icn, iface, jn = lk >> 4, (lk >> 3) & 1, lk & 7
            nx, ny = nrm[j]
            cc = ins.c0[j, ic]
            own, nbr = tr[(ic, j)], tr[(icn, jn)] * sg[None, :]
            if med == 0:
                sc = -1.0 if adjoint else 1.0
                if not iface:
                    pF = (own[0] + nbr[0]) * cc
                else:
                    pF = (own[0] + sc * (nx * nbr[0] + ny * nbr[1]) * itau[icn]) * cc
                w = G[j] @ pF
                rmx += nx * w
                rmy += ny * w
                rp += t * w
            else:
                if not iface:
                    vFx, vFy = (own[0] + nbr[0]) * cc, (own[1] + nbr[1]) * cc
                else:
                    sc = -1.0 if adjoint else 1.0
                    pF = (nbr[0] - sc * (nx * own[0] + ny * own[1]) * itau[ic]) * cc
                    vFx, vFy = (own[0] + sc * nx * pF) * itau[ic], (own[1] + sc * ny * pF) * itau[ic]
                wx, wy = G[j] @ vFx, G[j] @ vFy
                rs1 += nx * wx
                rs2 += ny * wy
                rs3 += R2 * (ny * wx + nx * wy)
                rvx += t * wx
                rvy += t * wy
        c = cell_of_ic[ic]
        irho, stiff, lam, tmu = ins.mat[0, ic], ins.mat[1, ic], ins.mat[3, ic], ins.mat[4, ic]
        if adjoint:
            k = np.concatenate([rp, -rmx, -rmy]) if med == 0 else np.concatenate([rvx, rvy, -rs1, -rs2, -rs3])
        elif med == 0:
            k = np.concatenate([stiff * rp, irho * rmx, irho * rmy])
        else:
            k = np.concatenate([irho * rvx, irho * rvy, stiff * rs1 + lam * rs2, lam * rs1 + stiff * rs2,
                                tmu * rs3])
        out[ext_off[c]:ext_off[c + 1]] = k
    return out
