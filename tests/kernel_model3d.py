"""NumPy model of the three-dimensional stage kernels' arithmetic (stage3d.h), driven by the host
plan that libhho.so exports through include/hho_inspect.h (hho_inspect3d_create; no GPU needed).

Used by the CPU tests to check the library's three-dimensional host side (shape classes and
their face frames, class tables, face links, face-solve coefficients, materials) against the
three-dimensional FP64 oracle before any kernel runs: the stage derivative k = M^{-1}(-K_eff U)
assembled from the tables must equal the oracle's.
"""
import numpy as np

R2 = 1.0 / np.sqrt(2.0)


_DEG = (0, 1, 1, 1, 2, 2, 2, 2, 2, 2)
_DEGF = (0, 1, 1, 2, 2, 2)


def _unpack_pooled(t, off, N, F, nF):
    """Dense tables from a pooled (packed) table: the entries of B_x, B_y, B_z with deg(b) < deg(r),
    the upper triangle of S, the entries of G_j with deg(psi_i) <= deg(phi_a), the normals."""
    pos = off
    B = []
    for _ in range(3):
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
                if _DEGF[i] <= _DEG[a]:
                    G[j, a, i] = t[pos]
                    pos += 1
    return B, Sm, G, t[pos:pos + 3 * nF].reshape(nF, 3)


def _tables(ins, ic, nF, pooled=False):
    N, F = ins.N, ins.F
    off = int(ins.ic_tab[ic])
    t = ins.tables
    if pooled:
        return _unpack_pooled(t, off, N, F, nF)
    B = [t[off + d * N * N: off + (d + 1) * N * N].reshape(N, N) for d in range(3)]
    Sm = t[off + 3 * N * N: off + 4 * N * N].reshape(N, N)
    g0 = off + 4 * N * N
    G = t[g0: g0 + nF * N * F].reshape(nF, N, F)
    nrm = t[g0 + nF * N * F: g0 + nF * N * F + 3 * nF].reshape(nF, 3)
    return B, Sm, G, nrm


def stage_derivative(ins, mesh, U):
    """k = M^{-1}(-K_eff U) for the external state U, following the kernel's algebra."""
    N = ins.N
    med = np.asarray(mesh["medium"])
    nc = len(med)
    rows = np.where(med == 0, 4, 9)
    off = np.concatenate([[0], np.cumsum(rows * N)])
    group_of_ic = -np.ones(ins.n_ic, int)
    for g in range(ins.n_groups):
        b, n = ins.groups[g, 3], ins.groups[g, 4]
        group_of_ic[b:b + n] = g
    cell_of_ic = -np.ones(ins.n_ic, int)
    cell_of_ic[ins.ic_of_cell] = np.arange(nc)
    state, tabs, own = {}, {}, {}
    for c in range(nc):
        ic = ins.ic_of_cell[c]
        g = group_of_ic[ic]
        nF = int(ins.groups[g, 1])
        state[ic] = U[off[c]:off[c + 1]].reshape(rows[c], N)
        tabs[ic] = _tables(ins, ic, nF, bool(ins.pooled[g]))
    tau = ins.mat[2]
    itau = ins.mat[5]
    # outgoing contributions of every cell on its own faces
    for c in range(nc):
        ic = ins.ic_of_cell[c]
        B, Sm, G, nrm = tabs[ic]
        y = state[ic]
        out = []
        for j in range(G.shape[0]):
            n = nrm[j]
            lk = ins.link[j, ic]
            if med[c] == 0:
                q = tau[ic] * y[0] - n[0] * y[1] - n[1] * y[2] - n[2] * y[3]
                out.append(G[j].T @ q)
            else:
                sxy, sxz, syz = R2 * y[6], R2 * y[7], R2 * y[8]
                t = [y[3] * n[0] + sxy * n[1] + sxz * n[2], sxy * n[0] + y[4] * n[1] + syz * n[2],
                     sxz * n[0] + syz * n[1] + y[5] * n[2]]
                w = itau[ic] if (lk >= 0 and (lk >> 3) & 1) else 1.0
                out.append(np.stack([w * (G[j].T @ (tau[ic] * y[cc] - t[cc])) for cc in range(3)]))
        own[ic] = out
    K = np.zeros_like(U)
    for c in range(nc):
        ic = ins.ic_of_cell[c]
        B, Sm, G, nrm = tabs[ic]
        y = state[ic]
        t_ = tau[ic]
        irho, stiff, lam, tmu = ins.mat[0, ic], ins.mat[1, ic], ins.mat[3, ic], ins.mat[4, ic]
        if med[c] == 0:
            p, m = y[0], y[1:4]
            rm = [B[d] @ p for d in range(3)]
            rp = -sum(B[d].T @ m[d] for d in range(3)) - t_ * (Sm @ p)
            for j in range(G.shape[0]):
                lk = ins.link[j, ic]
                if lk < 0:
                    continue
                icn, jn, itf = lk >> 4, lk & 7, (lk >> 3) & 1
                r = own[ic][j]
                rn = own[icn][jn]
                n = nrm[j]
                pF = (r + rn) * ins.c0[j, ic] if not itf else (r + n[0] * rn[0] + n[1] * rn[1] + n[2] * rn[2]) * ins.c0[j, ic]
                w = G[j] @ pF
                for d in range(3):
                    rm[d] = rm[d] + n[d] * w
                rp = rp + t_ * w
            k = np.concatenate([stiff * rp] + [irho * r for r in rm])
        else:
            v, s = y[0:3], y[3:9]
            h4, h5, h6 = R2 * s[3], R2 * s[4], R2 * s[5]
            rs = [B[0] @ v[0], B[1] @ v[1], B[2] @ v[2], R2 * (B[1] @ v[0] + B[0] @ v[1]),
                  R2 * (B[2] @ v[0] + B[0] @ v[2]), R2 * (B[2] @ v[1] + B[1] @ v[2])]
            rv = [-(B[0].T @ s[0] + B[1].T @ h4 + B[2].T @ h5) - t_ * (Sm @ v[0]),
                  -(B[0].T @ h4 + B[1].T @ s[1] + B[2].T @ h6) - t_ * (Sm @ v[1]),
                  -(B[0].T @ h5 + B[1].T @ h6 + B[2].T @ s[2]) - t_ * (Sm @ v[2])]
            for j in range(G.shape[0]):
                lk = ins.link[j, ic]
                if lk < 0:
                    continue
                icn, jn, itf = lk >> 4, lk & 7, (lk >> 3) & 1
                n = nrm[j]
                r = own[ic][j] if not itf else own[ic][j] / itau[ic]  # own r_s without the 1/tau scaling
                rn = own[icn][jn]
                if not itf:
                    vF = (r + rn) * ins.c0[j, ic]
                else:
                    pF = (rn - (n[0] * r[0] + n[1] * r[1] + n[2] * r[2]) * itau[ic]) * ins.c0[j, ic]
                    vF = np.stack([(r[cc] + n[cc] * pF) * itau[ic] for cc in range(3)])
                w = [G[j] @ vF[cc] for cc in range(3)]
                rs[0] = rs[0] + n[0] * w[0]
                rs[1] = rs[1] + n[1] * w[1]
                rs[2] = rs[2] + n[2] * w[2]
                rs[3] = rs[3] + R2 * (n[1] * w[0] + n[0] * w[1])
                rs[4] = rs[4] + R2 * (n[2] * w[0] + n[0] * w[2])
                rs[5] = rs[5] + R2 * (n[2] * w[1] + n[1] * w[2])
                for cc in range(3):
                    rv[cc] = rv[cc] + t_ * w[cc]
            tr = lam * (rs[0] + rs[1] + rs[2])
            k = np.concatenate([irho * rv[0], irho * rv[1], irho * rv[2], tr + tmu * rs[0], tr + tmu * rs[1],
                                tr + tmu * rs[2], tmu * rs[3], tmu * rs[4], tmu * rs[5]])
        K[off[c]:off[c + 1]] = k
    return K
