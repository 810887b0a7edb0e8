// HIP kernels (gfx950) of one explicit Runge-Kutta stage of the HHO elasto-acoustic
// semi-discretisation in three dimensions (tetrahedra and hexahedra), face unknowns eliminated
// (Sec. 4.2, eq. ex_solve; the method of Sec. 2-3 with d = 3).
//
// Same organisation as the two-dimensional stage (kernels.hip): one lane per (cell, shot),
// workgroups of one (medium, shape class) group whose class table is read through scalar loads,
// per-lane arrays [row][lane] in one arena addressed by a buffer resource, and the face
// coupling exchanged through trace buffers [slot = 3 j + c][lane][mode]: every lane stores the
// contributions of its own faces and gathers its neighbours'.  Differences:
//   * state rows: fluid [p | m_x | m_y | m_z], solid [v_x | v_y | v_z | s_1 .. s_6], N each, with
//     s_1..s_3 the diagonal and s_4..s_6 the (xy, xz, yz) components of the stress in the
//     Frobenius-orthonormal basis of symmetric tensors (E_ij = (e_i e_j + e_j e_i) / sqrt 2);
//   * F = (k+1)(k+2)/2 face modes in a face basis defined by the face itself (both cells of a
//     face use the same one), so neighbour contributions need no orientation flip;
//   * class table: B_x, B_y, B_z, S (N x N), then G_j (N x F) and the outward normal n_j (3
//     values) of every face.
// Included by kernels3d_k1/2/3.hip, one translation unit per degree (compiled in parallel).
// Per stage and lane:
//   r_T = tau G^T u - G^T (flux . n) per face (flux: m for the fluid, the stress for the solid),
//   same medium  u_F = (r_T + r_T') / (tau_T + tau_T'),
//   interface    tau_f p_F - n_f . v_F = r_f,  tau_s v_F + n_f p_F = r_s,
//   cell residual (the weak form of eq. HHO1 / HHO2), k = M^{-1} R, Runge-Kutta combine (eq. ERK).
#pragma once

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace hho {
namespace {

template <int K>
struct Dim3 {
    static constexpr int N = (K + 1) * (K + 2) * (K + 3) / 6;
    static constexpr int F = (K + 1) * (K + 2) / 2;
};

// Total degree of the functions of the graded three-dimensional cell basis and of the graded
// face basis (degree-major orders).
constexpr int kDeg3[20] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3};
constexpr int kDegF3[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
// B_d[r][b] can be nonzero only when deg(b) < deg(r); G_j[a][i] only when deg(psi_i) <= deg(phi_a)
// (exact zeros in the host plan; the products are dropped at compile time).
__device__ constexpr bool b3_nonzero(int r, int b) { return kDeg3[b] < kDeg3[r]; }
__device__ constexpr bool g3_nonzero(int a, int i) { return kDegF3[i] <= kDeg3[a]; }

// Class tables: dense for the shared tables (B_x, B_y, B_z, S: N x N row-major; per face G_j
// N x F and n_j, 3 values), packed for the per-cell tables of pooled groups: the entries of B_x, B_y,
// B_z with deg(b) < deg(r), the upper triangle of S, per face the entries of G_j with
// deg(psi_i) <= deg(phi_a), then the normals.  Tab3 reads either layout by compile-time indices.
template <int K>
struct Packed3 {
    static constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
    static constexpr int count_b() {
        int c = 0;
        for (int r = 0; r < N; ++r)
            for (int b = 0; b < N; ++b) c += kDeg3[b] < kDeg3[r];
        return c;
    }
    static constexpr int count_g() {
        int c = 0;
        for (int a = 0; a < N; ++a)
            for (int i = 0; i < F; ++i) c += kDegF3[i] <= kDeg3[a];
        return c;
    }
    static constexpr int nB = count_b(), nS = N * (N + 1) / 2, nG = count_g();
    static constexpr int bidx(int r, int b) {
        int c = 0;
        for (int rr = 0; rr < N; ++rr)
            for (int bb = 0; bb < N; ++bb) {
                if (rr == r && bb == b) return c;
                c += kDeg3[bb] < kDeg3[rr];
            }
        return -1;
    }
    static constexpr int sidx(int r, int b) {
        const int lo = r < b ? r : b, hi = r < b ? b : r;
        return lo * N - lo * (lo - 1) / 2 + (hi - lo);
    }
    static constexpr int gidx(int a, int i) {
        int c = 0;
        for (int aa = 0; aa < N; ++aa)
            for (int ii = 0; ii < F; ++ii) {
                if (aa == a && ii == i) return c;
                c += kDegF3[ii] <= kDeg3[aa];
            }
        return -1;
    }
};

template <int K, typename R, bool PACKED>
struct Tab3 {
    static constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
    using P = Packed3<K>;
    const HHO_CONST R *t;
    int nF;  // faces of the table layout
    __device__ __forceinline__ R b(int d, int r, int c) const {
        return PACKED ? t[d * P::nB + P::bidx(r, c)] : t[d * N * N + r * N + c];
    }
    __device__ __forceinline__ R s(int r, int c) const {
        return PACKED ? t[3 * P::nB + P::sidx(r, c)] : t[3 * N * N + r * N + c];
    }
    __device__ __forceinline__ R g(int j, int a, int i) const {
        return PACKED ? t[3 * P::nB + P::nS + j * P::nG + P::gidx(a, i)] : t[4 * N * N + (j * N + a) * F + i];
    }
    __device__ __forceinline__ R n(int j, int c) const {
        return PACKED ? t[3 * P::nB + P::nS + nF * P::nG + 3 * j + c] : t[4 * N * N + nF * N * F + 3 * j + c];
    }
};

// Stage input Y_i = U^n + D_{i-1} (U^n on the first stage).
template <int ND, typename R>
__device__ __forceinline__ void load_state3(const StageArgs<R> &a, const Bufs<R> &B, unsigned boff, R *y) {
    if (a.first) {
#pragma unroll
        for (int r = 0; r < ND; ++r) y[r] = bld<R>(B.r, boff, B.yin + r * B.rowb);
    } else {
#pragma unroll
        for (int r = 0; r < ND; ++r) y[r] = bld<R>(B.r, boff, B.u + r * B.rowb) + bld<R>(B.r, boff, B.yin + r * B.rowb);
    }
}

// Runge-Kutta combine (eq. ERK) in the increment form of the two-dimensional stage: before the
// last stage D_i = cY D_{i-1} + ck dt k_i (and the partial sum Q), on the last stage
// U^{n+1} = U^n + Q + cd D_{s-2} + cb dt k_s.  CHUNKED (launches with shared tables): U^n is read
// again in every stage, the first included, so that the stage input is not held in registers
// through the residual, and the rows are combined a third (solid) or a quarter (fluid) at a
// time, so that at most that share of U^n, D_{i-1} and Q is in registers at once beside k_i.
// Otherwise (pooled launches, one wave per SIMD, where the loads of later chunks would wait
// behind the stores of earlier ones) every row at once, U^n taken from the stage input y on the
// first stage.
template <int ND, typename R, int POL, bool CHUNKED>
__device__ __forceinline__ void rk_update3(const StageArgs<R> &a, const Bufs<R> &B, unsigned boff, const R *y,
                                           const R *kv, R *out, int shot) {
    const R dt = R(shot_dt(a, shot));
    if constexpr (!CHUNKED) {
        R u[ND], din[ND];
        if (a.first) {
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                u[r] = y[r];
                din[r] = R(0);
            }
        } else {
            const bool need_d = a.last ? a.cd != R(0) : (a.cY != R(0) || a.q_write);
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                u[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
                din[r] = need_d ? bld<R>(B.r, boff, B.yin + r * B.rowb) : R(0);
            }
        }
        if (!a.last) {
            const R ckdt = a.ck * dt;
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                const R d = a.cY * din[r] + ckdt * kv[r];
                bst<POL>(B.r, boff, B.yout + r * B.rowb, d);
                if (a.q_write) bst<POL>(B.r, boff, B.yq + r * B.rowb, a.qa * din[r] + a.qb * d);
                out[r] = u[r] + d;
            }
        } else {
            R q[ND];
#pragma unroll
            for (int r = 0; r < ND; ++r) q[r] = a.q_read ? bld<R>(B.r, boff, B.yq + r * B.rowb) : R(0);
            const R cb = a.cb * dt;
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                out[r] = u[r] + (q[r] + a.cd * din[r] + cb * kv[r]);
                bst<POL>(B.r, boff, B.u + r * B.rowb, out[r]);
            }
        }
    } else {
        const bool need_d = !a.first && (a.last ? a.cd != R(0) : (a.cY != R(0) || a.q_write));
        constexpr int CH = ND % 3 == 0 ? ND / 3 : ND / 4;
        static_assert(ND % CH == 0, "whole chunks");
#pragma unroll
        for (int c0 = 0; c0 < ND; c0 += CH) {
            R u[CH], din[CH];
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                u[r] = bld<R>(B.r, boff, B.u + (c0 + r) * B.rowb);
                din[r] = need_d ? bld<R>(B.r, boff, B.yin + (c0 + r) * B.rowb) : R(0);
            }
            if (!a.last) {
                const R ckdt = a.ck * dt;
#pragma unroll
                for (int r = 0; r < CH; ++r) {
                    const R d = a.cY * din[r] + ckdt * kv[c0 + r];
                    bst<POL>(B.r, boff, B.yout + (c0 + r) * B.rowb, d);
                    if (a.q_write) bst<POL>(B.r, boff, B.yq + (c0 + r) * B.rowb, a.qa * din[r] + a.qb * d);
                    out[c0 + r] = u[r] + d;
                }
            } else {
                R q[CH];
#pragma unroll
                for (int r = 0; r < CH; ++r)
                    q[r] = a.q_read ? bld<R>(B.r, boff, B.yq + (c0 + r) * B.rowb) : R(0);
                const R cb = a.cb * dt;
#pragma unroll
                for (int r = 0; r < CH; ++r) {
                    out[c0 + r] = u[r] + (q[r] + a.cd * din[r] + cb * kv[c0 + r]);
                    bst<POL>(B.r, boff, B.u + (c0 + r) * B.rowb, out[c0 + r]);
                }
            }
        }
    }
}

// One incoming contribution (F modes) of the neighbour across face j, component c.
template <int F, typename R>
__device__ __forceinline__ void gather3(const Bufs<R> &B, int S, int shot, int link, int c, R *v) {
    const int jn = link & 7;
    const unsigned nb = (unsigned)((link >> 4) * S + shot) * (unsigned)sizeof(R);
    bldv<F, R>(B.r, F * nb, B.tin + (jn * 3 + c) * F * B.rowb, v);
}

// ------------------------------------------------------------------------- outgoing traces
template <int K, int NF, typename R, int POL = 0, bool PK = false>
__device__ __forceinline__ void fluid_traces3(const Bufs<R> &B, const Tab3<K, R, PK> &T, const int *lk,
                                              unsigned boff, const R *p, const R *mx, const R *my, const R *mz,
                                              R tau) {
    constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
        const R nx = T.n(j, 0), ny = T.n(j, 1), nz = T.n(j, 2);
        R o[F];
#pragma unroll
        for (int i = 0; i < F; ++i) o[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R q = tau * p[b] - nx * mx[b] - ny * my[b] - nz * mz[b];
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (g3_nonzero(b, i)) o[i] += T.g(j, b, i) * q;
        }
        bstv<F, R, POL>(B.r, F * boff, B.tout + (j * 3) * F * B.rowb, o);
    }
}

// (sigma n)_c of the stress rows at basis function b (s4..s6 carry the 1/sqrt 2 of E_ij)
template <typename R>
__device__ __forceinline__ void stress_n(const R *s, int N, int b, R nx, R ny, R nz, R &tx, R &ty, R &tz) {
    const R r2 = R(kRsqrt2);
    const R sxy = r2 * s[3 * N + b], sxz = r2 * s[4 * N + b], syz = r2 * s[5 * N + b];
    tx = s[b] * nx + sxy * ny + sxz * nz;
    ty = sxy * nx + s[N + b] * ny + syz * nz;
    tz = sxz * nx + syz * ny + s[2 * N + b] * nz;
}

template <int K, int NF, typename R, int POL = 0, bool PK = false>
__device__ __forceinline__ void solid_traces3(const Bufs<R> &B, const Tab3<K, R, PK> &T, const int *lk,
                                              unsigned boff, const R *v, const R *s, R tau, R itau) {
    constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
        const R nx = T.n(j, 0), ny = T.n(j, 1), nz = T.n(j, 2);
        R o[3][F];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < F; ++i) o[c][i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R tx, ty, tz;
            stress_n(s, N, b, nx, ny, nz, tx, ty, tz);
            const R q[3] = {tau * v[b] - tx, tau * v[N + b] - ty, tau * v[2 * N + b] - tz};
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g3_nonzero(b, i)) continue;
                const R g = T.g(j, b, i);
#pragma unroll
                for (int c = 0; c < 3; ++c) o[c][i] += g * q[c];
            }
        }
        // across the interface the fluid side needs r_s / tau_s
        const R w = ((lk[j] >> 3) & 1) ? itau : R(1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int i = 0; i < F; ++i) o[c][i] *= w;
            bstv<F, R, POL>(B.r, F * boff, B.tout + (j * 3 + c) * F * B.rowb, o[c]);
        }
    }
}

// ------------------------------------------------------------------------- fluid cells
template <int K, int NF, typename R, int POL, bool PK>
__device__ __forceinline__ double fluid_stage3(const StageArgs<R> &a, const Bufs<R> &B, const Tab3<K, R, PK> &T, int nF,
                                               const LaneInfo &L, bool want_e) {
    constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    int lk[NF];
    R cc[NF];
    load_links<NF, R>(B, nF, ic, lk, cc);
    R y[4 * N];
    load_state3<4 * N, R>(a, B, boff, y);
    const R *p = y, *m[3] = {y + N, y + 2 * N, y + 3 * N};
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R kap = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    R rp[N], rm[3][N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R sd = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R sx = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                if (b3_nonzero(r, b)) sx += T.b(d, r, b) * p[b];
                if (b3_nonzero(b, r)) sd += T.b(d, b, r) * m[d][b];
            }
            rm[d][r] = sx;
        }
        R st = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) st += T.s(r, b) * p[b];
        rp[r] = -sd - tau * st;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: p_F = 0
        const R nx = T.n(j, 0), ny = T.n(j, 1), nz = T.n(j, 2);
        const bool itf = (lk[j] >> 3) & 1;
        R rn0[F], rn1[F], rn2[F];
        gather3<F, R>(B, a.S, shot, lk[j], 0, rn0);
        if (itf) {
            gather3<F, R>(B, a.S, shot, lk[j], 1, rn1);
            gather3<F, R>(B, a.S, shot, lk[j], 2, rn2);
        }
        R r[F];
#pragma unroll
        for (int i = 0; i < F; ++i) r[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R q = tau * p[b] - nx * m[0][b] - ny * m[1][b] - nz * m[2][b];
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (g3_nonzero(b, i)) r[i] += T.g(j, b, i) * q;
        }
        R pF[F];
        if (!itf) {
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + rn0[i]) * cc[j];
        } else {
            // neighbour solid, its contribution divided by tau_s: eliminate v_F
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + nx * rn0[i] + ny * rn1[i] + nz * rn2[i]) * cc[j];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R w = 0;
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (g3_nonzero(b, i)) w += T.g(j, b, i) * pF[i];
            rm[0][b] += nx * w;
            rm[1][b] += ny * w;
            rm[2][b] += nz * w;
            rp[b] += tau * w;
        }
    }
    // point sources (pressure): R(t) amp d_x phi(x_s)
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &sr = a.src[e];
            if (sr.shot == shot) {
                const R w = R(sr.amp * ricker(stage_time(a, shot), sr.f0, sr.t0) * sr.dirx);
#pragma unroll
                for (int b = 0; b < N; ++b) rp[b] += w * R(sr.phi[b]);
            }
            e = sr.next;
        }
    }
    R kv[4 * N], nw[4 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        kv[b] = kap * rp[b];
        kv[N + b] = irho * rm[0][b];
        kv[2 * N + b] = irho * rm[1][b];
        kv[3 * N + b] = irho * rm[2][b];
    }
    rk_update3<4 * N, R, POL, !PK>(a, B, boff, y, kv, nw, shot);
    fluid_traces3<K, NF, R, POL, PK>(B, T, lk, boff, nw, nw + N, nw + 2 * N, nw + 3 * N, tau);
    double energy = 0.0;
    if (a.last && want_e) {
        double sp = 0, sm = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            sp += (double)nw[b] * (double)nw[b];
#pragma unroll
            for (int d = 1; d <= 3; ++d) sm += (double)nw[d * N + b] * (double)nw[d * N + b];
        }
        energy = 0.5 * (a.emat[(long long)nic + ic] * sp + a.emat[ic] * sm);
    }
    if (a.last && a.rec_first) {
        const int step = uni(a.clock)->step;
        for (int e = a.rec_first[ic]; e >= 0;) {
            const RecDev &rc = a.rec[e];
            double v = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) v += rc.phi[b] * (double)nw[b];
            if (step < a.rec_steps) {
                double *o = a.rec_out + (((long long)shot * a.rec_steps + step) * a.nrec + rc.r) * a.rec_w;
                o[0] = v;
                o[1] = 0.0;
                o[2] = 0.0;
            }
            e = rc.next;
        }
    }
    return energy;
}

// ------------------------------------------------------------------------- solid cells
template <int K, int NF, typename R, int POL, bool PK>
__device__ __forceinline__ double solid_stage3(const StageArgs<R> &a, const Bufs<R> &B, const Tab3<K, R, PK> &T, int nF,
                                               const LaneInfo &L, bool want_e) {
    constexpr int N = Dim3<K>::N, F = Dim3<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    const R r2 = R(kRsqrt2);
    int lk[NF];
    R cc[NF];
    load_links<NF, R>(B, nF, ic, lk, cc);
    R y[9 * N];
    load_state3<9 * N, R>(a, B, boff, y);
    const R *v = y, *s = y + 3 * N;
    const R *vx = v, *vy = v + N, *vz = v + 2 * N;
    const R *s1 = s, *s2 = s + N, *s3 = s + 2 * N, *s4 = s + 3 * N, *s5 = s + 4 * N, *s6 = s + 5 * N;
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R itau = bld<R>(B.r, coff, B.mat + kInvTau * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    const R l2m = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R lam = bld<R>(B.r, coff, B.mat + kLam * B.crowb);
    const R tmu = bld<R>(B.r, coff, B.mat + kTwoMu * B.crowb);
    R rv[3][N], rs[6][N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, bx = 0, by = 0, bz = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            if (b3_nonzero(r, b)) {
                const R X = T.b(0, r, b), Y = T.b(1, r, b), Z = T.b(2, r, b);
                a1 += X * vx[b];
                a2 += Y * vy[b];
                a3 += Z * vz[b];
                a4 += Y * vx[b] + X * vy[b];
                a5 += Z * vx[b] + X * vz[b];
                a6 += Z * vy[b] + Y * vz[b];
            }
            if (b3_nonzero(b, r)) {
                const R X = T.b(0, b, r), Y = T.b(1, b, r), Z = T.b(2, b, r);
                const R h4 = r2 * s4[b], h5 = r2 * s5[b], h6 = r2 * s6[b];
                bx += X * s1[b] + Y * h4 + Z * h5;
                by += X * h4 + Y * s2[b] + Z * h6;
                bz += X * h5 + Y * h6 + Z * s3[b];
            }
        }
        R sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R w = T.s(r, b);
            sx += w * vx[b];
            sy += w * vy[b];
            sz += w * vz[b];
        }
        rs[0][r] = a1;
        rs[1][r] = a2;
        rs[2][r] = a3;
        rs[3][r] = r2 * a4;
        rs[4][r] = r2 * a5;
        rs[5][r] = r2 * a6;
        rv[0][r] = -bx - tau * sx;
        rv[1][r] = -by - tau * sy;
        rv[2][r] = -bz - tau * sz;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: v_F = 0
        const R nx = T.n(j, 0), ny = T.n(j, 1), nz = T.n(j, 2);
        const bool itf = (lk[j] >> 3) & 1;
        R rn[3][F];
        gather3<F, R>(B, a.S, shot, lk[j], 0, rn[0]);
        if (!itf) {
            gather3<F, R>(B, a.S, shot, lk[j], 1, rn[1]);
            gather3<F, R>(B, a.S, shot, lk[j], 2, rn[2]);
        }
        R rc[3][F];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < F; ++i) rc[c][i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R tx, ty, tz;
            stress_n(s, N, b, nx, ny, nz, tx, ty, tz);
            const R q[3] = {tau * vx[b] - tx, tau * vy[b] - ty, tau * vz[b] - tz};
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g3_nonzero(b, i)) continue;
                const R g = T.g(j, b, i);
#pragma unroll
                for (int c = 0; c < 3; ++c) rc[c][i] += g * q[c];
            }
        }
        R vF[3][F];
        if (!itf) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < F; ++i) vF[c][i] = (rc[c][i] + rn[c][i]) * cc[j];
        } else {
            // neighbour fluid: eliminate p_F, then v_F
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const R pF = (rn[0][i] - (nx * rc[0][i] + ny * rc[1][i] + nz * rc[2][i]) * itau) * cc[j];
                vF[0][i] = (rc[0][i] + nx * pF) * itau;
                vF[1][i] = (rc[1][i] + ny * pF) * itau;
                vF[2][i] = (rc[2][i] + nz * pF) * itau;
            }
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R wx = 0, wy = 0, wz = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g3_nonzero(b, i)) continue;
                const R g = T.g(j, b, i);
                wx += g * vF[0][i];
                wy += g * vF[1][i];
                wz += g * vF[2][i];
            }
            rs[0][b] += nx * wx;
            rs[1][b] += ny * wy;
            rs[2][b] += nz * wz;
            rs[3][b] += r2 * (ny * wx + nx * wy);
            rs[4][b] += r2 * (nz * wx + nx * wz);
            rs[5][b] += r2 * (nz * wy + ny * wz);
            rv[0][b] += tau * wx;
            rv[1][b] += tau * wy;
            rv[2][b] += tau * wz;
        }
    }
    // point forces: R(t) amp d phi(x_s) on the velocity rows
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &sr = a.src[e];
            if (sr.shot == shot) {
                const double w = sr.amp * ricker(stage_time(a, shot), sr.f0, sr.t0);
                const R wx = R(w * sr.dirx), wy = R(w * sr.diry), wz = R(w * sr.dirz);
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    rv[0][b] += wx * R(sr.phi[b]);
                    rv[1][b] += wy * R(sr.phi[b]);
                    rv[2][b] += wz * R(sr.phi[b]);
                }
            }
            e = sr.next;
        }
    }
    R kv[9 * N], nw[9 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        kv[b] = irho * rv[0][b];
        kv[N + b] = irho * rv[1][b];
        kv[2 * N + b] = irho * rv[2][b];
        const R tr = lam * (rs[0][b] + rs[1][b] + rs[2][b]);
        kv[3 * N + b] = tr + tmu * rs[0][b];
        kv[4 * N + b] = tr + tmu * rs[1][b];
        kv[5 * N + b] = tr + tmu * rs[2][b];
        kv[6 * N + b] = tmu * rs[3][b];
        kv[7 * N + b] = tmu * rs[4][b];
        kv[8 * N + b] = tmu * rs[5][b];
    }
    (void)l2m;
    rk_update3<9 * N, R, POL, !PK>(a, B, boff, y, kv, nw, shot);
    solid_traces3<K, NF, R, POL, PK>(B, T, lk, boff, nw, nw + 3 * N, tau, itau);
    double energy = 0.0;
    if (a.last && want_e) {
        const double ca = a.emat[(long long)nic + ic], cb = a.emat[(long long)2 * nic + ic];
        const double c3 = a.emat[(long long)3 * nic + ic];
        double sv = 0, ss = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const double x1 = nw[3 * N + b], x2 = nw[4 * N + b], x3 = nw[5 * N + b];
            const double x4 = nw[6 * N + b], x5 = nw[7 * N + b], x6 = nw[8 * N + b];
            sv += (double)nw[b] * (double)nw[b] + (double)nw[N + b] * (double)nw[N + b] +
                  (double)nw[2 * N + b] * (double)nw[2 * N + b];
            ss += ca * (x1 * x1 + x2 * x2 + x3 * x3) + 2.0 * cb * (x1 * x2 + x1 * x3 + x2 * x3) +
                  c3 * (x4 * x4 + x5 * x5 + x6 * x6);
        }
        energy = 0.5 * (a.emat[ic] * sv + ss);
    }
    if (a.last && a.rec_first) {
        const int step = uni(a.clock)->step;
        for (int e = a.rec_first[ic]; e >= 0;) {
            const RecDev &rc = a.rec[e];
            double v0 = 0, v1 = 0, v2 = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                v0 += rc.phi[b] * (double)nw[b];
                v1 += rc.phi[b] * (double)nw[N + b];
                v2 += rc.phi[b] * (double)nw[2 * N + b];
            }
            if (step < a.rec_steps) {
                double *o = a.rec_out + (((long long)shot * a.rec_steps + step) * a.nrec + rc.r) * a.rec_w;
                o[0] = v0;
                o[1] = v1;
                o[2] = v2;
            }
            e = rc.next;
        }
    }
    return energy;
}

template <int K, int NF, typename R, int POL, bool POOLED>
__device__ __forceinline__ double stage_body3(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L, bool want_e) {
    const Tab3<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    if (G.medium == kFluid) return fluid_stage3<K, NF, R, POL, POOLED>(a, B, T, G.nF, L, want_e);
    return solid_stage3<K, NF, R, POL, POOLED>(a, B, T, G.nF, L, want_e);
}

// Stage launch; with pooled groups two launches over the same grid as in two dimensions.
template <int K, typename R, int POL, bool POOLED>
__device__ __forceinline__ void stage_entry3(const StageArgs<R> &a) {
    if ((!POOLED || a.all_pooled) && a.last && a.clock_next && blockIdx.x == 0 && threadIdx.x == 0) {
        Clock c = *a.clock;
        c.step += 1;
        *a.clock_next = c;
    }
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if ((POOLED || a.has_pooled) && (G.pooled != 0) != POOLED) return;
    const bool want_e = a.last && a.e_part;
    double e = 0.0;
    if (L.active) {
        if (G.nF <= 4) e = stage_body3<K, 4, R, POL, POOLED>(a, G, L, want_e);
        else e = stage_body3<K, 6, R, POL, POOLED>(a, G, L, want_e);
    }
    if (want_e) block_energy(e, a.S, a.cpb, energy_slot(a));
}

template <int K, typename R, int POL, bool POOLED = false>
__global__ __launch_bounds__(kBlock) void stage_kernel3(StageArgs<R> a) {
    stage_entry3<K, R, POL, POOLED>(a);
}

// The same stage with a lane's registers (VGPRs and AGPRs together) capped at 256, so that two
// waves share a SIMD.
template <int K, typename R, int POL, bool POOLED = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void stage_kernel3_w2(StageArgs<R> a) {
    stage_entry3<K, R, POL, POOLED>(a);
}

template <int K, int NF, typename R, bool POOLED>
__device__ __forceinline__ void traces_body3(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L) {
    constexpr int N = Dim3<K>::N;
    const Tab3<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    int lk[NF];
    load_links<NF, R>(B, G.nF, L.ic, lk, (R *)nullptr);
    const R tau = bld<R>(B.r, L.coff, B.mat + kTau * B.crowb);
    if (G.medium == kFluid) {
        R y[4 * N];
#pragma unroll
        for (int r = 0; r < 4 * N; ++r) y[r] = bld<R>(B.r, L.boff, B.yin + r * B.rowb);
        fluid_traces3<K, NF, R, 0, POOLED>(B, T, lk, L.boff, y, y + N, y + 2 * N, y + 3 * N, tau);
    } else {
        const R itau = bld<R>(B.r, L.coff, B.mat + kInvTau * B.crowb);
        R y[9 * N];
#pragma unroll
        for (int r = 0; r < 9 * N; ++r) y[r] = bld<R>(B.r, L.boff, B.yin + r * B.rowb);
        solid_traces3<K, NF, R, 0, POOLED>(B, T, lk, L.boff, y, y + 3 * N, tau, itau);
    }
}

template <int K, typename R, bool POOLED = false>
__global__ __launch_bounds__(kBlock) void trace_kernel3(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if (!L.active || ((POOLED || a.has_pooled) && (G.pooled != 0) != POOLED)) return;
    if (G.nF <= 4) traces_body3<K, 4, R, POOLED>(a, G, L);
    else traces_body3<K, 6, R, POOLED>(a, G, L);
}

// Energy of the state in a.Yin (Sec. 5.1), float64 partials per block and shot.
template <int K, typename R>
__global__ __launch_bounds__(kBlock) void energy_kernel3(StageArgs<R> a) {
    constexpr int N = Dim3<K>::N;
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    double e = 0.0;
    if (L.active) {
        const int nic = a.n_ic, ic = L.ic;
        const Bufs<R> B = make_bufs(a);
        auto val = [&](int r) { return (double)bld<R>(B.r, L.boff, B.yin + r * B.rowb); };
        if (G.medium == kFluid) {
            double sp = 0, sm = 0;
            for (int b = 0; b < N; ++b) {
                const double p = val(b), x = val(N + b), y = val(2 * N + b), z = val(3 * N + b);
                sp += p * p;
                sm += x * x + y * y + z * z;
            }
            e = 0.5 * (a.emat[(long long)nic + ic] * sp + a.emat[ic] * sm);
        } else {
            const double ca = a.emat[(long long)nic + ic], cb = a.emat[(long long)2 * nic + ic];
            const double c3 = a.emat[(long long)3 * nic + ic];
            double sv = 0, ss = 0;
            for (int b = 0; b < N; ++b) {
                const double v0 = val(b), v1 = val(N + b), v2 = val(2 * N + b);
                const double x1 = val(3 * N + b), x2 = val(4 * N + b), x3 = val(5 * N + b);
                const double x4 = val(6 * N + b), x5 = val(7 * N + b), x6 = val(8 * N + b);
                sv += v0 * v0 + v1 * v1 + v2 * v2;
                ss += ca * (x1 * x1 + x2 * x2 + x3 * x3) + 2.0 * cb * (x1 * x2 + x1 * x3 + x2 * x3) +
                      c3 * (x4 * x4 + x5 * x5 + x6 * x6);
            }
            e = 0.5 * (a.emat[ic] * sv + ss);
        }
    }
    block_energy(e, a.S, a.cpb, a.e_part);
}

}  // namespace

template <int K, typename R>
hipError_t launch_stage3(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    const dim3 grid(n_blocks), block(a.cpb * a.S);
    // float32 shared-table launches capped at two waves per SIMD; pooled launches (per-lane tables
    // in vector registers) and float64 uncapped, where the cap would spill
    if (!a.all_pooled) {
        if constexpr (sizeof(R) == 4) {
            if (a.nt_stores)
                hipLaunchKernelGGL((stage_kernel3_w2<K, R, kNonTemporal>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((stage_kernel3_w2<K, R, 0>), grid, block, 0, st, a);
        } else {
            if (a.nt_stores)
                hipLaunchKernelGGL((stage_kernel3<K, R, kNonTemporal>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((stage_kernel3<K, R, 0>), grid, block, 0, st, a);
        }
    }
    if (a.has_pooled) hipLaunchKernelGGL((stage_kernel3<K, R, 0, true>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_traces3(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    if (!a.all_pooled) hipLaunchKernelGGL((trace_kernel3<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    if (a.has_pooled) hipLaunchKernelGGL((trace_kernel3<K, R, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_energy3(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL((energy_kernel3<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

}  // namespace hho
