// HIP kernels (gfx950) of the discrete adjoint of the explicit Runge-Kutta path, and the
// receiver-misfit gradient with respect to the per-cell materials.
//
// Forward stage (Sec. 4.2, eq. ex_solve): k_i = L Y_i + M^{-1} F(t_i), L = -M^{-1} K_eff.
// Reverse sweep of a step (subdiagonal tableaux of eq. ERK), from lambda = lambda^{n+1}:
//   mu_s = dt b_s lambda,  mu_i = dt b_i lambda + dt a_{i+1,i} Ybar_{i+1},  Ybar_i = L^T mu_i,
//   lambda^n = lambda + sum_i Ybar_i + dJ/dU^n.
// L^T is applied with the forward machinery: K is a skew part (reconstructions eq. rec_a /
// rec_e, the interface coupling) plus the symmetric stabilisation (eq. stab), so
// K^T = D K_c D, where D flips the sign of the dual unknowns (m, s) and K_c is K with the
// interface coupling reversed; hence L^T mu = D R_c(z) with z = D M^{-1} mu and R_c = -K_c,eff
// evaluated by the same face-condensed cell residual as the forward stage.  The lanes keep
// z between stages (and exchange its trace contributions exactly as the forward stage does).
//
// Gradient: mu^T (dL/dtheta) Y = -w^T (dM/dtheta) k - (dtau_T/dtheta) sum_{F in dT}
// (Y_T - Y_F, w_T - W_F)_F with w = M^{-1} mu = D z, Y_F the forward face values of Y (stored
// by the recompute) and W_F the face values of the adjoint face solve: the Schur-complement
// derivative is a bilinear form on the cell-and-face system, and only the mass matrices
// (eq. mass) and the stabilisation weight tau_T depend on the materials.  Accumulated per
// lane in float64.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace hho {
namespace {

// Parameter-derivative slots of StageArgs::gm ([8][n_ic]).
//   fluid: 0 d(1/kappa)/drho, 1 d(1/kappa)/dc, 2 dtau/drho, 3 dtau/dc
//   solid: 0 dtau/drho, 1 dtau/dlambda, 2 dtau/dmu, 3 dA/dlambda (= dB/dlambda),
//          4 dA/dmu, 5 dB/dmu, 6 dC/dmu   (compliance [[A, B, 0], [B, A, 0], [0, 0, C]])

// Forward step whose misfit derivative enters lambda in this launch: a.inject is relative (0 =
// none) to the step offset held by the adjoint clock, which the host sets before each checkpoint
// segment, so that the captured adjoint stages of a segment replay unchanged for every segment.
template <typename R>
__device__ __forceinline__ int inject_step(const StageArgs<R> &a) {
    return a.inject >= 1 ? a.inject + uni(a.clock)->step : 0;
}

template <typename R>
__device__ __forceinline__ double gmv(const StageArgs<R> &a, int slot, int ic) {
    return a.gm[(long long)slot * a.n_ic + ic];
}

__device__ __forceinline__ void add_grad(double *g, long long LT, long long lane, double g0, double g1, double g2) {
    g[lane] += g0;
    g[LT + lane] += g1;
    g[2 * LT + lane] += g2;
}

// lambda and the running sum of L^T mu of one lane (the sum starts at zero on the first
// adjoint stage of a step)
template <int ND, typename R>
__device__ __forceinline__ void load_lambda(const StageArgs<R> &a, const Bufs<R> &B, unsigned boff, R *lam, R *lac) {
    if (a.first) {
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            lam[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
            lac[r] = R(0);
        }
    } else {
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            lam[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
            lac[r] = bld<R>(B.r, boff, B.acc + r * B.rowb);
        }
    }
}

// Read lambda, the running sum and the gradient accumulators at the start of the stage (their
// latency then overlaps the residual) where registers allow; otherwise after the residual.
template <int K, typename R>
constexpr bool kEarlyLambda = sizeof(R) == 4 && K <= 2;

// ------------------------------------------------------------------------- fluid cells
template <int K, int NF, typename R, bool PK>
__device__ __forceinline__ void fluid_adjoint(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T, int nF,
                                              const LaneInfo &L) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    const long long lane = boff / sizeof(R), LT = a.LT;
    int lk[NF];
    R cc[NF], rn[NF][2][F];
    load_links<NF, R>(B, nF, ic, lk, cc);
    R p[N], mx[N], my[N];  // z = D M^{-1} mu
#pragma unroll
    for (int b = 0; b < N; ++b) {
        p[b] = bld<R>(B.r, boff, B.yin + (b)*B.rowb);
        mx[b] = bld<R>(B.r, boff, B.yin + (N + b) * B.rowb);
        my[b] = bld<R>(B.r, boff, B.yin + (2 * N + b) * B.rowb);
    }
    load_incoming<K, NF, R>(B, kFluid, a.S, shot, lk, rn);
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R kap = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    R lam[3 * N], lac[3 * N];
    double g0 = 0, g1 = 0;
    if constexpr (kEarlyLambda<K, R>) {
        load_lambda<3 * N, R>(a, B, boff, lam, lac);
        g0 = a.gacc[lane], g1 = a.gacc[LT + lane];
    }
    // stored forward data of this stage: primal rows of Y, the derivative k, the face values
    R yp[N], yf[NF][F];
    double wk_p = 0, wk_m = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        yp[b] = a.yfwd[(long long)b * LT + lane];
        const R kp = a.kfwd[(long long)b * LT + lane];
        const R kmx = a.kfwd[(long long)(N + b) * LT + lane], kmy = a.kfwd[(long long)(2 * N + b) * LT + lane];
        // w = D z: w_p = p, w_m = -m
        wk_p += (double)p[b] * (double)kp;
        wk_m -= (double)mx[b] * (double)kmx + (double)my[b] * (double)kmy;
    }
    // issued for every face of the group without waiting for the links (the rows of a boundary
    // face hold no values of this stage and are zeroed once the links have arrived)
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int i = 0; i < F; ++i) yf[j][i] = j < nF ? a.ffwd[(long long)((j * 2) * F + i) * LT + lane] : R(0);
    // material derivatives of the gradient terms, read with the other loads
    const double gm0 = gmv(a, 0, ic), gm1 = gmv(a, 1, ic), gm2 = gmv(a, 2, ic), gm3 = gmv(a, 3, ic);
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int i = 0; i < F; ++i)
            if (lk[j] < 0) yf[j][i] = R(0);
    // adjoint residual R_c(z) (interface coupling reversed) and the stabilisation pairing
    R rp[N], rmx[N], rmy[N], tp[N];
#pragma unroll
    for (int b = 0; b < N; ++b) tp[b] = tau * p[b];
    double stab = 0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R sx = 0, sy = 0, sd = 0;
        double ys = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            if (b_nonzero(r, b)) {
                sx += T.bx(r, b) * p[b];
                sy += T.by(r, b) * p[b];
            }
            if (b_nonzero(b, r)) sd += T.bx(b, r) * mx[b] + T.by(b, r) * my[b];
            sd += T.s(r, b) * tp[b];
            ys += (double)T.s(r, b) * (double)p[b];
        }
        rmx[r] = sx;
        rmy[r] = sy;
        rp[r] = -sd;
        stab += (double)yp[r] * ys;  // Y_T^T S w_T  (S = sum over all faces of E_j)
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: face values 0
        const R nx = T.n(j, 0), ny = T.n(j, 1);
        R r[F];
#pragma unroll
        for (int i = 0; i < F; ++i) r[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R q = tp[b] - nx * mx[b] - ny * my[b];
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (g_nonzero(b, i)) r[i] += T.g(j, b, i) * q;
        }
        R pF[F];
        if (!((lk[j] >> 3) & 1)) {
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + rn[j][0][i]) * cc[j];
        } else {
            // interface with the coupling reversed: n_G -> -n_G
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] - nx * rn[j][0][i] - ny * rn[j][1][i]) * cc[j];
        }
        double sj = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R w = 0;
            double gy = 0, gw = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g_nonzero(b, i)) continue;
                w += T.g(j, b, i) * pF[i];
                gy += (double)T.g(j, b, i) * (double)pF[i];
                gw += (double)T.g(j, b, i) * (double)yf[j][i];
            }
            rmx[b] += nx * w;
            rmy[b] += ny * w;
            rp[b] += tau * w;
            sj += (double)yp[b] * gy + (double)p[b] * gw;  // Y_T^T G W_F + w_T^T G Y_F
        }
#pragma unroll
        for (int i = 0; i < F; ++i) sj -= (double)yf[j][i] * (double)pF[i];  // - Y_F . W_F
        stab -= sj;
    }
    // Ybar = D R_c(z)
    R yb[3 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        yb[b] = rp[b];
        yb[N + b] = -rmx[b];
        yb[2 * N + b] = -rmy[b];
    }
    if constexpr (!kEarlyLambda<K, R>) {
        // every load before the first store
        load_lambda<3 * N, R>(a, B, boff, lam, lac);
        g0 = a.gacc[lane], g1 = a.gacc[LT + lane];
    }
    g0 -= gm0 * wk_p + wk_m + gm2 * stab;
    g1 -= gm1 * wk_p + gm3 * stab;
    a.gacc[lane] = g0;
    a.gacc[LT + lane] = g1;
    R mu[3 * N];
    if (!a.last) {
#pragma unroll
        for (int r = 0; r < 3 * N; ++r) {
            const R acc = lac[r] + yb[r];
            bst(B.r, boff, B.acc + r * B.rowb, acc);
            mu[r] = a.mu_b * lam[r] + a.mu_a * yb[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 3 * N; ++r) lam[r] += lac[r] + yb[r];
        const int inj = inject_step(a);
        if (inj >= 1 && a.rec_first) {
            for (int e = a.rec_first[ic]; e >= 0;) {
                const RecDev &rc = a.rec[e];
                double v = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) v += rc.phi[b] * (double)yp[b];
                const double d = a.dobs[(((long long)shot * a.nobs + inj - 1) * a.nrec + rc.r) * 2];
                const double w = uni(a.clock)->dt * (v - d);
#pragma unroll
                for (int b = 0; b < N; ++b) lam[b] += R(w * rc.phi[b]);
                e = rc.next;
            }
        }
#pragma unroll
        for (int r = 0; r < 3 * N; ++r) {
            bst(B.r, boff, B.u + r * B.rowb, lam[r]);
            mu[r] = a.zs_b * lam[r];
        }
    }
    // next adjoint stage input z = D M^{-1} mu and its outgoing traces
    R zp[N], zx[N], zy[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        zp[b] = kap * mu[b];
        zx[b] = -irho * mu[N + b];
        zy[b] = -irho * mu[2 * N + b];
        bst(B.r, boff, B.yout + b * B.rowb, zp[b]);
        bst(B.r, boff, B.yout + (N + b) * B.rowb, zx[b]);
        bst(B.r, boff, B.yout + (2 * N + b) * B.rowb, zy[b]);
    }
    fluid_traces<K, NF, R, 0, PK>(a, B, T, lk, boff, zp, zx, zy, tau);
}

// ------------------------------------------------------------------------- solid cells
template <int K, int NF, typename R, bool PK>
__device__ __forceinline__ void solid_adjoint(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T, int nF,
                                              const LaneInfo &L) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    const long long lane = boff / sizeof(R), LT = a.LT;
    const R r2 = R(kRsqrt2);
    int lk[NF];
    R cc[NF], rn[NF][2][F];
    load_links<NF, R>(B, nF, ic, lk, cc);
    R vx[N], vy[N], s1[N], s2[N], s3[N];  // z = D M^{-1} mu
#pragma unroll
    for (int b = 0; b < N; ++b) {
        vx[b] = bld<R>(B.r, boff, B.yin + (b)*B.rowb);
        vy[b] = bld<R>(B.r, boff, B.yin + (N + b) * B.rowb);
        s1[b] = bld<R>(B.r, boff, B.yin + (2 * N + b) * B.rowb);
        s2[b] = bld<R>(B.r, boff, B.yin + (3 * N + b) * B.rowb);
        s3[b] = bld<R>(B.r, boff, B.yin + (4 * N + b) * B.rowb);
    }
    load_incoming<K, NF, R>(B, kSolid, a.S, shot, lk, rn);
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R itau = bld<R>(B.r, coff, B.mat + kInvTau * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    const R l2m = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R lam_ = bld<R>(B.r, coff, B.mat + kLam * B.crowb);
    const R tmu = bld<R>(B.r, coff, B.mat + kTwoMu * B.crowb);
    R lam[5 * N], lac[5 * N];
    double g0 = 0, g1 = 0, g2 = 0;
    if constexpr (kEarlyLambda<K, R>) {
        load_lambda<5 * N, R>(a, B, boff, lam, lac);
        g0 = a.gacc[lane], g1 = a.gacc[LT + lane], g2 = a.gacc[2 * LT + lane];
    }
    R yx[N], yy[N], yf[NF][2][F];
    double wk_v = 0, P11 = 0, P12 = 0, P21 = 0, P22 = 0, P33 = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        yx[b] = a.yfwd[(long long)b * LT + lane];
        yy[b] = a.yfwd[(long long)(N + b) * LT + lane];
        const double k0 = a.kfwd[(long long)b * LT + lane], k1 = a.kfwd[(long long)(N + b) * LT + lane];
        const double k2 = a.kfwd[(long long)(2 * N + b) * LT + lane];
        const double k3 = a.kfwd[(long long)(3 * N + b) * LT + lane];
        const double k4 = a.kfwd[(long long)(4 * N + b) * LT + lane];
        // w = D z: w_v = v, w_s = -s
        wk_v += (double)vx[b] * k0 + (double)vy[b] * k1;
        P11 -= (double)s1[b] * k2;
        P12 -= (double)s1[b] * k3;
        P21 -= (double)s2[b] * k2;
        P22 -= (double)s2[b] * k3;
        P33 -= (double)s3[b] * k4;
    }
    // issued for every face of the group without waiting for the links (zeroed below for
    // boundary faces, whose rows hold no values of this stage)
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < F; ++i)
                yf[j][c][i] = j < nF ? a.ffwd[(long long)((j * 2 + c) * F + i) * LT + lane] : R(0);
    // material derivatives of the gradient terms, read with the other loads
    double gm[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) gm[q] = gmv(a, q, ic);
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (lk[j] < 0) yf[j][c][i] = R(0);
    R rvx[N], rvy[N], rs1[N], rs2[N], rs3[N], tvx[N], tvy[N], hs3[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        tvx[b] = tau * vx[b];
        tvy[b] = tau * vy[b];
        hs3[b] = r2 * s3[b];
    }
    double stab = 0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R a1 = 0, a2 = 0, a3 = 0, bx = 0, by = 0;
        double yx_s = 0, yy_s = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R srb = T.s(r, b);
            if (b_nonzero(r, b)) {
                const R bxrb = T.bx(r, b), byrb = T.by(r, b);
                a1 += bxrb * vx[b];
                a2 += byrb * vy[b];
                a3 += byrb * vx[b] + bxrb * vy[b];
            }
            if (b_nonzero(b, r)) {
                const R bxbr = T.bx(b, r), bybr = T.by(b, r);
                bx += bxbr * s1[b] + bybr * hs3[b];
                by += bybr * s2[b] + bxbr * hs3[b];
            }
            bx += srb * tvx[b];
            by += srb * tvy[b];
            yx_s += (double)srb * (double)vx[b];
            yy_s += (double)srb * (double)vy[b];
        }
        rs1[r] = a1;
        rs2[r] = a2;
        rs3[r] = r2 * a3;
        rvx[r] = -bx;
        rvy[r] = -by;
        stab += (double)yx[r] * yx_s + (double)yy[r] * yy_s;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
        const R nx = T.n(j, 0), ny = T.n(j, 1);
        R rx[F], ry[F];
#pragma unroll
        for (int i = 0; i < F; ++i) rx[i] = ry[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R qx = tvx[b] - nx * s1[b] - ny * hs3[b];
            const R qy = tvy[b] - nx * hs3[b] - ny * s2[b];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g_nonzero(b, i)) continue;
                rx[i] += T.g(j, b, i) * qx;
                ry[i] += T.g(j, b, i) * qy;
            }
        }
        R vFx[F], vFy[F];
        if (!((lk[j] >> 3) & 1)) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                vFx[i] = (rx[i] + rn[j][0][i]) * cc[j];
                vFy[i] = (ry[i] + rn[j][1][i]) * cc[j];
            }
        } else {
            // interface with the coupling reversed: n_G -> -n_G
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const R pF = (rn[j][0][i] + (nx * rx[i] + ny * ry[i]) * itau) * cc[j];
                vFx[i] = (rx[i] - nx * pF) * itau;
                vFy[i] = (ry[i] - ny * pF) * itau;
            }
        }
        double sj = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R wx = 0, wy = 0;
            double gyx = 0, gyy = 0, gwx = 0, gwy = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g_nonzero(b, i)) continue;
                const R g = T.g(j, b, i);
                wx += g * vFx[i];
                wy += g * vFy[i];
                gyx += (double)g * (double)vFx[i];
                gyy += (double)g * (double)vFy[i];
                gwx += (double)g * (double)yf[j][0][i];
                gwy += (double)g * (double)yf[j][1][i];
            }
            rs1[b] += nx * wx;
            rs2[b] += ny * wy;
            rs3[b] += r2 * (ny * wx + nx * wy);
            rvx[b] += tau * wx;
            rvy[b] += tau * wy;
            sj += (double)yx[b] * gyx + (double)yy[b] * gyy + (double)vx[b] * gwx + (double)vy[b] * gwy;
        }
#pragma unroll
        for (int i = 0; i < F; ++i) sj -= (double)yf[j][0][i] * (double)vFx[i] + (double)yf[j][1][i] * (double)vFy[i];
        stab -= sj;
    }
    R yb[5 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        yb[b] = rvx[b];
        yb[N + b] = rvy[b];
        yb[2 * N + b] = -rs1[b];
        yb[3 * N + b] = -rs2[b];
        yb[4 * N + b] = -rs3[b];
    }
    if constexpr (!kEarlyLambda<K, R>) {
        // every load before the first store
        load_lambda<5 * N, R>(a, B, boff, lam, lac);
        g0 = a.gacc[lane], g1 = a.gacc[LT + lane], g2 = a.gacc[2 * LT + lane];
    }
    g0 -= wk_v + gm[0] * stab;
    g1 -= gm[3] * (P11 + P12 + P21 + P22) + gm[1] * stab;
    g2 -= gm[4] * (P11 + P22) + gm[5] * (P12 + P21) + gm[6] * P33 + gm[2] * stab;
    a.gacc[lane] = g0;
    a.gacc[LT + lane] = g1;
    a.gacc[2 * LT + lane] = g2;
    R mu[5 * N];
    if (!a.last) {
#pragma unroll
        for (int r = 0; r < 5 * N; ++r) {
            bst(B.r, boff, B.acc + r * B.rowb, lac[r] + yb[r]);
            mu[r] = a.mu_b * lam[r] + a.mu_a * yb[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 5 * N; ++r) lam[r] += lac[r] + yb[r];
        const int inj = inject_step(a);
        if (inj >= 1 && a.rec_first) {
            for (int e = a.rec_first[ic]; e >= 0;) {
                const RecDev &rc = a.rec[e];
                double v0 = 0, v1 = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    v0 += rc.phi[b] * (double)yx[b];
                    v1 += rc.phi[b] * (double)yy[b];
                }
                const double *d = a.dobs + (((long long)shot * a.nobs + inj - 1) * a.nrec + rc.r) * 2;
                const double dt = uni(a.clock)->dt;
                const double w0 = dt * (v0 - d[0]), w1 = dt * (v1 - d[1]);
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    lam[b] += R(w0 * rc.phi[b]);
                    lam[N + b] += R(w1 * rc.phi[b]);
                }
                e = rc.next;
            }
        }
#pragma unroll
        for (int r = 0; r < 5 * N; ++r) {
            bst(B.r, boff, B.u + r * B.rowb, lam[r]);
            mu[r] = a.zs_b * lam[r];
        }
    }
    R zx[N], zy[N], z1[N], z2[N], z3[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        zx[b] = irho * mu[b];
        zy[b] = irho * mu[N + b];
        z1[b] = -(l2m * mu[2 * N + b] + lam_ * mu[3 * N + b]);
        z2[b] = -(lam_ * mu[2 * N + b] + l2m * mu[3 * N + b]);
        z3[b] = -tmu * mu[4 * N + b];
        bst(B.r, boff, B.yout + b * B.rowb, zx[b]);
        bst(B.r, boff, B.yout + (N + b) * B.rowb, zy[b]);
        bst(B.r, boff, B.yout + (2 * N + b) * B.rowb, z1[b]);
        bst(B.r, boff, B.yout + (3 * N + b) * B.rowb, z2[b]);
        bst(B.r, boff, B.yout + (4 * N + b) * B.rowb, z3[b]);
    }
    solid_traces<K, NF, R, 0, PK>(a, B, T, lk, boff, zx, zy, z1, z2, z3, tau, itau);
}

template <int K, int NF, typename R, bool POOLED>
__device__ __forceinline__ void adjoint_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L) {
    const Tab<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    if (G.medium == kFluid)
        fluid_adjoint<K, NF, R, POOLED>(a, B, T, G.nF, L);
    else
        solid_adjoint<K, NF, R, POOLED>(a, B, T, G.nF, L);
}

// On a mesh with pooled groups every adjoint launch is two launches over the same grid, as the
// forward stage: POOLED = false for the groups with shared tables, true for the pooled ones; a
// workgroup whose group is of the other kind returns at once.
template <int K, typename R, bool POOLED>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if (!L.active || ((POOLED || a.has_pooled) && (G.pooled != 0) != POOLED)) return;
    if (G.nF <= 4) adjoint_body<K, 4, R, POOLED>(a, G, L);
    else adjoint_body<K, kMaxFaces, R, POOLED>(a, G, L);
}

// Start of the reverse sweep: lambda += dt R^T (R U - d^n) (primal rows of U read from a.yfwd,
// n = inject_step(a); receivers of the lane's cell), then z = D M^{-1}(zs_b lambda) and its outgoing
// traces.
template <int K, int NF, typename R, bool POOLED>
__device__ __forceinline__ void start_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L) {
    constexpr int N = Dim<K>::N;
    const Tab<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    const int ic = L.ic, nb = G.medium == kFluid ? 3 : 5, ncomp = G.medium == kFluid ? 1 : 2;
    const unsigned boff = L.boff, coff = L.coff;
    int lk[NF];
    load_links<NF, R>(B, G.nF, ic, lk, (R *)nullptr);
    R u[2][N], lam[5 * N];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < N; ++b) u[c][b] = c < ncomp ? a.yfwd[(long long)(c * N + b) * a.LT + L.ic * a.S + L.shot] : R(0);
#pragma unroll
    for (int r = 0; r < 5 * N; ++r) lam[r] = r < nb * N ? bld<R>(B.r, boff, B.u + r * B.rowb) : R(0);
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R itau = bld<R>(B.r, coff, B.mat + kInvTau * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    const R stiff = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R lamL = bld<R>(B.r, coff, B.mat + kLam * B.crowb);
    const R tmu = bld<R>(B.r, coff, B.mat + kTwoMu * B.crowb);
    const int inj = inject_step(a);
    if (inj >= 1 && a.rec_first) {
        for (int e = a.rec_first[ic]; e >= 0;) {
            const RecDev &rc = a.rec[e];
            const double *d = a.dobs + (((long long)L.shot * a.nobs + inj - 1) * a.nrec + rc.r) * 2;
            const double dt = uni(a.clock)->dt;
            for (int c = 0; c < ncomp; ++c) {
                double v = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) v += rc.phi[b] * (double)u[c][b];
                const double w = dt * (v - d[c]);
#pragma unroll
                for (int b = 0; b < N; ++b) lam[c * N + b] += R(w * rc.phi[b]);
            }
            e = rc.next;
        }
    }
#pragma unroll
    for (int r = 0; r < 5 * N; ++r)
        if (r < nb * N) bst(B.r, boff, B.u + r * B.rowb, lam[r]);
    R z[5][N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        if (G.medium == kFluid) {
            z[0][b] = stiff * a.zs_b * lam[b];
            z[1][b] = -irho * a.zs_b * lam[N + b];
            z[2][b] = -irho * a.zs_b * lam[2 * N + b];
            z[3][b] = z[4][b] = R(0);
        } else {
            z[0][b] = irho * a.zs_b * lam[b];
            z[1][b] = irho * a.zs_b * lam[N + b];
            z[2][b] = -a.zs_b * (stiff * lam[2 * N + b] + lamL * lam[3 * N + b]);
            z[3][b] = -a.zs_b * (lamL * lam[2 * N + b] + stiff * lam[3 * N + b]);
            z[4][b] = -a.zs_b * tmu * lam[4 * N + b];
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int b = 0; b < N; ++b)
            if (q < nb) bst(B.r, boff, B.yout + (q * N + b) * B.rowb, z[q][b]);
    if (G.medium == kFluid)
        fluid_traces<K, NF, R, 0, POOLED>(a, B, T, lk, L.boff, z[0], z[1], z[2], tau);
    else
        solid_traces<K, NF, R, 0, POOLED>(a, B, T, lk, L.boff, z[0], z[1], z[2], z[3], z[4], tau, itau);
}

template <int K, typename R, bool POOLED>
__global__ __launch_bounds__(kBlock) void adjoint_start_kernel(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if (!L.active || ((POOLED || a.has_pooled) && (G.pooled != 0) != POOLED)) return;
    if (G.nF <= 4) start_body<K, 4, R, POOLED>(a, G, L);
    else start_body<K, kMaxFaces, R, POOLED>(a, G, L);
}

// grad[c][q] = sum over shots of the lane accumulators of cell c (input cell order).
__global__ __launch_bounds__(256) void grad_reduce_kernel(const double *gacc, long long LT, int S,
                                                         const int32_t *ic_of_cell, int n_cells, double *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const long long base = (long long)ic_of_cell[c] * S;
    for (int q = 0; q < 3; ++q) {
        double v = 0;
        for (int sh = 0; sh < S; ++sh) v += gacc[q * LT + base + sh];
        out[3 * c + q] = v;
    }
}

}  // namespace

hipError_t launch_grad_reduce(const double *gacc, long long LT, int S, const int32_t *ic_of_cell, int n_cells,
                              double *out, hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((n_cells + 255) / 256), dim3(256), 0, st, gacc, LT, S, ic_of_cell,
                       n_cells, out);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_adjoint_stage(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    if (!a.all_pooled) hipLaunchKernelGGL((adjoint_kernel<K, R, false>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    if (a.has_pooled) hipLaunchKernelGGL((adjoint_kernel<K, R, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_adjoint_start(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    if (!a.all_pooled)
        hipLaunchKernelGGL((adjoint_start_kernel<K, R, false>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    if (a.has_pooled)
        hipLaunchKernelGGL((adjoint_start_kernel<K, R, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

#define HHO_ADJ_INST(K, R)                                                                      \
    template hipError_t launch_adjoint_stage<K, R>(const StageArgs<R> &, int, hipStream_t);    \
    template hipError_t launch_adjoint_start<K, R>(const StageArgs<R> &, int, hipStream_t);
HHO_ADJ_INST(1, double)
HHO_ADJ_INST(2, double)
HHO_ADJ_INST(3, double)
HHO_ADJ_INST(1, float)
HHO_ADJ_INST(2, float)
HHO_ADJ_INST(3, float)

}  // namespace hho
