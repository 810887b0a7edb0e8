// HIP kernels (gfx950) of one explicit Runge-Kutta stage of the HHO elasto-acoustic
// semi-discretisation with the face unknowns eliminated (Sec. 4.2, eq. ex_solve).
//
// One lane = one (cell, shot).  Cells are grouped by (medium, shape class): a workgroup
// holds cells of one group, so its class table has uniform addresses and is read with
// scalar loads through the constant address space, and the (medium, face count) code
// path is uniform.  The state is structure-of-arrays, [row][lane], so every row load and
// store of a wavefront is coalesced.
//
// Fused stage, for every cell T of the group (bases orthonormal, so the cell and face
// mass matrices are identities):
//   1. face solves (eq. ex_solve, first line) for every non-boundary face F of T:
//        r_T = tau_T G^T u_T - G^T (flux_T . n)       (own trace contribution)
//        r_T' read from the neighbour's trace buffer  (written by the previous stage,
//                                                      in the neighbour's face basis:
//                                                      mode i changes sign as (-1)^i)
//        same medium:  u_F = (r_T + r_T') / (tau_T + tau_T')
//        interface:    tau_f p_F + n_G.v_F = r_f,  -n_G p_F + tau_s v_F = r_s   (3f x 3f)
//   2. cell residual (eq. ex_solve, second line) R = F_T - K_T u_T - K_TF u_F,
//   3. k = M^{-1} R (1/rho, kappa, or the stiffness C in the E basis),
//   4. Runge-Kutta combine (eq. ERK), and the trace contributions of the new stage state
//      for the neighbours (written once, read once by the cell across each face).
#include <hip/hip_runtime.h>

#include "device.h"
#include "plan.h"

#define HHO_CONST __attribute__((address_space(4)))

namespace hho {

namespace {

template <int K>
struct Dim {
    static constexpr int N = (K + 1) * (K + 2) / 2;
    static constexpr int F = K + 1;
};

// Read-only data with wavefront-uniform addresses: the constant address space lets the
// compiler use scalar loads.
template <typename T>
__device__ __forceinline__ const HHO_CONST T *uni(const T *p) {
    return (const HHO_CONST T *)p;
}

template <typename R>
__device__ __forceinline__ R sgn(int i) {
    return (i & 1) ? R(-1) : R(1);
}

__device__ __forceinline__ double ricker(double t, double f0, double t0) {
    const double a = 3.14159265358979323846 * f0 * (t - t0);
    return (1.0 - 2.0 * a * a) * exp(-a * a);
}

struct LaneInfo {
    int ic, shot;
    long long lane;
    bool active;
};

template <typename R>
__device__ __forceinline__ LaneInfo decode_lane(const StageArgs<R> &a, GroupDev &G) {
    const int g = uni(a.blk_group)[blockIdx.x];
    const HHO_CONST GroupDev *gd = uni(a.groups) + g;
    G.medium = gd->medium;
    G.nF = gd->nF;
    G.tab_off = gd->tab_off;
    G.ic_begin = gd->ic_begin;
    G.ncells = gd->ncells;
    G.blk_begin = gd->blk_begin;
    LaneInfo L;
    const int tid = threadIdx.x;
    const int cl = tid / a.S;
    L.shot = tid - cl * a.S;
    const int l = (blockIdx.x - G.blk_begin) * a.cpb + cl;
    L.active = l < G.ncells;
    L.ic = G.ic_begin + l;
    L.lane = (long long)L.ic * a.S + L.shot;
    return L;
}

constexpr double kRsqrt2 = 0.70710678118654752440;

// ------------------------------------------------------------------------- traces
// Own trace contributions of a fluid state on every non-boundary face.
template <int K, int NF, typename R>
__device__ __forceinline__ void fluid_traces(const StageArgs<R> &a, const HHO_CONST R *tb, int nF,
                                             const int *lk, long long lane, const R *p, const R *mx, const R *my, R tau) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const HHO_CONST R *Gt = tb + 3 * N * N;
    const HHO_CONST R *nr = Gt + nF * N * F;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
        const R nx = nr[2 * j], ny = nr[2 * j + 1];
        R r[F];
#pragma unroll
        for (int i = 0; i < F; ++i) r[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R q = tau * p[b] - (nx * mx[b] + ny * my[b]);
#pragma unroll
            for (int i = 0; i < F; ++i) r[i] += Gt[(j * N + b) * F + i] * q;
        }
#pragma unroll
        for (int i = 0; i < F; ++i) a.Tout[((long long)(j * 2) * F + i) * a.LT + lane] = r[i];
    }
}

template <int K, int NF, typename R>
__device__ __forceinline__ void solid_traces(const StageArgs<R> &a, const HHO_CONST R *tb, int nF,
                                             const int *lk, long long lane, const R *vx, const R *vy, const R *s1, const R *s2,
                                             const R *s3, R tau) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const R r2 = R(kRsqrt2);
    const HHO_CONST R *Gt = tb + 3 * N * N;
    const HHO_CONST R *nr = Gt + nF * N * F;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
        const R nx = nr[2 * j], ny = nr[2 * j + 1];
        R rx[F], ry[F];
#pragma unroll
        for (int i = 0; i < F; ++i) rx[i] = ry[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R qx = tau * vx[b] - (nx * s1[b] + r2 * ny * s3[b]);
            const R qy = tau * vy[b] - (r2 * nx * s3[b] + ny * s2[b]);
#pragma unroll
            for (int i = 0; i < F; ++i) {
                rx[i] += Gt[(j * N + b) * F + i] * qx;
                ry[i] += Gt[(j * N + b) * F + i] * qy;
            }
        }
#pragma unroll
        for (int i = 0; i < F; ++i) {
            a.Tout[((long long)(j * 2) * F + i) * a.LT + lane] = rx[i];
            a.Tout[((long long)(j * 2 + 1) * F + i) * a.LT + lane] = ry[i];
        }
    }
}

// Links of every local face and the neighbour trace contributions (both components;
// the second only where it is needed), issued before any arithmetic.
// The link and coefficient arrays hold one row per face of the largest cell of the mesh:
// rows j >= nF of this group are never read (their links count as -1).
template <int K, int NF, typename R>
__device__ __forceinline__ void load_faces(const StageArgs<R> &a, int medium, int nF, int ic, int shot, int *lk,
                                           R *cc, R (*rn)[2][Dim<K>::F], R *its) {
    constexpr int F = Dim<K>::F;
    const int nic = a.n_ic;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        lk[j] = -1;
        cc[j] = R(0);
        if (j < nF) {
            lk[j] = a.link[(long long)j * nic + ic];
            cc[j] = a.c0[(long long)j * nic + ic];
        }
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        its[j] = R(0);
#pragma unroll
        for (int i = 0; i < F; ++i) rn[j][0][i] = rn[j][1][i] = R(0);
        if (lk[j] < 0) continue;
        const int icn = lk[j] >> 4, jn = lk[j] & 7;
        const bool iface = (lk[j] >> 3) & 1;
        const long long nl = (long long)icn * a.S + shot;
        const R *t0 = a.Tin + (long long)(jn * 2) * F * a.LT + nl;
#pragma unroll
        for (int i = 0; i < F; ++i) rn[j][0][i] = sgn<R>(i) * t0[(long long)i * a.LT];
        // second component: solid neighbours (same-medium solid face, or interface seen from the fluid)
        if (medium == kSolid ? !iface : iface) {
            const R *t1 = t0 + (long long)F * a.LT;
#pragma unroll
            for (int i = 0; i < F; ++i) rn[j][1][i] = sgn<R>(i) * t1[(long long)i * a.LT];
        }
        if (iface && medium == kFluid) its[j] = a.mat[(long long)kInvTau * nic + icn];
    }
}

// ------------------------------------------------------------------------- fluid cells
template <int K, int NF, typename R>
__device__ __forceinline__ void fluid_stage(const StageArgs<R> &a, const HHO_CONST R *tb, int nF, int ic, int shot,
                                            long long lane, double *energy) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const long long LT = a.LT;
    const int nic = a.n_ic;
    const HHO_CONST R *Bx = tb;
    const HHO_CONST R *By = tb + N * N;
    const HHO_CONST R *Sm = tb + 2 * N * N;
    const HHO_CONST R *Gt = tb + 3 * N * N;
    const HHO_CONST R *nr = Gt + nF * N * F;
    int lk[NF];
    R cc[NF], its[NF], rn[NF][2][F];
    load_faces<K, NF, R>(a, kFluid, nF, ic, shot, lk, cc, rn, its);
    R p[N], mx[N], my[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        p[b] = a.Yin[(long long)b * LT + lane];
        mx[b] = a.Yin[(long long)(N + b) * LT + lane];
        my[b] = a.Yin[(long long)(2 * N + b) * LT + lane];
    }
    const R tau = a.mat[(long long)kTau * nic + ic];
    const R kap = a.mat[(long long)kStiff * nic + ic];
    const R irho = a.mat[(long long)kInvRho * nic + ic];
    R rp[N], rmx[N], rmy[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R sx = 0, sy = 0, sd = 0, ss = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            sx += Bx[r * N + b] * p[b];
            sy += By[r * N + b] * p[b];
            sd += Bx[b * N + r] * mx[b] + By[b * N + r] * my[b];
            ss += Sm[r * N + b] * p[b];
        }
        rmx[r] = sx;
        rmy[r] = sy;
        rp[r] = -(sd + tau * ss);
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: p_F = 0 (homogeneous Dirichlet)
        const R nx = nr[2 * j], ny = nr[2 * j + 1];
        R r[F];
#pragma unroll
        for (int i = 0; i < F; ++i) r[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R q = tau * p[b] - (nx * mx[b] + ny * my[b]);
#pragma unroll
            for (int i = 0; i < F; ++i) r[i] += Gt[(j * N + b) * F + i] * q;
        }
        R pF[F];
        if (!((lk[j] >> 3) & 1)) {
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + rn[j][0][i]) * cc[j];
        } else {
            // interface, neighbour solid: n_G = -n_T, eliminate v_F
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + (nx * rn[j][0][i] + ny * rn[j][1][i]) * its[j]) * cc[j];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R w = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) w += Gt[(j * N + b) * F + i] * pF[i];
            rmx[b] += nx * w;
            rmy[b] += ny * w;
            rp[b] += tau * w;
        }
    }
    // loads F_T(t)
    for (int m = 0; m < a.nterms; ++m) {
        const R w = a.wterm[m];
        const R *g = a.gload + (long long)m * 5 * N * nic + ic;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            rp[b] += w * g[(long long)b * nic];
            rmx[b] += w * g[(long long)(N + b) * nic];
            rmy[b] += w * g[(long long)(2 * N + b) * nic];
        }
    }
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &s = a.src[e];
            if (s.shot == shot) {
                const R w = R(s.amp * ricker(a.t, s.f0, s.t0) * s.dirx);
#pragma unroll
                for (int b = 0; b < N; ++b) rp[b] += w * R(s.phi[b]);
            }
            e = s.next;
        }
    }
    // k = M^{-1} R and the Runge-Kutta combine
    R np[N], nmx[N], nmy[N];
#pragma unroll
    for (int row = 0; row < 3 * N; ++row) {
        const int b = row % N, blk = row / N;
        const R kv = blk == 0 ? kap * rp[b] : irho * (blk == 1 ? rmx[b] : rmy[b]);
        const R y = blk == 0 ? p[b] : (blk == 1 ? mx[b] : my[b]);
        const long long ix = (long long)row * LT + lane;
        R out;
        if (!a.last) {
            const R u = a.first ? y : a.U[ix];
            out = a.cU * u + a.cY * y + a.ck * a.dt * kv;
            a.Yout[ix] = out;
            a.acc[ix] = (a.first ? R(0) : a.acc[ix]) + a.cb * kv;
        } else {
            const R u = a.first ? y : a.U[ix];
            out = u + a.dt * ((a.first ? R(0) : a.acc[ix]) + a.cb * kv);
            a.U[ix] = out;
        }
        if (blk == 0) np[b] = out;
        else if (blk == 1) nmx[b] = out;
        else nmy[b] = out;
    }
    fluid_traces<K, NF, R>(a, tb, nF, lk, lane, np, nmx, nmy, tau);
    if (a.last) {
        if (energy) {
            double sp = 0, sm = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                sp += (double)np[b] * (double)np[b];
                sm += (double)nmx[b] * (double)nmx[b] + (double)nmy[b] * (double)nmy[b];
            }
            *energy = 0.5 * (a.emat[(long long)1 * nic + ic] * sp + a.emat[ic] * sm);
        }
        if (a.rec_first) {
            for (int e = a.rec_first[ic]; e >= 0;) {
                const RecDev &rc = a.rec[e];
                double v = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) v += rc.phi[b] * (double)np[b];
                double *o = a.rec_out + (((long long)shot * a.rec_steps + a.step) * a.nrec + rc.r) * 2;
                o[0] = v;
                o[1] = 0.0;
                e = rc.next;
            }
        }
    }
}

// ------------------------------------------------------------------------- solid cells
template <int K, int NF, typename R>
__device__ __forceinline__ void solid_stage(const StageArgs<R> &a, const HHO_CONST R *tb, int nF, int ic, int shot,
                                            long long lane, double *energy) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const long long LT = a.LT;
    const int nic = a.n_ic;
    const R r2 = R(kRsqrt2);
    const HHO_CONST R *Bx = tb;
    const HHO_CONST R *By = tb + N * N;
    const HHO_CONST R *Sm = tb + 2 * N * N;
    const HHO_CONST R *Gt = tb + 3 * N * N;
    const HHO_CONST R *nr = Gt + nF * N * F;
    int lk[NF];
    R cc[NF], its[NF], rn[NF][2][F];
    load_faces<K, NF, R>(a, kSolid, nF, ic, shot, lk, cc, rn, its);
    R vx[N], vy[N], s1[N], s2[N], s3[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        vx[b] = a.Yin[(long long)b * LT + lane];
        vy[b] = a.Yin[(long long)(N + b) * LT + lane];
        s1[b] = a.Yin[(long long)(2 * N + b) * LT + lane];
        s2[b] = a.Yin[(long long)(3 * N + b) * LT + lane];
        s3[b] = a.Yin[(long long)(4 * N + b) * LT + lane];
    }
    const R tau = a.mat[(long long)kTau * nic + ic];
    const R itau = a.mat[(long long)kInvTau * nic + ic];
    const R irho = a.mat[(long long)kInvRho * nic + ic];
    const R l2m = a.mat[(long long)kStiff * nic + ic];
    const R lam = a.mat[(long long)kLam * nic + ic];
    const R tmu = a.mat[(long long)kTwoMu * nic + ic];
    R rvx[N], rvy[N], rs1[N], rs2[N], rs3[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R a1 = 0, a2 = 0, a3 = 0, bx = 0, by = 0, sx = 0, sy = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R bxrb = Bx[r * N + b], byrb = By[r * N + b];
            const R bxbr = Bx[b * N + r], bybr = By[b * N + r], srb = Sm[r * N + b];
            a1 += bxrb * vx[b];
            a2 += byrb * vy[b];
            a3 += byrb * vx[b] + bxrb * vy[b];
            bx += bxbr * s1[b] + bybr * (r2 * s3[b]);
            by += bybr * s2[b] + bxbr * (r2 * s3[b]);
            sx += srb * vx[b];
            sy += srb * vy[b];
        }
        rs1[r] = a1;
        rs2[r] = a2;
        rs3[r] = r2 * a3;
        rvx[r] = -(bx + tau * sx);
        rvy[r] = -(by + tau * sy);
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: v_F = 0 (homogeneous Dirichlet)
        const R nx = nr[2 * j], ny = nr[2 * j + 1];
        R rx[F], ry[F];
#pragma unroll
        for (int i = 0; i < F; ++i) rx[i] = ry[i] = R(0);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const R qx = tau * vx[b] - (nx * s1[b] + r2 * ny * s3[b]);
            const R qy = tau * vy[b] - (r2 * nx * s3[b] + ny * s2[b]);
#pragma unroll
            for (int i = 0; i < F; ++i) {
                rx[i] += Gt[(j * N + b) * F + i] * qx;
                ry[i] += Gt[(j * N + b) * F + i] * qy;
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
            // interface, neighbour fluid: n_G = n_T, eliminate p_F then v_F
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const R pF = (rn[j][0][i] - (nx * rx[i] + ny * ry[i]) * itau) * cc[j];
                vFx[i] = (rx[i] + nx * pF) * itau;
                vFy[i] = (ry[i] + ny * pF) * itau;
            }
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R wx = 0, wy = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                wx += Gt[(j * N + b) * F + i] * vFx[i];
                wy += Gt[(j * N + b) * F + i] * vFy[i];
            }
            rs1[b] += nx * wx;
            rs2[b] += ny * wy;
            rs3[b] += r2 * (ny * wx + nx * wy);
            rvx[b] += tau * wx;
            rvy[b] += tau * wy;
        }
    }
    for (int m = 0; m < a.nterms; ++m) {
        const R w = a.wterm[m];
        const R *g = a.gload + (long long)m * 5 * N * nic + ic;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            rvx[b] += w * g[(long long)b * nic];
            rvy[b] += w * g[(long long)(N + b) * nic];
            rs1[b] += w * g[(long long)(2 * N + b) * nic];
            rs2[b] += w * g[(long long)(3 * N + b) * nic];
            rs3[b] += w * g[(long long)(4 * N + b) * nic];
        }
    }
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &s = a.src[e];
            if (s.shot == shot) {
                const double w = s.amp * ricker(a.t, s.f0, s.t0);
                const R wx = R(w * s.dirx), wy = R(w * s.diry);
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    rvx[b] += wx * R(s.phi[b]);
                    rvy[b] += wy * R(s.phi[b]);
                }
            }
            e = s.next;
        }
    }
    R nvx[N], nvy[N], ns1[N], ns2[N], ns3[N];
#pragma unroll
    for (int row = 0; row < 5 * N; ++row) {
        const int b = row % N, blk = row / N;
        R kv, y;
        switch (blk) {
            case 0: kv = irho * rvx[b]; y = vx[b]; break;
            case 1: kv = irho * rvy[b]; y = vy[b]; break;
            case 2: kv = l2m * rs1[b] + lam * rs2[b]; y = s1[b]; break;
            case 3: kv = lam * rs1[b] + l2m * rs2[b]; y = s2[b]; break;
            default: kv = tmu * rs3[b]; y = s3[b]; break;
        }
        const long long ix = (long long)row * LT + lane;
        R out;
        if (!a.last) {
            const R u = a.first ? y : a.U[ix];
            out = a.cU * u + a.cY * y + a.ck * a.dt * kv;
            a.Yout[ix] = out;
            a.acc[ix] = (a.first ? R(0) : a.acc[ix]) + a.cb * kv;
        } else {
            const R u = a.first ? y : a.U[ix];
            out = u + a.dt * ((a.first ? R(0) : a.acc[ix]) + a.cb * kv);
            a.U[ix] = out;
        }
        switch (blk) {
            case 0: nvx[b] = out; break;
            case 1: nvy[b] = out; break;
            case 2: ns1[b] = out; break;
            case 3: ns2[b] = out; break;
            default: ns3[b] = out; break;
        }
    }
    solid_traces<K, NF, R>(a, tb, nF, lk, lane, nvx, nvy, ns1, ns2, ns3, tau);
    if (a.last) {
        if (energy) {
            const double ca = a.emat[(long long)1 * nic + ic], cb = a.emat[(long long)2 * nic + ic];
            const double c3 = a.emat[(long long)3 * nic + ic];
            double sv = 0, ss = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const double x1 = ns1[b], x2 = ns2[b], x3 = ns3[b];
                sv += (double)nvx[b] * (double)nvx[b] + (double)nvy[b] * (double)nvy[b];
                ss += ca * (x1 * x1 + x2 * x2) + 2.0 * cb * x1 * x2 + c3 * x3 * x3;
            }
            *energy = 0.5 * (a.emat[ic] * sv + ss);
        }
        if (a.rec_first) {
            for (int e = a.rec_first[ic]; e >= 0;) {
                const RecDev &rc = a.rec[e];
                double v0 = 0, v1 = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    v0 += rc.phi[b] * (double)nvx[b];
                    v1 += rc.phi[b] * (double)nvy[b];
                }
                double *o = a.rec_out + (((long long)shot * a.rec_steps + a.step) * a.nrec + rc.r) * 2;
                o[0] = v0;
                o[1] = v1;
                e = rc.next;
            }
        }
    }
}

// Block reduction of per-lane energies into one partial per shot.
__device__ void block_energy(double e, int S, int cpb, double *out) {
    __shared__ double buf[kBlock];
    buf[threadIdx.x] = e;
    __syncthreads();
    if ((int)threadIdx.x < S) {
        double s = 0;
        for (int m = 0; m < cpb; ++m) s += buf[threadIdx.x + m * S];
        out[(long long)blockIdx.x * S + threadIdx.x] = s;
    }
}

template <int K, int NF, typename R>
__device__ __forceinline__ void stage_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L, double *e) {
    const HHO_CONST R *tb = uni(a.tab) + G.tab_off;
    if (G.medium == kFluid)
        fluid_stage<K, NF, R>(a, tb, G.nF, L.ic, L.shot, L.lane, e);
    else
        solid_stage<K, NF, R>(a, tb, G.nF, L.ic, L.shot, L.lane, e);
}

template <int K, typename R>
__global__ __launch_bounds__(kBlock) void stage_kernel(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    const bool want_e = a.last && a.e_part;
    double e = 0.0;
    double *ep = want_e ? &e : nullptr;
    if (L.active) {
        // faces beyond a cell's count carry link -1 and are skipped like boundary faces
        if (G.nF <= 4) stage_body<K, 4, R>(a, G, L, ep);
        else stage_body<K, kMaxFaces, R>(a, G, L, ep);
    }
    if (want_e) block_energy(e, a.S, a.cpb, a.e_part);
}

// Trace contributions of the state in a.Yin (used once after the state is set).
template <int K, int NF, typename R>
__device__ __forceinline__ void traces_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L) {
    constexpr int N = Dim<K>::N;
    const HHO_CONST R *tb = uni(a.tab) + G.tab_off;
    int lk[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) lk[j] = j < G.nF ? a.link[(long long)j * a.n_ic + L.ic] : -1;
    const R tau = a.mat[(long long)kTau * a.n_ic + L.ic];
    R v[5][N];
    const int nb = G.medium == kFluid ? 3 : 5;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int b = 0; b < N; ++b) v[q][b] = q < nb ? a.Yin[(long long)(q * N + b) * a.LT + L.lane] : R(0);
    if (G.medium == kFluid)
        fluid_traces<K, NF, R>(a, tb, G.nF, lk, L.lane, v[0], v[1], v[2], tau);
    else
        solid_traces<K, NF, R>(a, tb, G.nF, lk, L.lane, v[0], v[1], v[2], v[3], v[4], tau);
}

template <int K, typename R>
__global__ __launch_bounds__(kBlock) void trace_kernel(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if (!L.active) return;
    if (G.nF <= 4) traces_body<K, 4, R>(a, G, L);
    else traces_body<K, kMaxFaces, R>(a, G, L);
}

// Energy of the state in a.Yin (Sec. 5.1), float64 partials per block and shot.
template <int K, typename R>
__global__ __launch_bounds__(kBlock) void energy_kernel(StageArgs<R> a) {
    constexpr int N = Dim<K>::N;
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    double e = 0.0;
    if (L.active) {
        const int nic = a.n_ic, ic = L.ic;
        auto ld = [&](int row) { return (double)a.Yin[(long long)row * a.LT + L.lane]; };
        if (G.medium == kFluid) {
            double sp = 0, sm = 0;
            for (int b = 0; b < N; ++b) {
                sp += ld(b) * ld(b);
                sm += ld(N + b) * ld(N + b) + ld(2 * N + b) * ld(2 * N + b);
            }
            e = 0.5 * (a.emat[(long long)nic + ic] * sp + a.emat[ic] * sm);
        } else {
            const double ca = a.emat[(long long)nic + ic], cb = a.emat[(long long)2 * nic + ic];
            const double c3 = a.emat[(long long)3 * nic + ic];
            double sv = 0, ss = 0;
            for (int b = 0; b < N; ++b) {
                const double x1 = ld(2 * N + b), x2 = ld(3 * N + b), x3 = ld(4 * N + b);
                sv += ld(b) * ld(b) + ld(N + b) * ld(N + b);
                ss += ca * (x1 * x1 + x2 * x2) + 2.0 * cb * x1 * x2 + c3 * x3 * x3;
            }
            e = 0.5 * (a.emat[ic] * sv + ss);
        }
    }
    block_energy(e, a.S, a.cpb, a.e_part);
}

__global__ void energy_reduce_kernel(const double *part, int n_blocks, int S, double *out) {
    __shared__ double buf[kBlock];
    const int s = blockIdx.x;
    double acc = 0;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) acc += part[(long long)b * S + s];
    buf[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = buf[0];
}

template <typename R>
__global__ void scatter_kernel(const double *ext, const int64_t *map, long long n, int shot, R *state) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) state[map[e] + shot] = R(ext[e]);
}

template <typename R>
__global__ void gather_kernel(const R *state, const int64_t *map, long long n, int shot, double *ext) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) ext[e] = (double)state[map[e] + shot];
}

}  // namespace

template <int K, typename R>
hipError_t launch_stage(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL((stage_kernel<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_traces(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL((trace_kernel<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_energy(const StageArgs<R> &a, const R *state, int n_blocks, hipStream_t st) {
    StageArgs<R> b = a;
    b.Yin = state;
    hipLaunchKernelGGL((energy_kernel<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const double *part, int n_blocks, int S, double *out, hipStream_t st) {
    hipLaunchKernelGGL(energy_reduce_kernel, dim3(S), dim3(kBlock), 0, st, part, n_blocks, S, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter(const double *ext, const int64_t *map, long long n, int shot, R *state, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((scatter_kernel<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ext, map, n, shot,
                       state);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gather(const R *state, const int64_t *map, long long n, int shot, double *ext, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((gather_kernel<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, state, map, n, shot,
                       ext);
    return hipGetLastError();
}

#define HHO_INST(K, R)                                                                              \
    template hipError_t launch_stage<K, R>(const StageArgs<R> &, int, hipStream_t);                \
    template hipError_t launch_traces<K, R>(const StageArgs<R> &, int, hipStream_t);               \
    template hipError_t launch_energy<K, R>(const StageArgs<R> &, const R *, int, hipStream_t);
HHO_INST(1, double)
HHO_INST(2, double)
HHO_INST(3, double)
HHO_INST(1, float)
HHO_INST(2, float)
HHO_INST(3, float)
template hipError_t launch_scatter<double>(const double *, const int64_t *, long long, int, double *, hipStream_t);
template hipError_t launch_scatter<float>(const double *, const int64_t *, long long, int, float *, hipStream_t);
template hipError_t launch_gather<double>(const double *, const int64_t *, long long, int, double *, hipStream_t);
template hipError_t launch_gather<float>(const float *, const int64_t *, long long, int, double *, hipStream_t);

}  // namespace hho
