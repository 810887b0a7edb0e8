// HIP kernels (gfx950) of one explicit Runge-Kutta stage of the HHO elasto-acoustic
// semi-discretisation with the face unknowns eliminated (Sec. 4.2, eq. ex_solve).
//
// One lane = one (cell, shot).  Cells are grouped by (medium, shape class): a workgroup
// holds cells of one group, so its class table has uniform addresses and is read with
// scalar loads through the constant address space, and the code path is uniform.  All
// per-lane arrays are structure-of-arrays, [row][lane], read and written through buffer
// resources: the uniform row offset sits in a scalar register and each lane adds a 32-bit
// byte offset, so accesses are coalesced, need no 64-bit address arithmetic, and are
// range-checked by the hardware.
//
// Fused stage, for every cell T of the group (bases orthonormal, so the cell and face
// mass matrices are identities):
//   1. face solves (eq. ex_solve, first line) for every non-boundary face F of T:
//        r_T = tau_T G^T u_T - G^T (flux_T . n)       (own trace contribution)
//        r_T'                                          (the neighbour's, gathered from the
//                                                      neighbour's own trace slots)
//        same medium:  u_F = (r_T + r_T') / (tau_T + tau_T')
//        interface:    tau_f p_F + n_G.v_F = r_f,  -n_G p_F + tau_s v_F = r_s   (3f x 3f)
//   2. cell residual (eq. ex_solve, second line) R = F_T - K_T u_T - K_TF u_F,
//   3. k = M^{-1} R (1/rho, kappa, or the stiffness C in the E basis),
//   4. Runge-Kutta combine (eq. ERK); then T computes the trace contributions of its new
//      stage state on each of its faces and stores them in its own slots, already in the
//      neighbour's face basis (mode i flips sign as (-1)^i between the two orientations of a
//      face; a solid cell's contribution across the interface is also divided by its tau_s,
//      which the fluid side needs).  Trace buffers are [slot][lane][mode] (slot = local face
//      and component), so these stores are coalesced and each lane writes whole F-mode
//      pieces; the next stage gathers, through the face links, the pieces of its neighbours
//      (one wide load of F modes per face and component).
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace hho {
namespace {

// Register budget of the stage kernel: the least number of waves per SIMD the compiler must leave
// room for, per degree k = 1, 2, 3 (4 waves leave 128 VGPRs per lane, 3 leave 168, 2 leave 256;
// 1 sets no budget), for float32 and float64 stepping.  It applies to the plain stage launches
// (shared tables, no recompute stores); a float64 launch with a budget of two waves also
// combines its rows in chunks (rk_update), which is what brings it within 256 registers.
#ifndef HHO_STAGE_WAVES_F32
#define HHO_STAGE_WAVES_F32 1, 1, 1
#endif
#ifndef HHO_STAGE_WAVES_F64
#define HHO_STAGE_WAVES_F64 1, 2, 1
#endif
// Highest degree whose float32 stage keeps U^n and D_{i-1} in registers for the combine (float64:
// k = 1 only); the others read them again (cache hits), which costs fewer registers.
#ifndef HHO_KEEP_MAX_K_F32
#define HHO_KEEP_MAX_K_F32 2
#endif
template <int K, typename R, bool STORE = false, bool POOLED = false>
constexpr int stage_waves() {
    constexpr int w32[3] = {HHO_STAGE_WAVES_F32}, w64[3] = {HHO_STAGE_WAVES_F64};
    if (STORE || POOLED) return 1;
    return sizeof(R) == 4 ? w32[K - 1] : w64[K - 1];
}
// float64 plain launches under a two-wave budget combine their rows in chunks
template <int K, typename R, bool STORE, bool POOLED>
constexpr bool chunked_combine() {
    return sizeof(R) == 8 && stage_waves<K, R, STORE, POOLED>() >= 2;
}
template <int K, typename R>
constexpr bool keep_in_registers() {
    return sizeof(R) == 4 ? K <= HHO_KEEP_MAX_K_F32 : K <= 1;
}
// float32 k = 3 plain launches park D_{i-1} in LDS between the stage's first read and the combine
// (their registers do not hold it, and read again from memory it misses the L2); one row of
// blockDim floats per unknown row, each lane reading back only what it wrote
template <int K, typename R, bool STORE, bool POOLED>
constexpr bool lds_increment() {
    return sizeof(R) == 4 && K == 3 && !STORE && !POOLED && !keep_in_registers<K, R>();
}
template <int K, typename R>
constexpr size_t lds_increment_bytes(int lanes) {
    return lds_increment<K, R, false, false>() ? (size_t)lanes * 5 * Dim<K>::N * sizeof(R) : 0;
}
extern __shared__ unsigned char hho_stage_lds[];

// Stage state of one lane.  The stage buffers hold increments D_i = Y_{i+1} - U^n rather than
// the stage states: the stage input is Y_i = U^n + D_{i-1} (U^n itself on the first stage).
// Kept as increments, the values that the final combination below sums keep their full
// relative precision in float32 (a stored Y_i would round away the low bits of dt k_i).
// With KEEP, U^n and D_{i-1} stay in registers (uk, dk) for the combine; otherwise the combine
// reads them again (cache hits), which keeps the register count of the larger degrees down.
template <int ND, typename R, bool KEEP, bool LDSD = false>
__device__ __forceinline__ void load_state(const StageArgs<R> &a, const Bufs<R> &B, unsigned boff, R *y, R *uk,
                                           R *dk) {
    if (a.first) {
#pragma unroll
        for (int r = 0; r < ND; ++r) y[r] = bld<R>(B.r, boff, B.yin + r * B.rowb);
        if (KEEP) {
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                uk[r] = y[r];
                dk[r] = R(0);
            }
        }
    } else {
        R d[ND], u[ND];
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            d[r] = bld<R>(B.r, boff, B.yin + r * B.rowb);
            u[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
        }
#pragma unroll
        for (int r = 0; r < ND; ++r) y[r] = u[r] + d[r];
        if (LDSD) {
            R *dl = reinterpret_cast<R *>(hho_stage_lds);
#pragma unroll
            for (int r = 0; r < ND; ++r) dl[r * blockDim.x + threadIdx.x] = d[r];
        }
        if (KEEP) {
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                uk[r] = u[r];
                dk[r] = d[r];
            }
        }
    }
}

// Runge-Kutta combine of all ND rows of a lane (eq. ERK).  Before the last stage:
// D_i = cY D_{i-1} + ck dt k_i (so that Y_{i+1} = cU U + cY Y_i + ck dt k_i with cU + cY = 1).
// For i < s, dt k_i = (D_i - cY_i D_{i-1}) / ck_i, so U^{n+1} = U^n + dt sum_i b_i k_i is U^n plus
// a fixed combination of the increments and b_s dt k_s.  One middle stage folds the earlier
// increments into a partial sum Q (stored in place of its input), and the last stage forms
// U^{n+1} = U^n + Q + cd D_{s-2} + b_s dt k_s.  No accumulator of b_i k_i is kept: a step of
// ERK(4) moves 13 words per unknown instead of 17.  U^n and D_{i-1} were read at the start of
// this stage and are read again here (cache hits) rather than held in registers through the
// residual.  out = the new stage state (Y_{i+1} or U^{n+1}), from which the outgoing traces are
// formed.  Every load is issued before the first store: the arrays share one buffer resource,
// so the compiler cannot move a load above an earlier store.
template <int ND, typename R, bool KEEP, int POL, bool CHUNK = false, bool LDSD = false>
__device__ __forceinline__ void rk_update(const StageArgs<R> &a, const Bufs<R> &B, unsigned boff, const R *y,
                                          const R *kv, R *out, const R *uk, const R *dk, int shot) {
    if constexpr (CHUNK) {
        // U^n read again on every stage (the stage input y is not kept for the first one) and the
        // rows combined a fifth (or a third) at a time, so that only that share of U^n, D_{i-1}
        // and Q is in registers beside k_i
        const R dt = R(shot_dt(a, shot));
        const bool need_d = !a.first && (a.last ? a.cd != R(0) : (a.cY != R(0) || a.q_write));
        constexpr int CH = ND % 5 == 0 ? ND / 5 : ND / 3;
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
        return;
    }
    const R dt = R(shot_dt(a, shot));
    R u[ND], din[ND];
    const bool need_d = a.last ? a.cd != R(0) : (a.cY != R(0) || a.q_write);
    if (KEEP) {
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            u[r] = uk[r];
            din[r] = dk[r];
        }
    } else if (a.first) {
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            u[r] = y[r];
            din[r] = R(0);
        }
    } else if (need_d) {
        const R *dl = reinterpret_cast<const R *>(hho_stage_lds);
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            u[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
            din[r] = LDSD ? dl[r * blockDim.x + threadIdx.x] : bld<R>(B.r, boff, B.yin + r * B.rowb);
        }
    } else {
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            u[r] = bld<R>(B.r, boff, B.u + r * B.rowb);
            din[r] = R(0);
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
        if (a.q_read) {
#pragma unroll
            for (int r = 0; r < ND; ++r) q[r] = bld<R>(B.r, boff, B.yq + r * B.rowb);
        } else {
#pragma unroll
            for (int r = 0; r < ND; ++r) q[r] = R(0);
        }
        const R cb = a.cb * dt;
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            out[r] = u[r] + (q[r] + a.cd * din[r] + cb * kv[r]);
            bst<POL>(B.r, boff, B.u + r * B.rowb, out[r]);
        }
    }
}

// Recompute stores of one lane for the adjoint: stage input, stage derivative, face values
// (after the combine, so these stores do not hold back the combine's loads).
// NC = primal components (1: p, 2: v); only the primal rows of Y and of the face values are kept.
template <int K, int NF, int ND, typename R, int NFV, int NC>
__device__ __forceinline__ void store_recompute(const StageArgs<R> &a, const int *lk, unsigned boff, const R *y,
                                                const R *kv, const R (*fv)[2][Dim<K>::F]) {
    constexpr int F = Dim<K>::F, N = Dim<K>::N;
    const long long lane = boff / sizeof(R);
#pragma unroll
    for (int r = 0; r < NC * N; ++r) a.ystore[(long long)r * a.LT + lane] = y[r];
#pragma unroll
    for (int r = 0; r < ND; ++r) a.kstore[(long long)r * a.LT + lane] = kv[r];
#pragma unroll
    for (int j = 0; j < NFV; ++j) {
        if (lk[j] < 0) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int i = 0; i < F; ++i) a.fstore[(long long)((j * 2 + c) * F + i) * a.LT + lane] = fv[j][c][i];
    }
}

// ------------------------------------------------------------------------- fluid cells
template <int K, int NF, typename R, bool STORE, int POL, bool PK>
__device__ __forceinline__ double fluid_stage(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T,
                                              int nF, const LaneInfo &L, bool want_e) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    int lk[NF];
    R cc[NF], rn[NF][2][F];
    R fv[STORE ? NF : 1][2][F];  // face values, kept for the recompute stores
    load_links<NF, R>(B, nF, ic, lk, cc);
    constexpr bool KEEP = keep_in_registers<K, R>();
    R y[3 * N], uk[KEEP ? 3 * N : 1], dk[KEEP ? 3 * N : 1];
    load_state<3 * N, R, KEEP, lds_increment<K, R, STORE, PK>()>(a, B, boff, y, uk, dk);
    const R *p = y, *mx = y + N, *my = y + 2 * N;
    load_incoming<K, NF, R>(B, kFluid, a.S, shot, lk, rn);
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R kap = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    R rp[N], rmx[N], rmy[N], tp[N];
#pragma unroll
    for (int b = 0; b < N; ++b) tp[b] = tau * p[b];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R sx = 0, sy = 0, sd = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            if (b_nonzero(r, b)) {
                sx += T.bx(r, b) * p[b];
                sy += T.by(r, b) * p[b];
            }
            if (b_nonzero(b, r)) sd += T.bx(b, r) * mx[b] + T.by(b, r) * my[b];
            sd += T.s(r, b) * tp[b];
        }
        rmx[r] = sx;
        rmy[r] = sy;
        rp[r] = -sd;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: p_F = 0 (homogeneous Dirichlet)
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
            // interface, neighbour solid (its contribution arrives divided by tau_s):
            // n_G = -n_T, eliminate v_F
#pragma unroll
            for (int i = 0; i < F; ++i) pF[i] = (r[i] + nx * rn[j][0][i] + ny * rn[j][1][i]) * cc[j];
        }
        if (STORE) {
#pragma unroll
            for (int i = 0; i < F; ++i) fv[j][0][i] = pF[i];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R w = 0;
#pragma unroll
            for (int i = 0; i < F; ++i)
                if (g_nonzero(b, i)) w += T.g(j, b, i) * pF[i];
            rmx[b] += nx * w;
            rmy[b] += ny * w;
            rp[b] += tau * w;
        }
    }
    // loads F_T(t)
    for (int m = 0; m < a.nterms; ++m) {
        const R w = R(sin(a.omega[m] * stage_time(a, shot) + a.phase[m]));
        const int gr = m * 5 * N;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            rp[b] += w * a.gload[(long long)(gr + b) * nic + ic];
            rmx[b] += w * a.gload[(long long)(gr + N + b) * nic + ic];
            rmy[b] += w * a.gload[(long long)(gr + 2 * N + b) * nic + ic];
        }
    }
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &s = a.src[e];
            if (s.shot == shot) {
                const R w = R(s.amp * ricker(stage_time(a, shot), s.f0, s.t0) * s.dirx);
#pragma unroll
                for (int b = 0; b < N; ++b) rp[b] += w * R(s.phi[b]);
            }
            e = s.next;
        }
    }
    // k = M^{-1} R and the Runge-Kutta combine
    R kv[3 * N], nw[3 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        kv[b] = kap * rp[b];
        kv[N + b] = irho * rmx[b];
        kv[2 * N + b] = irho * rmy[b];
    }
    rk_update<3 * N, R, KEEP, POL, chunked_combine<K, R, STORE, PK>(), lds_increment<K, R, STORE, PK>()>(
        a, B, boff, y, kv, nw, uk, dk, shot);
    const R *np = nw, *nmx = nw + N, *nmy = nw + 2 * N;
    if (STORE) store_recompute<K, NF, 3 * N, R, NF, 1>(a, lk, boff, y, kv, fv);
    fluid_traces<K, NF, R, POL, PK>(a, B, T, lk, boff, np, nmx, nmy, tau);
    double energy = 0.0;
    if (a.last) {
        if (want_e) {
            double sp = 0, sm = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                sp += (double)np[b] * (double)np[b];
                sm += (double)nmx[b] * (double)nmx[b] + (double)nmy[b] * (double)nmy[b];
            }
            energy = 0.5 * (a.emat[(long long)1 * nic + ic] * sp + a.emat[ic] * sm);
        }
        if (a.rec_first) {
            for (int e = a.rec_first[ic]; e >= 0;) {
                const RecDev &rc = a.rec[e];
                double v = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) v += rc.phi[b] * (double)np[b];
                const int step = uni(a.clock)->step;
                if (step < a.rec_steps) {
                    double *o = a.rec_out + (((long long)shot * a.rec_steps + step) * a.nrec + rc.r) * 2;
                    o[0] = v;
                    o[1] = 0.0;
                }
                e = rc.next;
            }
        }
    }
    return energy;
}

// ------------------------------------------------------------------------- solid cells
template <int K, int NF, typename R, bool STORE, int POL, bool PK>
__device__ __forceinline__ double solid_stage(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T,
                                              int nF, const LaneInfo &L, bool want_e) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const int nic = a.n_ic, ic = L.ic, shot = L.shot;
    const unsigned boff = L.boff, coff = L.coff;
    const R r2 = R(kRsqrt2);
    int lk[NF];
    R cc[NF], rn[NF][2][F];
    R fv[STORE ? NF : 1][2][F];  // face values, kept for the recompute stores
    load_links<NF, R>(B, nF, ic, lk, cc);
    constexpr bool KEEP = keep_in_registers<K, R>();
    R y[5 * N], uk[KEEP ? 5 * N : 1], dk[KEEP ? 5 * N : 1];
    load_state<5 * N, R, KEEP, lds_increment<K, R, STORE, PK>()>(a, B, boff, y, uk, dk);
    const R *vx = y, *vy = y + N, *s1 = y + 2 * N, *s2 = y + 3 * N, *s3 = y + 4 * N;
    load_incoming<K, NF, R>(B, kSolid, a.S, shot, lk, rn);
    const R tau = bld<R>(B.r, coff, B.mat + kTau * B.crowb);
    const R itau = bld<R>(B.r, coff, B.mat + kInvTau * B.crowb);
    const R irho = bld<R>(B.r, coff, B.mat + kInvRho * B.crowb);
    const R l2m = bld<R>(B.r, coff, B.mat + kStiff * B.crowb);
    const R lam = bld<R>(B.r, coff, B.mat + kLam * B.crowb);
    const R tmu = bld<R>(B.r, coff, B.mat + kTwoMu * B.crowb);
    R rvx[N], rvy[N], rs1[N], rs2[N], rs3[N], tvx[N], tvy[N], hs3[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        tvx[b] = tau * vx[b];
        tvy[b] = tau * vy[b];
        hs3[b] = r2 * s3[b];
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R a1 = 0, a2 = 0, a3 = 0, bx = 0, by = 0;
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
        }
        rs1[r] = a1;
        rs2[r] = a2;
        rs3[r] = r2 * a3;
        rvx[r] = -bx;
        rvy[r] = -by;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;  // boundary face: v_F = 0 (homogeneous Dirichlet)
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
            // interface, neighbour fluid: n_G = n_T, eliminate p_F then v_F
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const R pF = (rn[j][0][i] - (nx * rx[i] + ny * ry[i]) * itau) * cc[j];
                vFx[i] = (rx[i] + nx * pF) * itau;
                vFy[i] = (ry[i] + ny * pF) * itau;
            }
        }
        if (STORE) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                fv[j][0][i] = vFx[i];
                fv[j][1][i] = vFy[i];
            }
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            R wx = 0, wy = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if (!g_nonzero(b, i)) continue;
                wx += T.g(j, b, i) * vFx[i];
                wy += T.g(j, b, i) * vFy[i];
            }
            rs1[b] += nx * wx;
            rs2[b] += ny * wy;
            rs3[b] += r2 * (ny * wx + nx * wy);
            rvx[b] += tau * wx;
            rvy[b] += tau * wy;
        }
    }
    for (int m = 0; m < a.nterms; ++m) {
        const R w = R(sin(a.omega[m] * stage_time(a, shot) + a.phase[m]));
        const int gr = m * 5 * N;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            rvx[b] += w * a.gload[(long long)(gr + b) * nic + ic];
            rvy[b] += w * a.gload[(long long)(gr + N + b) * nic + ic];
            rs1[b] += w * a.gload[(long long)(gr + 2 * N + b) * nic + ic];
            rs2[b] += w * a.gload[(long long)(gr + 3 * N + b) * nic + ic];
            rs3[b] += w * a.gload[(long long)(gr + 4 * N + b) * nic + ic];
        }
    }
    if (a.src_first) {
        for (int e = a.src_first[ic]; e >= 0;) {
            const SrcDev &s = a.src[e];
            if (s.shot == shot) {
                const double w = s.amp * ricker(stage_time(a, shot), s.f0, s.t0);
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
    R kv[5 * N], nw[5 * N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        kv[b] = irho * rvx[b];
        kv[N + b] = irho * rvy[b];
        kv[2 * N + b] = l2m * rs1[b] + lam * rs2[b];
        kv[3 * N + b] = lam * rs1[b] + l2m * rs2[b];
        kv[4 * N + b] = tmu * rs3[b];
    }
    rk_update<5 * N, R, KEEP, POL, chunked_combine<K, R, STORE, PK>(), lds_increment<K, R, STORE, PK>()>(
        a, B, boff, y, kv, nw, uk, dk, shot);
    const R *nvx = nw, *nvy = nw + N, *ns1 = nw + 2 * N, *ns2 = nw + 3 * N, *ns3 = nw + 4 * N;
    if (STORE) store_recompute<K, NF, 5 * N, R, NF, 2>(a, lk, boff, y, kv, fv);
    solid_traces<K, NF, R, POL, PK>(a, B, T, lk, boff, nvx, nvy, ns1, ns2, ns3, tau, itau);
    double energy = 0.0;
    if (a.last) {
        if (want_e) {
            const double ca = a.emat[(long long)1 * nic + ic], cb = a.emat[(long long)2 * nic + ic];
            const double c3 = a.emat[(long long)3 * nic + ic];
            double sv = 0, ss = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const double x1 = ns1[b], x2 = ns2[b], x3 = ns3[b];
                sv += (double)nvx[b] * (double)nvx[b] + (double)nvy[b] * (double)nvy[b];
                ss += ca * (x1 * x1 + x2 * x2) + 2.0 * cb * x1 * x2 + c3 * x3 * x3;
            }
            energy = 0.5 * (a.emat[ic] * sv + ss);
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
                const int step = uni(a.clock)->step;
                if (step < a.rec_steps) {
                    double *o = a.rec_out + (((long long)shot * a.rec_steps + step) * a.nrec + rc.r) * 2;
                    o[0] = v0;
                    o[1] = v1;
                }
                e = rc.next;
            }
        }
    }
    return energy;
}

// One lane's stage; returns its energy (the last stage with energy recording), else 0.
template <int K, int NF, typename R, bool STORE, int POL, bool POOLED>
__device__ __forceinline__ double stage_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L, bool want_e) {
    const Tab<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    if (G.medium == kFluid) return fluid_stage<K, NF, R, STORE, POL, POOLED>(a, B, T, G.nF, L, want_e);
    return solid_stage<K, NF, R, STORE, POL, POOLED>(a, B, T, G.nF, L, want_e);
}

// With pooled groups a stage is two launches over the same grid: the one for the ordinary groups
// (POOLED = false, which also advances the clock) and the one for the pooled groups; each
// workgroup of a launch whose group is of the other kind returns at once.  When every group is
// pooled only the pooled launch runs, and it advances the clock.
template <int K, typename R, bool STORE, int POL, bool POOLED = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(stage_waves<K, R, STORE, POOLED>(), 8))) void stage_kernel(
    StageArgs<R> a) {
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
        // faces beyond a cell's count carry link -1 and are skipped like boundary faces
        if (G.nF <= 4) e = stage_body<K, 4, R, STORE, POL, POOLED>(a, G, L, want_e);
        else e = stage_body<K, kMaxFaces, R, STORE, POL, POOLED>(a, G, L, want_e);
    }
    if (want_e) block_energy(e, a.S, a.cpb, energy_slot(a));
}

// Outgoing trace contributions of the state in a.Yin (used once after the state is set).
template <int K, int NF, typename R, bool POOLED>
__device__ __forceinline__ void traces_body(const StageArgs<R> &a, const GroupDev &G, const LaneInfo &L) {
    constexpr int N = Dim<K>::N;
    const Tab<K, R, POOLED> T{class_table<POOLED>(a, G, L.ic), G.nF};
    const Bufs<R> B = make_bufs(a);
    int lk[NF];
    load_links<NF, R>(B, G.nF, L.ic, lk, (R *)nullptr);
    const R tau = bld<R>(B.r, L.coff, B.mat + kTau * B.crowb);
    const R itau = bld<R>(B.r, L.coff, B.mat + kInvTau * B.crowb);
    R v[5][N];
    const int nb = G.medium == kFluid ? 3 : 5;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int b = 0; b < N; ++b) v[q][b] = q < nb ? bld<R>(B.r, L.boff, B.yin + (q * N + b) * B.rowb) : R(0);
    if (G.medium == kFluid)
        fluid_traces<K, NF, R, 0, POOLED>(a, B, T, lk, L.boff, v[0], v[1], v[2], tau);
    else
        solid_traces<K, NF, R, 0, POOLED>(a, B, T, lk, L.boff, v[0], v[1], v[2], v[3], v[4], tau, itau);
}

template <int K, typename R, bool POOLED = false>
__global__ __launch_bounds__(kBlock) void trace_kernel(StageArgs<R> a) {
    GroupDev G;
    const LaneInfo L = decode_lane(a, G);
    if (!L.active || ((POOLED || a.has_pooled) && (G.pooled != 0) != POOLED)) return;
    if (G.nF <= 4) traces_body<K, 4, R, POOLED>(a, G, L);
    else traces_body<K, kMaxFaces, R, POOLED>(a, G, L);
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
        const int nb = G.medium == kFluid ? 3 : 5;
        const Bufs<R> B = make_bufs(a);
        double v[5][N];
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int b = 0; b < N; ++b)
                v[q][b] = q < nb ? (double)bld<R>(B.r, L.boff, B.yin + (q * N + b) * B.rowb) : 0.0;
        if (G.medium == kFluid) {
            double sp = 0, sm = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                sp += v[0][b] * v[0][b];
                sm += v[1][b] * v[1][b] + v[2][b] * v[2][b];
            }
            e = 0.5 * (a.emat[(long long)nic + ic] * sp + a.emat[ic] * sm);
        } else {
            const double ca = a.emat[(long long)nic + ic], cb = a.emat[(long long)2 * nic + ic];
            const double c3 = a.emat[(long long)3 * nic + ic];
            double sv = 0, ss = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                sv += v[0][b] * v[0][b] + v[1][b] * v[1][b];
                ss += ca * (v[2][b] * v[2][b] + v[3][b] * v[3][b]) + 2.0 * cb * v[2][b] * v[3][b] +
                      c3 * v[4][b] * v[4][b];
            }
            e = 0.5 * (a.emat[ic] * sv + ss);
        }
    }
    block_energy(e, a.S, a.cpb, a.e_part);
}


// Sum of the energy partials of every block, one workgroup of kReduceBlock lanes per shot: four
// independent partial sums per lane (loads in flight together), a shuffle fold per wavefront, and
// the wavefronts' sums added in LDS.
constexpr int kReduceBlock = 1024;
__global__ __launch_bounds__(kReduceBlock) void energy_reduce_kernel(const double *part, int n_blocks, int S,
                                                                     double *out, const Clock *clock, int cap) {
    __shared__ double buf[kReduceBlock / 64];
    const int s = blockIdx.x, tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int b = tid;
    for (; b + 3 * kReduceBlock < n_blocks; b += 4 * kReduceBlock)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += part[(long long)(b + u * kReduceBlock) * S + s];
    for (; b < n_blocks; b += kReduceBlock) acc[0] += part[(long long)b * S + s];
    double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) buf[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kReduceBlock / 64; ++w) t += buf[w];
        if (!clock) out[s] = t;
        else if (clock->step < cap) out[(long long)clock->step * S + s] = t;
    }
}

// History of several steps: workgroup (s, j) sums the partials of step clock->step - j, shot s.
__global__ __launch_bounds__(kReduceBlock) void energy_reduce_steps_kernel(const double *part, int n_blocks, int S,
                                                                           long long stride, int slots, double *out,
                                                                           const Clock *clock, int cap) {
    __shared__ double buf[kReduceBlock / 64];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int m = clock->step - (int)blockIdx.y;
    if (m < 0 || m >= cap) return;  // uniform over the workgroup
    const double *p = part + (long long)(m % slots) * stride;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int b = tid;
    for (; b + 3 * kReduceBlock < n_blocks; b += 4 * kReduceBlock)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += p[(long long)(b + u * kReduceBlock) * S + s];
    for (; b < n_blocks; b += kReduceBlock) acc[0] += p[(long long)b * S + s];
    double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) buf[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kReduceBlock / 64; ++w) t += buf[w];
        out[(long long)m * S + s] = t;
    }
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
    if (a.dim == 3) {
        if constexpr (K <= kMaxK3) return launch_stage3<K, R>(a, n_blocks, st);
        else return hipErrorNotSupported;
    }
    if (!a.all_pooled) {
        const size_t lds = lds_increment_bytes<K, R>(a.cpb * a.S);
        if (a.nt_stores)
            hipLaunchKernelGGL((stage_kernel<K, R, false, kNonTemporal>), dim3(n_blocks), dim3(a.cpb * a.S), lds, st, a);
        else
            hipLaunchKernelGGL((stage_kernel<K, R, false, 0>), dim3(n_blocks), dim3(a.cpb * a.S), lds, st, a);
    }
    if (a.has_pooled)
        hipLaunchKernelGGL((stage_kernel<K, R, false, 0, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_stage_store(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    if (a.dim == 3) return hipErrorNotSupported;  // the adjoint is two-dimensional
    if (!a.all_pooled)
        hipLaunchKernelGGL((stage_kernel<K, R, true, 0>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    if (a.has_pooled)
        hipLaunchKernelGGL((stage_kernel<K, R, true, 0, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_traces(const StageArgs<R> &a, int n_blocks, hipStream_t st) {
    if (a.dim == 3) {
        if constexpr (K <= kMaxK3) return launch_traces3<K, R>(a, n_blocks, st);
        else return hipErrorNotSupported;
    }
    if (!a.all_pooled) hipLaunchKernelGGL((trace_kernel<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    if (a.has_pooled) hipLaunchKernelGGL((trace_kernel<K, R, true>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, a);
    return hipGetLastError();
}

template <int K, typename R>
hipError_t launch_energy(const StageArgs<R> &a, const R *state, int n_blocks, hipStream_t st) {
    StageArgs<R> b = a;
    b.Yin = state;
    if (a.dim == 3) {
        if constexpr (K <= kMaxK3) return launch_energy3<K, R>(b, n_blocks, st);
        else return hipErrorNotSupported;
    }
    hipLaunchKernelGGL((energy_kernel<K, R>), dim3(n_blocks), dim3(a.cpb * a.S), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const double *part, int n_blocks, int S, double *out, const Clock *clock, int cap,
                                hipStream_t st) {
    hipLaunchKernelGGL(energy_reduce_kernel, dim3(S), dim3(kReduceBlock), 0, st, part, n_blocks, S, out, clock, cap);
    return hipGetLastError();
}

hipError_t launch_energy_reduce_steps(const double *part, int n_blocks, int S, long long stride, int slots,
                                      double *out, const Clock *clock, int count, int cap, hipStream_t st) {
    hipLaunchKernelGGL(energy_reduce_steps_kernel, dim3(S, count), dim3(kReduceBlock), 0, st, part, n_blocks, S,
                       stride, slots, out, clock, cap);
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
    template hipError_t launch_stage_store<K, R>(const StageArgs<R> &, int, hipStream_t);          \
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
