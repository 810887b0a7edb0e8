// Device helpers shared by the forward stage kernels (kernels.hip) and the adjoint stage
// kernels (adjoint.hip): buffer addressing of the arena, lane decoding, face links, incoming
// trace contributions (gathered from the neighbours) and the outgoing trace stores.  Included
// once per translation unit.
#pragma once

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

// Per-lane arrays are addressed through buffer resources: the uniform row offset goes in a
// scalar register, the lane's byte offset in a vector register, and the hardware range check
// against the array size turns a stray access into a zero load or a dropped store.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw (untyped) access

template <typename T>
__device__ __forceinline__ Rsrc rsrc(const T *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T bld(Rsrc r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bld<float>(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ int bld<int>(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(int, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bld<double>(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// Stores take a cache policy POL: 0 = default, kNonTemporal = streaming (used when the working
// set of a context is larger than the last-level cache, so that stage outputs go through to
// memory while the launch runs instead of in one write-back at its end).
constexpr int kNonTemporal = 2;
template <int POL = 0>
__device__ __forceinline__ void bst(Rsrc r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, POL);
}
template <int POL = 0>
__device__ __forceinline__ void bst(Rsrc r, unsigned voff, unsigned soff, double v) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)voff, (int)soff, POL);
}

// D contiguous dwords of one lane in the widest buffer accesses (16, 12, 8, 4 bytes).
typedef unsigned Dw2 __attribute__((ext_vector_type(2)));
typedef unsigned Dw3 __attribute__((ext_vector_type(3)));
typedef unsigned Dw4 __attribute__((ext_vector_type(4)));
template <int D, int O = 0>
__device__ __forceinline__ void bld_dw(Rsrc r, unsigned voff, unsigned soff, unsigned *w) {
    if constexpr (D - O >= 4) {
        const Dw4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)(soff + 4 * O), 0);
        w[O] = v.x, w[O + 1] = v.y, w[O + 2] = v.z, w[O + 3] = v.w;
        bld_dw<D, O + 4>(r, voff, soff, w);
    } else if constexpr (D - O == 3) {
        const Dw3 v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)voff, (int)(soff + 4 * O), 0);
        w[O] = v.x, w[O + 1] = v.y, w[O + 2] = v.z;
    } else if constexpr (D - O == 2) {
        const Dw2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)(soff + 4 * O), 0);
        w[O] = v.x, w[O + 1] = v.y;
    } else if constexpr (D - O == 1) {
        w[O] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)(soff + 4 * O), 0);
    }
}
template <int D, int O = 0, int POL = 0>
__device__ __forceinline__ void bst_dw(Rsrc r, unsigned voff, unsigned soff, const unsigned *w) {
    if constexpr (D - O >= 4) {
        const Dw4 v = {w[O], w[O + 1], w[O + 2], w[O + 3]};
        __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)(soff + 4 * O), POL);
        bst_dw<D, O + 4, POL>(r, voff, soff, w);
    } else if constexpr (D - O == 3) {
        const Dw3 v = {w[O], w[O + 1], w[O + 2]};
        __builtin_amdgcn_raw_buffer_store_b96(v, r, (int)voff, (int)(soff + 4 * O), POL);
    } else if constexpr (D - O == 2) {
        const Dw2 v = {w[O], w[O + 1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)(soff + 4 * O), POL);
    } else if constexpr (D - O == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(w[O], r, (int)voff, (int)(soff + 4 * O), POL);
    }
}
// F contiguous reals of one lane: v[i] at byte soff + i sizeof(R) (plus the lane's voff).
template <int F, typename R>
__device__ __forceinline__ void bldv(Rsrc r, unsigned voff, unsigned soff, R *v) {
    constexpr int D = F * (int)sizeof(R) / 4;
    unsigned w[D];
    bld_dw<D>(r, voff, soff, w);
#pragma unroll
    for (int i = 0; i < F; ++i) {
        if constexpr (sizeof(R) == 4) v[i] = __builtin_bit_cast(R, w[i]);
        else v[i] = __builtin_bit_cast(R, ((unsigned long long)w[2 * i + 1] << 32) | w[2 * i]);
    }
}
template <int F, typename R, int POL = 0>
__device__ __forceinline__ void bstv(Rsrc r, unsigned voff, unsigned soff, const R *v) {
    constexpr int D = F * (int)sizeof(R) / 4;
    unsigned w[D];
#pragma unroll
    for (int i = 0; i < F; ++i) {
        if constexpr (sizeof(R) == 4) {
            w[i] = __builtin_bit_cast(unsigned, v[i]);
        } else {
            const unsigned long long b = __builtin_bit_cast(unsigned long long, v[i]);
            w[2 * i] = (unsigned)b;
            w[2 * i + 1] = (unsigned)(b >> 32);
        }
    }
    bst_dw<D, 0, POL>(r, voff, soff, w);
}

// Buffer addressing of one stage launch (uniform): one resource over the arena, and the
// byte offset of each array in it.
template <typename R>
struct Bufs {
    Rsrc r;
    unsigned yin, yout, u, acc, tin, tout, link, c0, mat, yq;
    unsigned rowb;   // bytes of one [lane] row: LT * sizeof(R)
    unsigned crowb;  // bytes of one [cell] row of reals: n_ic * sizeof(R)
    unsigned irowb;  // bytes of one [cell] row of int32: n_ic * 4
};

template <typename R>
__device__ __forceinline__ Bufs<R> make_bufs(const StageArgs<R> &a) {
    Bufs<R> b;
    b.r = rsrc(a.arena, a.arena_bytes);
    b.yin = a.o_yin;
    b.yout = a.o_yout;
    b.u = a.o_u;
    b.acc = a.o_acc;
    b.tin = a.o_tin;
    b.tout = a.o_tout;
    b.link = a.o_link;
    b.c0 = a.o_c0;
    b.mat = a.o_mat;
    b.yq = a.o_yq;
    b.rowb = (unsigned)a.LT * (unsigned)sizeof(R);
    b.crowb = (unsigned)a.n_ic * (unsigned)sizeof(R);
    b.irowb = (unsigned)a.n_ic * 4u;
    return b;
}

// Time step of a shot: the clock's dt, times the shot's multiplier when one is set.
template <typename R>
__device__ __forceinline__ double shot_dt(const StageArgs<R> &a, int shot) {
    const double dt = uni(a.clock)->dt;
    return a.dt_scale ? dt * a.dt_scale[shot] : dt;
}

// Time of the current stage of a shot: t_n + c dt with t_n = t0 + step dt.
template <typename R>
__device__ __forceinline__ double stage_time(const StageArgs<R> &a, int shot) {
    const HHO_CONST Clock *c = uni(a.clock);
    return c->t0 + ((double)c->step + a.c) * shot_dt(a, shot);
}

template <typename R>
__device__ __forceinline__ R sgn(int i) {
    return (i & 1) ? R(-1) : R(1);
}

__device__ __forceinline__ double ricker(double t, double f0, double t0) {
    const double a = 3.14159265358979323846 * f0 * (t - t0);
    return (1.0 - 2.0 * a * a) * exp(-a * a);
}

constexpr double kRsqrt2 = 0.70710678118654752440;

// Total degree of the i-th function of the graded cell basis (degree-major order, k <= 3).
constexpr int kBasisDegree[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};

// B_c = D_c - sum_j n_{j,c} E_j equals -D_c^T (integration by parts), and in the orthonormal
// graded basis the derivative of a basis function is orthogonal to every basis function of equal
// or higher degree, so B_c[r][b] can be nonzero only when deg(b) < deg(r).  The host plan stores
// exact zeros there; the kernels skip those products at compile time.
__device__ constexpr bool b_nonzero(int r, int b) { return kBasisDegree[b] < kBasisDegree[r]; }

// G_j[a][i] = (phi_a, psi_i)_F: the trace of phi_a on a straight face is a polynomial of degree
// deg(a), orthogonal to the face Legendre polynomial psi_i of higher degree, so G_j[a][i] can be
// nonzero only when i <= deg(a) (exact zeros in the host plan as well).
__device__ constexpr bool g_nonzero(int a, int i) { return i <= kBasisDegree[a]; }

// Class tables.  Shared (group) tables are dense: B_x, B_y, S (N x N row-major), then per face G_j
// (N x F) and n_j (2).  The per-cell tables of pooled groups, read by every lane, are packed
// without their structural zeros: the entries of B_x and of B_y with deg(b) < deg(r) (row-major),
// the upper triangle of the symmetric S (r <= b, row-major), per face the entries of G_j with
// i <= deg(a) (row-major), then the normals.  Tab reads either layout by compile-time indices.
template <int K>
struct Packed {
    static constexpr int N = Dim<K>::N, F = Dim<K>::F;
    static constexpr int count_b() {
        int c = 0;
        for (int r = 0; r < N; ++r)
            for (int b = 0; b < N; ++b) c += kBasisDegree[b] < kBasisDegree[r];
        return c;
    }
    static constexpr int count_g() {
        int c = 0;
        for (int a = 0; a < N; ++a)
            for (int i = 0; i < F; ++i) c += i <= kBasisDegree[a];
        return c;
    }
    static constexpr int nB = count_b(), nS = N * (N + 1) / 2, nG = count_g();
    static constexpr int bidx(int r, int b) {
        int c = 0;
        for (int rr = 0; rr < N; ++rr)
            for (int bb = 0; bb < N; ++bb) {
                if (rr == r && bb == b) return c;
                c += kBasisDegree[bb] < kBasisDegree[rr];
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
                c += ii <= kBasisDegree[aa];
            }
        return -1;
    }
};

template <int K, typename R, bool PACKED>
struct Tab {
    static constexpr int N = Dim<K>::N, F = Dim<K>::F;
    using P = Packed<K>;
    const HHO_CONST R *t;
    int nF;  // faces of the table layout
    __device__ __forceinline__ R bx(int r, int b) const { return PACKED ? t[P::bidx(r, b)] : t[r * N + b]; }
    __device__ __forceinline__ R by(int r, int b) const {
        return PACKED ? t[P::nB + P::bidx(r, b)] : t[N * N + r * N + b];
    }
    __device__ __forceinline__ R s(int r, int b) const {
        return PACKED ? t[2 * P::nB + P::sidx(r, b)] : t[2 * N * N + r * N + b];
    }
    __device__ __forceinline__ R g(int j, int a, int i) const {
        return PACKED ? t[2 * P::nB + P::nS + j * P::nG + P::gidx(a, i)] : t[3 * N * N + (j * N + a) * F + i];
    }
    __device__ __forceinline__ R n(int j, int c) const {
        return PACKED ? t[2 * P::nB + P::nS + nF * P::nG + 2 * j + c] : t[3 * N * N + nF * N * F + 2 * j + c];
    }
};

struct LaneInfo {
    int ic, shot;
    unsigned boff;   // byte offset of this lane in a [row][lane] array of reals
    unsigned coff;   // byte offset of this cell in a [row][cell] array of reals
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
    G.pooled = gd->pooled;
    LaneInfo L;
    const int tid = threadIdx.x;
    const int cl = tid / a.S;
    L.shot = tid - cl * a.S;
    const int l = (blockIdx.x - G.blk_begin) * a.cpb + cl;
    L.active = l < G.ncells;
    L.ic = G.ic_begin + l;
    L.boff = (unsigned)(L.ic * a.S + L.shot) * (unsigned)sizeof(R);
    L.coff = (unsigned)L.ic * (unsigned)sizeof(R);
    return L;
}

// Per-cell face data: links (rows j >= nF of this group are never read; their links count
// as -1, like boundary faces) and face-solve coefficients.
template <int NF, typename R>
__device__ __forceinline__ void load_links(const Bufs<R> &B, int nF, int ic, int *lk, R *cc) {
    const unsigned ioff = (unsigned)ic * 4u, roff = (unsigned)ic * (unsigned)sizeof(R);
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        lk[j] = -1;
        if (cc) cc[j] = R(0);
        if (j < nF) {
            lk[j] = bld<int>(B.r, ioff, B.link + j * B.irowb);
            if (cc) cc[j] = bld<R>(B.r, roff, B.c0 + j * B.crowb);
        }
    }
}

// Neighbour contributions across the faces of a lane.  Trace buffers are [slot = 2 j + c][lane]
// [mode i] (byte offset ((2 j + c) LT + lane) F sizeof(R) + i sizeof(R)); every lane stores the
// contributions of its own faces in its own slots (coalesced stores, see fluid_traces) and
// gathers its neighbours' here: across face j the neighbour icn = link >> 4 wrote slot 2 jn + c of
// its lane (icn, shot), jn = link & 7.  Boundary faces (link -1) read nothing.  Components: a
// fluid neighbour writes c = 0 (its scalar contribution), a solid one c = 0 and 1 (the vector);
// a fluid cell reads c = 1 only across the interface, a solid cell only away from it.
template <int K, int NF, typename R>
__device__ __forceinline__ void load_incoming(const Bufs<R> &B, int medium, int S, int shot, const int *lk,
                                              R (*rn)[2][Dim<K>::F]) {
    constexpr int F = Dim<K>::F;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
#pragma unroll
        for (int i = 0; i < F; ++i) rn[j][0][i] = rn[j][1][i] = R(0);
        if (lk[j] < 0) continue;
        const int jn = lk[j] & 7;
        const bool itf = (lk[j] >> 3) & 1;
        const unsigned nb = (unsigned)((lk[j] >> 4) * S + shot) * (unsigned)sizeof(R);
        bldv<F, R>(B.r, F * nb, B.tin + (jn * 2) * F * B.rowb, rn[j][0]);
        if (medium == kSolid ? !itf : itf) bldv<F, R>(B.r, F * nb, B.tin + (jn * 2 + 1) * F * B.rowb, rn[j][1]);
    }
}

// Class tables: one per group, read through scalar loads; in a pooled group (cells of small
// shape classes together) each lane finds its class's table at its own offset and reads it
// through vector loads.
template <bool POOLED, typename R>
__device__ __forceinline__ const HHO_CONST R *class_table(const StageArgs<R> &a, const GroupDev &G, int ic) {
    return POOLED ? uni(a.tab) + a.ic_tab[ic] : uni(a.tab) + G.tab_off;
}

// ------------------------------------------------------------------------- outgoing traces
template <int K, int NF, typename R, int POL = 0, bool PK = false>
__device__ __forceinline__ void fluid_traces(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T,
                                             const int *lk, unsigned boff, const R *p, const R *mx, const R *my,
                                             R tau) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    R tp[N];
#pragma unroll
    for (int b = 0; b < N; ++b) tp[b] = tau * p[b];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        if (lk[j] < 0) continue;
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
        R o[F];
#pragma unroll
        for (int i = 0; i < F; ++i) o[i] = sgn<R>(i) * r[i];
        bstv<F, R, POL>(B.r, F * boff, B.tout + (j * 2) * F * B.rowb, o);
    }
}

template <int K, int NF, typename R, int POL = 0, bool PK = false>
__device__ __forceinline__ void solid_traces(const StageArgs<R> &a, const Bufs<R> &B, const Tab<K, R, PK> &T,
                                             const int *lk, unsigned boff, const R *vx, const R *vy, const R *s1,
                                             const R *s2, const R *s3, R tau, R itau) {
    constexpr int N = Dim<K>::N, F = Dim<K>::F;
    const R r2 = R(kRsqrt2);
    R tvx[N], tvy[N], hs3[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        tvx[b] = tau * vx[b];
        tvy[b] = tau * vy[b];
        hs3[b] = r2 * s3[b];
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
        // across the interface the fluid side needs r_s / tau_s
        const R w = ((lk[j] >> 3) & 1) ? itau : R(1);
        R ox[F], oy[F];
#pragma unroll
        for (int i = 0; i < F; ++i) {
            ox[i] = sgn<R>(i) * w * rx[i];
            oy[i] = sgn<R>(i) * w * ry[i];
        }
        bstv<F, R, POL>(B.r, F * boff, B.tout + (j * 2) * F * B.rowb, ox);
        bstv<F, R, POL>(B.r, F * boff, B.tout + (j * 2 + 1) * F * B.rowb, oy);
    }
}

// Energy partials of the current launch: the step's slot when partials are kept per step.
template <typename R>
__device__ __forceinline__ double *energy_slot(const StageArgs<R> &a) {
    if (a.e_slots <= 1) return a.e_part;
    return a.e_part + (long long)(uni(a.clock)->step % a.e_slots) * a.e_stride;
}

// Block reduction of per-lane energies into one partial per shot: lanes are (cell, shot) with the
// shot fastest, so lanes l and l + S hold the same shot.  When S divides the wavefront size, each
// wavefront folds its lanes with shuffles (offsets 32, 16, ... down to S keep the shot), and the
// first S lanes of the block add the wavefronts' partials; otherwise one lane per shot adds its
// block's cells through LDS.
__device__ void block_energy(double e, int S, int cpb, double *out) {
    __shared__ double buf[kBlock];
    const int tid = threadIdx.x;
    if (64 % S == 0) {
        for (int off = 32; off >= S; off >>= 1) e += __shfl_down(e, off, 64);
        const int wave = tid >> 6, lane = tid & 63;
        if (lane < S) buf[wave * S + lane] = e;
        __syncthreads();
        if (tid < S) {
            const int waves = (cpb * S + 63) >> 6;
            double s = 0;
            for (int w = 0; w < waves; ++w) s += buf[w * S + tid];
            out[(long long)blockIdx.x * S + tid] = s;
        }
        return;
    }
    buf[tid] = e;
    __syncthreads();
    if (tid < S) {
        double s = 0;
        for (int m = 0; m < cpb; ++m) s += buf[tid + m * S];
        out[(long long)blockIdx.x * S + tid] = s;
    }
}

}  // namespace
}  // namespace hho
