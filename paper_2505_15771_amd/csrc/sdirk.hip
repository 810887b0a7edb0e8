// SDIRK engine: device kernels and the C ABI of include/hho_sdirk.h.
//
// One SDIRK stage (Sec. 4.1, eq. SDIRK_compact and the two solves following eq. cp_dirk), float64,
// with every cell vector stored [row][cell] per cell group (medium, face-slot count):
//   1. B_T = M U^n + dt sum_{j<=i} a_ij F_j - dt sum_{j<i} a_ij Y_j       (stage_rhs, src_add)
//      with Y_j = K_T U_T^j + K_TF U_F^j the cell rows of K applied to stage j;
//   2. g = A_T^{-1} B_T and the per-slot products V_T B_T (cell_apply: one lane per output row
//      of the stacked per-cell matrix [A_T^{-1}; V_T], coalesced over the cells of a group);
//   3. face right-hand side b = B_F - sum_T V_T B_T (face_rhs), with
//      B_F^i = -sum_{j<i} (a_ij / a*) E_j and E_j = a* dt (K_FT U_T^j + K_F U_F^j) the face rows
//      of stage j (E_j = B_F^j minus the final residual of its face solve);
//   4. BiCGStab on S x = b, S = a* dt (K_F - a* dt K_FT A^{-1} K_TF), face-block Jacobi on the
//      right; scalars stay on the device, the host checks the residual every few iterations;
//   5. U_T = g - W_T x (recover) and Y_i = (B_T - M U_T) / (a* dt) (stage_Y: the stage equation
//      A_T U_T + a* dt K_TF U_F = B_T rearranged, so K is never applied);
//   last: U^{n+1} = U^n + dt M^{-1} sum_j b_j (F_j - Y_j) (final, src_add).
// The algebra of steps 3 and 5 is that of the printed scheme: it only uses the stage equations
// the solves satisfy (the face rows up to the residual that E_j carries).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/hho_sdirk.h"
#include "implicit_plan.h"
#include "initial.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxGroups = 32;

struct GroupTable {
    int ng;
    int medium[kMaxGroups], nT[kMaxGroups], nFT[kMaxGroups], n[kMaxGroups];
    long long vec_off[kMaxGroups], cf_off[kMaxGroups], mat_off[kMaxGroups], w_off[kMaxGroups], m_off[kMaxGroups];
    long long item_off[kMaxGroups + 1];  // items of the launch, per group (prefix)
    int Np, N;
};

__device__ __forceinline__ int find_group(const GroupTable &G, long long e) {
    int g = 0;
    while (g + 1 < G.ng && e >= G.item_off[g + 1]) ++g;
    return g;
}

// (M u)(e) for cell-vector element e = vec_off + r * n + i of group g
__device__ __forceinline__ double apply_mass(const GroupTable &G, int g, int r, int i, const double *u,
                                             const double *mat, bool inverse) {
    const int n = G.n[g];
    const long long vo = G.vec_off[g], mo = G.m_off[g];
    const double x = u[vo + (long long)r * n + i];
    if (G.medium[g] == 0) {
        if (r < G.Np) return x * mat[mo + (inverse ? 2 : 0) * n + i];
        return x * mat[mo + (inverse ? 3 : 1) * n + i];
    }
    if (r < 2 * G.Np) return x * mat[mo + (inverse ? 4 : 0) * n + i];
    const int q = r - 2 * G.Np, al = q / G.N, a = q - al * G.N;
    const double ca = mat[mo + (inverse ? 5 : 1) * n + i], cb = mat[mo + (inverse ? 6 : 2) * n + i];
    const double cc = mat[mo + (inverse ? 7 : 3) * n + i];
    const long long base = vo + (long long)(2 * G.Np + a) * n + i;
    const double s0 = u[base], s1 = u[base + (long long)G.N * n], s2 = u[base + 2LL * G.N * n];
    if (al == 0) return ca * s0 + cb * s1;
    if (al == 1) return cb * s0 + ca * s1;
    return cc * s2;
}

// B = M U0 - dt sum_{j<i} a_ij Y_j      (items: cell-vector elements)
__global__ void __launch_bounds__(kThreads) k_stage_rhs(GroupTable G, long long ndof, const double *__restrict__ U0,
                                                        const double *__restrict__ Y, int nprev, double w0, double w1,
                                                        const double *__restrict__ mat, double *__restrict__ B) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ndof) return;
    const int g = find_group(G, e);
    const long long loc = e - G.vec_off[g];
    const int r = (int)(loc / G.n[g]), i = (int)(loc - (long long)r * G.n[g]);
    double v = apply_mass(G, g, r, i, U0, mat, false);
    if (nprev > 0) v -= w0 * Y[e];
    if (nprev > 1) v -= w1 * Y[ndof + e];
    B[e] = v;
}

// out = mats x B per cell: rows [0, nT) -> g, rows [nT, nT + nFT) -> per-slot vector cf
__global__ void __launch_bounds__(kThreads) k_cell_apply(GroupTable G, long long nitems, const double *__restrict__ mats,
                                                         const double *__restrict__ B, double *__restrict__ gv,
                                                         double *__restrict__ cf) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= nitems) return;
    const int g = find_group(G, t);
    const int n = G.n[g], nT = G.nT[g];
    const long long loc = t - G.item_off[g];
    const int r = (int)(loc / n), i = (int)(loc - (long long)r * n);
    const double *m = mats + G.mat_off[g] + (long long)r * nT * n + i;
    const double *b = B + G.vec_off[g] + i;
    double acc = 0.0;
    for (int c = 0; c < nT; ++c) acc += m[(long long)c * n] * b[(long long)c * n];
    if (r < nT) gv[G.vec_off[g] + (long long)r * n + i] = acc;
    else cf[G.cf_off[g] + (long long)(r - nT) * n + i] = acc;
}

// bF_i = -sum_{j<i} (a_ij / a*) E_j ; rhs = D (bF_i - (V B) fed by the (at most two) cells)
__global__ void __launch_bounds__(kThreads) k_face_rhs(int nfd, const int *__restrict__ feed, const double *__restrict__ cf,
                                                       const double *__restrict__ E, int nprev, double q0, double q1,
                                                       const double *__restrict__ dsc, double *__restrict__ bF,
                                                       double *__restrict__ rhs) {
    const int d = blockIdx.x * kThreads + threadIdx.x;
    if (d >= nfd) return;
    double v = 0.0;
    if (nprev > 0) v -= q0 * E[d];
    if (nprev > 1) v -= q1 * E[(long long)nfd + d];
    bF[d] = v;
    const int f0 = feed[2 * d], f1 = feed[2 * d + 1];
    double s = v;
    if (f0 >= 0) s -= cf[f0];
    if (f1 >= 0) s -= cf[f1];
    rhs[d] = dsc[d] * s;   // right-hand side of the scaled system
}

// U = g - W x, x = D y the face unknowns     (items: cell-vector elements)
__global__ void __launch_bounds__(kThreads) k_recover(GroupTable G, long long ndof, const double *__restrict__ wmat,
                                                      const int *__restrict__ slot_dof, const double *__restrict__ y,
                                                      const double *__restrict__ dsc, const double *__restrict__ gv,
                                                      double *__restrict__ U) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ndof) return;
    const int g = find_group(G, e);
    const int n = G.n[g], nS = G.nFT[g];
    const long long loc = e - G.vec_off[g];
    const int r = (int)(loc / n), i = (int)(loc - (long long)r * n);
    const double *w = wmat + G.w_off[g] + (long long)r * nS * n + i;
    const int *sd = slot_dof + G.cf_off[g] + i;
    double acc = gv[e];
    for (int q = 0; q < nS; ++q) {
        const int d = sd[(long long)q * n];
        acc -= w[(long long)q * n] * (dsc[d] * y[d]);   // x = D y
    }
    U[e] = acc;
}

// Y_i = (B - M U) / (a* dt)
__global__ void __launch_bounds__(kThreads) k_stage_Y(GroupTable G, long long ndof, const double *__restrict__ B,
                                                      const double *__restrict__ U, const double *__restrict__ mat,
                                                      double inv_adt, double *__restrict__ Yi) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ndof) return;
    const int g = find_group(G, e);
    const long long loc = e - G.vec_off[g];
    const int r = (int)(loc / G.n[g]), i = (int)(loc - (long long)r * G.n[g]);
    Yi[e] = (B[e] - apply_mass(G, g, r, i, U, mat, false)) * inv_adt;
}

// U = U0 - dt M^{-1} sum_j b_j Y_j     (Z = sum_j b_j Y_j formed first into Zbuf)
__global__ void __launch_bounds__(kThreads) k_combine_Y(long long ndof, const double *__restrict__ Y, int s, double b0,
                                                        double b1, double b2, double *__restrict__ Z) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ndof) return;
    double v = b0 * Y[e];
    if (s > 1) v += b1 * Y[ndof + e];
    if (s > 2) v += b2 * Y[2 * ndof + e];
    Z[e] = v;
}

__global__ void __launch_bounds__(kThreads) k_final(GroupTable G, long long ndof, const double *__restrict__ U0,
                                                    const double *__restrict__ Z, const double *__restrict__ mat, double dt,
                                                    double *__restrict__ U) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ndof) return;
    const int g = find_group(G, e);
    const long long loc = e - G.vec_off[g];
    const int r = (int)(loc / G.n[g]), i = (int)(loc - (long long)r * G.n[g]);
    U[e] = U0[e] - dt * apply_mass(G, g, r, i, Z, mat, true);
}

struct SrcDev {
    long long idx;      // cell-vector element
    double coef;        // phi'_a(x_s) d
    double f0, t0, amp;
    double minv;        // inverse mass of that row (1/rho or kappa)
};

__device__ __forceinline__ double ricker(double t, double f0, double t0) {
    const double a = 3.14159265358979323846 * f0 * (t - t0);
    return (1.0 - 2.0 * a * a) * exp(-a * a);
}

// out[idx] += sum_j w_j amp R(t + c_j dt) coef (times minv when final)
__global__ void k_src_add(int n, const SrcDev *__restrict__ src, double t, double dt, int nw, double w0, double w1,
                          double w2, double c0, double c1, double c2, int final_update, double *__restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const SrcDev s = src[q];
    double acc = w0 * ricker(t + c0 * dt, s.f0, s.t0);
    if (nw > 1) acc += w1 * ricker(t + c1 * dt, s.f0, s.t0);
    if (nw > 2) acc += w2 * ricker(t + c2 * dt, s.f0, s.t0);
    acc *= dt * s.amp * s.coef;
    if (final_update) acc *= s.minv;
    atomicAdd(out + s.idx, acc);
}

// ---------------------------------------------------------------- BiCGStab
// Solver scalars live on the device.  Every dot product is summed per workgroup inside the kernel
// that produces its operands; the kernel that needs the result has each of its workgroups add
// those block sums itself (the same sums in the same order, so every workgroup gets the same
// value), and its workgroup 0 records the new scalars.  An iteration is five launches:
// p-update, S p_hat, s-update, S s_hat, x/r-update.  Iteration scalars are kept per parity of the
// iteration: iteration j reads block j & 1 and writes block (j & 1) ^ 1, so no workgroup reads a
// slot that workgroup 0 of the same launch writes.
enum Scalar { S_DONE = 0, S_BB, S_TOL2, S_TRR, S_ITER_OUT, S_RR_OUT, S_PAR = 8, kNumScalars = 32 };
enum ParScalar { P_RHO = 0, P_ALPHA, P_OMEGA, P_ITER, kParStride = 8 };

// Face matrix: row d's values val[ptr[d] .. ptr[d + 1]) against the columns cols[coff[d] + q];
// rows with the same column list (the rows of one face, as seen from its cells) share one list,
// so a nonzero moves 8 bytes plus a fraction of a column index.
// y = A x (mode 0) or y = b - A x (mode 1); 8 lanes per row
__global__ void __launch_bounds__(kThreads) k_spmv(int nrows, const int *__restrict__ ptr, const int *__restrict__ coff,
                                                   const int *__restrict__ cols, const double *__restrict__ val,
                                                   const double *__restrict__ x, const double *__restrict__ b,
                                                   double *__restrict__ y, int mode) {
    const int t = blockIdx.x * kThreads + threadIdx.x;
    const int row = t >> 3, lane = t & 7;
    double acc = 0.0;
    if (row < nrows) {
        const int v0 = ptr[row], len = ptr[row + 1] - v0;
        const int *cl = cols + coff[row];
        for (int q = lane; q < len; q += 8) acc += val[v0 + q] * x[cl[q]];
    }
    acc += __shfl_xor(acc, 4, 8);
    acc += __shfl_xor(acc, 2, 8);
    acc += __shfl_xor(acc, 1, 8);
    if (row < nrows && lane == 0) y[row] = mode ? b[row] - acc : acc;
}

// workgroup sums of two per-thread values into part[2 * blockIdx + {0, 1}]
__device__ __forceinline__ void block_partials(double x0, double x1, double *__restrict__ part) {
    __shared__ double s0[kThreads], s1[kThreads];
    s0[threadIdx.x] = x0;
    s1[threadIdx.x] = x1;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// the sums of nblk workgroup-sum pairs, in a fixed order (identical in every workgroup)
__device__ __forceinline__ void reduce_partials(int nblk, const double *__restrict__ part, double &a, double &b) {
    __shared__ double s0[kThreads], s1[kThreads];
    double x0 = 0.0, x1 = 0.0;
    for (int q = threadIdx.x; q < nblk; q += kThreads) {
        x0 += part[2 * q];
        x1 += part[2 * q + 1];
    }
    s0[threadIdx.x] = x0;
    s1[threadIdx.x] = x1;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    a = s0[0];
    b = s1[0];
    __syncthreads();
}

// partial sums of a.b and c.d per workgroup (grid-stride)
__global__ void __launch_bounds__(kThreads) k_dot2(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                   const double *__restrict__ c, const double *__restrict__ d,
                                                   double *__restrict__ part) {
    double x0 = 0.0, x1 = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < n; q += gridDim.x * kThreads) {
        x0 += a[q] * b[q];
        if (c) x1 += c[q] * d[q];
    }
    block_partials(x0, x1, part);
}

enum Finalize { F_INIT = 0, F_TRUE = 1 };

// one workgroup: reduce nblk partial pairs; F_INIT starts a solve (a = b.b, b = r.r with
// r_hat = r: the parity-0 scalars, and partA = (r.r, r_hat.r) in its first of nA pairs for the
// first iteration), F_TRUE stores a as the squared norm of a true residual
__global__ void __launch_bounds__(kThreads) k_finalize(int nblk, const double *__restrict__ part, double *__restrict__ sc,
                                                       int kind, double *__restrict__ partA, int nA) {
    double a, b;
    reduce_partials(nblk, part, a, b);
    if (kind == F_INIT) {
        for (int q = threadIdx.x; q < nA; q += kThreads) {
            partA[2 * q] = q == 0 ? b : 0.0;
            partA[2 * q + 1] = q == 0 ? b : 0.0;
        }
        if (threadIdx.x == 0) {
            double *p0 = sc + S_PAR;
            sc[S_BB] = a;
            sc[S_RR_OUT] = b;
            sc[S_ITER_OUT] = 0.0;
            p0[P_RHO] = b;
            p0[P_ALPHA] = 1.0;
            p0[P_OMEGA] = 1.0;
            p0[P_ITER] = 0.0;
            sc[S_DONE] = (b <= sc[S_TOL2] * a) ? 1.0 : 0.0;
        }
    } else if (threadIdx.x == 0) {
        sc[S_TRR] = a;
    }
}

// Face-block preconditioner: row d's block occupies the columns [pstart[d], pstart[d] + w) with
// w = pptr[d + 1] - pptr[d]; values pval[pptr[d] + j] (float32: the preconditioner only steers
// the iteration, the residual tests use the float64 matrix).

// iteration start: from the previous iteration's (r.r, r_hat.r) decide to stop (converged,
// breakdown, iteration limit); else beta = (rho / rho_old)(alpha / omega),
// p = r + beta (p_old - omega v) and p_hat = P p (the row's block of p recomputed from r, p_old, v)
__global__ void __launch_bounds__(kThreads) k_bicg_p(int n, const int *__restrict__ pptr, const int *__restrict__ pstart,
                                                     const float *__restrict__ pval, const double *__restrict__ r,
                                                     const double *__restrict__ v, const double *__restrict__ p_old,
                                                     double *__restrict__ p_new, double *__restrict__ ph, int nA,
                                                     const double *__restrict__ partA, double *__restrict__ sc, int par,
                                                     int max_iter) {
    if (sc[S_DONE] != 0.0) return;
    double rr, rho;
    reduce_partials(nA, partA, rr, rho);
    const double *so = sc + S_PAR + par * kParStride;
    double *sn = sc + S_PAR + (par ^ 1) * kParStride;
    const double it = so[P_ITER];
    int stop = 0;
    if (!isfinite(rr) || !isfinite(rho)) stop = 2;
    else if (rr <= sc[S_TOL2] * sc[S_BB]) stop = 1;
    else if (rho == 0.0 || so[P_OMEGA] == 0.0) stop = 2;
    else if (it >= (double)max_iter) stop = 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_RR_OUT] = rr;
        if (stop) {
            sc[S_DONE] = (double)stop;
        } else {
            sn[P_RHO] = rho;
            sn[P_ITER] = it + 1.0;
            sc[S_ITER_OUT] = it + 1.0;
        }
    }
    if (stop) return;
    const int d = blockIdx.x * kThreads + threadIdx.x;
    if (d >= n) return;
    const double beta = (rho / so[P_RHO]) * (so[P_ALPHA] / so[P_OMEGA]), om = so[P_OMEGA];
    const int q0 = pptr[d], w = pptr[d + 1] - q0, j0 = pstart[d];
    double acc = 0.0;
    for (int j = 0; j < w; ++j) acc += (double)pval[q0 + j] * (r[j0 + j] + beta * (p_old[j0 + j] - om * v[j0 + j]));
    p_new[d] = r[d] + beta * (p_old[d] - om * v[d]);
    ph[d] = acc;
}

// y = S x (8 lanes per row, grid-stride over rows) with the workgroup sums of (w.y) and (y.y); the grid
// is capped so that the consumers have few workgroup sums to add.  (Four rows per group of 8 lanes
// at a time, loaded together, measured 3 % faster at k = 1 and 6 % slower at k = 3.)
__global__ void __launch_bounds__(kThreads) k_bicg_spmv(int n, const int *__restrict__ ptr, const int *__restrict__ coff,
                                                        const int *__restrict__ cols, const double *__restrict__ val,
                                                        const double *__restrict__ x, double *__restrict__ y,
                                                        const double *__restrict__ w, double *__restrict__ part,
                                                        const double *__restrict__ sc) {
    if (sc[S_DONE] != 0.0) return;
    const int lane = threadIdx.x & 7;
    const int rows_per_pass = gridDim.x * (kThreads >> 3);
    double d0 = 0.0, d1 = 0.0;
    for (int base = 0; base < n; base += rows_per_pass) {
        const int row = base + blockIdx.x * (kThreads >> 3) + (threadIdx.x >> 3);
        double acc = 0.0;
        if (row < n) {
            const int v0 = ptr[row], len = ptr[row + 1] - v0;
            const int *cl = cols + coff[row];
            for (int q = lane; q < len; q += 8) acc += val[v0 + q] * x[cl[q]];
        }
        acc += __shfl_xor(acc, 4, 8);
        acc += __shfl_xor(acc, 2, 8);
        acc += __shfl_xor(acc, 1, 8);
        if (row < n && lane == 0) {
            y[row] = acc;
            d0 += w[row] * acc;
            d1 += acc * acc;
        }
    }
    block_partials(d0, d1, part);
}

// alpha = rho / (r_hat.v); s = r - alpha v and s_hat = P s
__global__ void __launch_bounds__(kThreads) k_bicg_s(int n, const int *__restrict__ pptr, const int *__restrict__ pstart,
                                                     const float *__restrict__ pval, const double *__restrict__ r,
                                                     const double *__restrict__ v, double *__restrict__ s,
                                                     double *__restrict__ sh, int nB, const double *__restrict__ partB,
                                                     double *__restrict__ sc, int par) {
    if (sc[S_DONE] != 0.0) return;
    double rv, unused;
    reduce_partials(nB, partB, rv, unused);
    double *sn = sc + S_PAR + (par ^ 1) * kParStride;
    if (rv == 0.0 || !isfinite(rv)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc[S_DONE] = 2.0;
        return;
    }
    const double al = sn[P_RHO] / rv;
    if (blockIdx.x == 0 && threadIdx.x == 0) sn[P_ALPHA] = al;
    const int d = blockIdx.x * kThreads + threadIdx.x;
    if (d >= n) return;
    const int q0 = pptr[d], w = pptr[d + 1] - q0, j0 = pstart[d];
    double acc = 0.0;
    for (int j = 0; j < w; ++j) acc += (double)pval[q0 + j] * (r[j0 + j] - al * v[j0 + j]);
    s[d] = r[d] - al * v[d];
    sh[d] = acc;
}

// omega = (t.s) / (t.t); x += alpha p_hat + omega s_hat; r = s - omega t; sums of (r.r), (r_hat.r)
__global__ void __launch_bounds__(kThreads) k_bicg_x(int n, double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ rh, const double *__restrict__ ph,
                                                     const double *__restrict__ sh, const double *__restrict__ s,
                                                     const double *__restrict__ t, int nC,
                                                     const double *__restrict__ partC, double *__restrict__ partA,
                                                     double *__restrict__ sc, int par) {
    if (sc[S_DONE] != 0.0) return;
    double ts, tt;
    reduce_partials(nC, partC, ts, tt);
    double *sn = sc + S_PAR + (par ^ 1) * kParStride;
    const double om = tt > 0.0 ? ts / tt : 0.0, al = sn[P_ALPHA];
    if (blockIdx.x == 0 && threadIdx.x == 0) sn[P_OMEGA] = om;
    const int d = blockIdx.x * kThreads + threadIdx.x;
    double d0 = 0.0, d1 = 0.0;
    if (d < n) {
        x[d] += al * ph[d] + om * sh[d];
        const double rn = s[d] - om * t[d];
        r[d] = rn;
        d0 = rn * rn;
        d1 = rh[d] * rn;
    }
    block_partials(d0, d1, partA);
}

// E_i = bF_i - (b - S x), the true residual of the scaled system given in res
__global__ void __launch_bounds__(kThreads) k_face_rows(int n, const double *__restrict__ bF, const double *__restrict__ res,
                                                        const double *__restrict__ dsc, double *__restrict__ Ei) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= n) return;
    Ei[q] = bF[q] - res[q] / dsc[q];   // res = D (b - S x)
}

// out = ca a + cb b
__global__ void __launch_bounds__(kThreads) k_axpby(int n, double ca, const double *__restrict__ a, double cb,
                                                    const double *__restrict__ b, double *__restrict__ out) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q < n) out[q] = ca * a[q] + cb * b[q];
}

__global__ void __launch_bounds__(kThreads) k_copy(long long n, const double *__restrict__ a, double *__restrict__ b) {
    const long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q < n) b[q] = a[q];
}

// receiver r, component c: out[2 r + c] = sum_a coef[(2 r + c) Np + a] U[idx[(2 r + c) Np + a]]
__global__ void k_record(int n2, int Np, const long long *__restrict__ idx, const double *__restrict__ coef,
                         const double *__restrict__ U, double *__restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n2) return;
    double acc = 0.0;
    for (int a = 0; a < Np; ++a) {
        const long long e = idx[(long long)q * Np + a];
        if (e >= 0) acc += coef[(long long)q * Np + a] * U[e];
    }
    out[q] = acc;
}

// energy partial sums: 1/2 U . M U per block
__global__ void __launch_bounds__(kThreads) k_energy(GroupTable G, long long ndof, const double *__restrict__ U,
                                                     const double *__restrict__ mat, double *__restrict__ part) {
    __shared__ double s0[kThreads];
    double acc = 0.0;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < ndof; e += (long long)gridDim.x * kThreads) {
        const int g = find_group(G, e);
        const long long loc = e - G.vec_off[g];
        const int r = (int)(loc / G.n[g]), i = (int)(loc - (long long)r * G.n[g]);
        acc += 0.5 * U[e] * apply_mass(G, g, r, i, U, mat, false);
    }
    s0[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s0[threadIdx.x] += s0[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = s0[0]; part[2 * blockIdx.x + 1] = 0.0; }
}

unsigned grid_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

constexpr int kDotBlocks = 512;
constexpr int kSpmvBlocks = 1024;  // grid cap of the solver's matrix products
constexpr int kChunk = 8;  // BiCGStab iterations between residual checks (even: parities repeat)

}  // namespace

struct hho_sdirk {
    hho::imp::Plan plan;
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    double tol = 1e-10;
    int max_iter = 1000;
    std::vector<void *> allocs;
    GroupTable gvec{}, gmat{};
    // device buffers
    double *mats = nullptr, *wmat = nullptr, *mat = nullptr;
    int *slot_dof = nullptr, *feed = nullptr;
    int *S_ptr = nullptr, *S_coff = nullptr, *S_cols = nullptr, *P_ptr = nullptr, *P_start = nullptr;
    float *P_val = nullptr;
    double *S_val = nullptr, *dsc = nullptr;
    double *U = nullptr, *U0 = nullptr, *B = nullptr, *gv = nullptr, *Y = nullptr, *Z = nullptr, *cf = nullptr;
    double *E = nullptr, *bF = nullptr, *rhs = nullptr;
    double *x = nullptr, *r = nullptr, *rh = nullptr, *pb[2] = {nullptr, nullptr}, *v = nullptr, *s = nullptr;
    double *t = nullptr, *ph = nullptr, *sh = nullptr, *part = nullptr, *sc = nullptr;
    double *partA = nullptr, *partB = nullptr, *partC = nullptr;  // workgroup sums of the solver kernels
    // kChunk iterations captured once as a graph (fixed arguments), replayed per chunk
    hipStream_t cap = nullptr;
    hipGraphExec_t chunk = nullptr;
    double *h_sc = nullptr;  // pinned
    SrcDev *src = nullptr;
    int n_src = 0;
    // receivers: per (receiver, component) Np (element, coefficient) pairs; traces of the last call
    long long *rec_idx = nullptr;
    double *rec_coef = nullptr, *traces = nullptr;
    int n_rec = 0;
    size_t trace_cap = 0;
    int last_steps = 0;
    int64_t solves = 0, iterations = 0;
    int64_t n_shared_cols = 0;  // column indices stored for the face matrix
    // face solutions of every stage at the last two steps (initial guesses by extrapolation)
    double *xhist = nullptr;     // [stage][2][n_fdof], slot = step parity
    int64_t step_count = 0;      // steps since the state was set
    int hist_valid = 0;          // steps of history available (0, 1, 2)
    double max_res = 0.0;
};

namespace {

std::string g_sdirk_error;

#define SCK(call)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                \
            return e_ == hipErrorOutOfMemory ? HHO_ERR_OOM : HHO_ERR_DEVICE;             \
        }                                                                                \
    } while (0)

template <typename T>
hho_status dev_alloc(hho_sdirk *ctx, T **p, size_t count) {
    void *q = nullptr;
    size_t bytes = std::max<size_t>(count * sizeof(T), 8);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        ctx->err = "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? HHO_ERR_OOM : HHO_ERR_DEVICE;
    }
    ctx->allocs.push_back(q);
    *p = (T *)q;
    e = hipMemsetAsync(q, 0, bytes, ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
        return HHO_ERR_DEVICE;
    }
    return HHO_OK;
}

// free a buffer made by dev_alloc (null-safe)
void release(hho_sdirk *ctx, void *p) {
    if (!p) return;
    auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
    if (it != ctx->allocs.end()) ctx->allocs.erase(it);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(p);
}

template <typename T>
hho_status upload(hho_sdirk *ctx, T **p, const std::vector<T> &v) {
    hho_status st = dev_alloc(ctx, p, v.size());
    if (st != HHO_OK) return st;
    if (!v.empty()) SCK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    SCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

hho::imp::Options options_of(const hho_sdirk_params *p) {
    hho::imp::Options o;
    o.k = p->k;
    o.mixed = p->mixed;
    o.alpha = p->alpha;
    o.eta_f = p->eta_f;
    o.eta_s = p->eta_s;
    o.stab_speed = p->stab_speed;
    o.ell = p->ell;
    o.stages = p->stages;
    o.dt = p->dt;
    return o;
}

std::string build_plan(const hho_mesh *m, const hho_sdirk_params *p, hho::imp::Plan &P, int *code) {
    if (!m || !p) {
        *code = HHO_ERR_ARG;
        return "null mesh or params";
    }
    return hho::imp::build(m->n_vertices, m->xy, m->n_cells, m->cell_ptr, m->cell_vtx, m->medium, m->rho, m->a, m->b,
                           options_of(p), P, code);
}

void fill_groups(hho_sdirk *ctx) {
    const auto &P = ctx->plan;
    GroupTable G{};
    G.ng = (int)P.groups.size();
    G.Np = P.Np;
    G.N = P.N;
    for (int g = 0; g < G.ng; ++g) {
        const auto &q = P.groups[g];
        G.medium[g] = q.medium;
        G.nT[g] = q.nT;
        G.nFT[g] = q.nFT;
        G.n[g] = q.n;
        G.vec_off[g] = q.vec_off;
        G.cf_off[g] = q.cf_off;
        G.mat_off[g] = q.mat_off;
        G.w_off[g] = q.w_off;
        G.m_off[g] = q.m_off;
    }
    ctx->gvec = G;
    ctx->gmat = G;
    long long acc = 0;
    for (int g = 0; g < G.ng; ++g) {
        ctx->gvec.item_off[g] = P.groups[g].vec_off;
        ctx->gmat.item_off[g] = acc;
        acc += (long long)(P.groups[g].nT + P.groups[g].nFT) * P.groups[g].n;
    }
    ctx->gvec.item_off[G.ng] = P.n_dof;
    ctx->gmat.item_off[G.ng] = acc;
}

long long mat_items(const hho_sdirk *ctx) { return ctx->gmat.item_off[ctx->gmat.ng]; }

// dot products a.b (and c.d) reduced into the solver scalars (F_INIT starts a solve, F_TRUE stores
// the true residual)
hho_status dots(hho_sdirk *ctx, const double *a, const double *b, const double *c, const double *d, int kind) {
    const int n = ctx->plan.n_fdof;
    const int nblk = std::min<int>(kDotBlocks, std::max<int>(1, (int)grid_for(n)));
    hipLaunchKernelGGL(k_dot2, dim3(nblk), dim3(kThreads), 0, ctx->stream, n, a, b, c, d, ctx->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, ctx->stream, nblk, ctx->part, ctx->sc, kind, ctx->partA,
                       (int)grid_for(n));
    SCK(hipGetLastError());
    return HHO_OK;
}

// r = b - S x
hho_status residual(hho_sdirk *ctx, const double *x, const double *b, double *r) {
    const int n = ctx->plan.n_fdof;
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(8LL * n)), dim3(kThreads), 0, ctx->stream, n, ctx->S_ptr, ctx->S_coff,
                       ctx->S_cols, ctx->S_val, x, b, r, 1);
    SCK(hipGetLastError());
    return HHO_OK;
}

hho_status read_scalars(hho_sdirk *ctx) {
    SCK(hipMemcpyAsync(ctx->h_sc, ctx->sc, kNumScalars * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

// kChunk BiCGStab iterations, five launches each, on stream st (p alternates between two buffers
// and the iteration scalars between two blocks by iteration parity; kChunk is even, so every
// chunk starts from parity 0)
void enqueue_chunk(hho_sdirk *ctx, hipStream_t st) {
    const int n = ctx->plan.n_fdof;
    const dim3 gr(grid_for(n)), gs(std::min<unsigned>(grid_for(8LL * n), kSpmvBlocks)), b(kThreads);
    const int nA = (int)gr.x, nS = (int)gs.x;
    for (int it = 0; it < kChunk; ++it) {
        const int par = it & 1;
        hipLaunchKernelGGL(k_bicg_p, gr, b, 0, st, n, ctx->P_ptr, ctx->P_start, ctx->P_val, ctx->r, ctx->v,
                           ctx->pb[par], ctx->pb[par ^ 1], ctx->ph, nA, ctx->partA, ctx->sc, par, ctx->max_iter);
        hipLaunchKernelGGL(k_bicg_spmv, gs, b, 0, st, n, ctx->S_ptr, ctx->S_coff, ctx->S_cols, ctx->S_val, ctx->ph,
                           ctx->v, ctx->rh, ctx->partB, ctx->sc);
        hipLaunchKernelGGL(k_bicg_s, gr, b, 0, st, n, ctx->P_ptr, ctx->P_start, ctx->P_val, ctx->r, ctx->v, ctx->s,
                           ctx->sh, nS, ctx->partB, ctx->sc, par);
        hipLaunchKernelGGL(k_bicg_spmv, gs, b, 0, st, n, ctx->S_ptr, ctx->S_coff, ctx->S_cols, ctx->S_val, ctx->sh,
                           ctx->t, ctx->s, ctx->partC, ctx->sc);
        hipLaunchKernelGGL(k_bicg_x, gr, b, 0, st, n, ctx->x, ctx->r, ctx->rh, ctx->ph, ctx->sh, ctx->s, ctx->t, nS,
                           ctx->partC, ctx->partA, ctx->sc, par);
    }
}

// capture one chunk into a graph (once per context); on failure chunks are launched directly
void capture_chunk(hho_sdirk *ctx) {
    if (ctx->chunk || !ctx->cap) return;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return;
    enqueue_chunk(ctx, ctx->cap);
    if (hipStreamEndCapture(ctx->cap, &graph) != hipSuccess || !graph) {
        (void)hipGetLastError();
        return;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) == hipSuccess) ctx->chunk = ex;
    (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
}

#define SST(call)                          \
    do {                                   \
        hho_status s_ = (call);            \
        if (s_ != HHO_OK) return s_;       \
    } while (0)

// BiCGStab on the scaled face system (D S D) y = D b (y holds the initial guess, the previous
// stage's solution); then E_i = bF - (b - S x).  A solve whose recursively updated residual met the
// tolerance but whose true residual is more than 10 tol restarts from its iterate (residual
// replacement), at most three times; a breakdown restarts at most twice.
hho_status face_solve(hho_sdirk *ctx, double *Ei) {
    const int n = ctx->plan.n_fdof;
    if (n == 0) return HHO_OK;
    const unsigned gr = grid_for(n);
    int restarts = 0, replacements = 0;
    capture_chunk(ctx);
    for (;;) {
        SST(residual(ctx, ctx->x, ctx->rhs, ctx->r));
        hipLaunchKernelGGL(k_copy, dim3(gr), dim3(kThreads), 0, ctx->stream, (long long)n, ctx->r, ctx->rh);
        SCK(hipMemsetAsync(ctx->pb[0], 0, n * sizeof(double), ctx->stream));
        SCK(hipMemsetAsync(ctx->v, 0, n * sizeof(double), ctx->stream));
        SST(dots(ctx, ctx->rhs, ctx->rhs, ctx->r, ctx->r, F_INIT));
        SST(read_scalars(ctx));
        if (ctx->h_sc[S_BB] == 0.0) {   // zero right-hand side: the solution is zero
            SCK(hipMemsetAsync(ctx->x, 0, n * sizeof(double), ctx->stream));
            break;
        }
        while (ctx->h_sc[S_DONE] == 0.0) {
            if (ctx->chunk) SCK(hipGraphLaunch(ctx->chunk, ctx->stream));
            else enqueue_chunk(ctx, ctx->stream);
            SCK(hipGetLastError());
            SST(read_scalars(ctx));
        }
        ctx->iterations += (int64_t)ctx->h_sc[S_ITER_OUT];
        if (ctx->h_sc[S_DONE] == 1.0) {
            SST(residual(ctx, ctx->x, ctx->rhs, ctx->r));
            SST(dots(ctx, ctx->r, ctx->r, nullptr, nullptr, F_TRUE));
            SST(read_scalars(ctx));
            if (ctx->h_sc[S_TRR] <= 100.0 * ctx->h_sc[S_TOL2] * ctx->h_sc[S_BB] || replacements >= 3) break;
            ++replacements;
            continue;
        }
        if (ctx->h_sc[S_DONE] == 3.0 || restarts >= 2) {
            ctx->err = ctx->h_sc[S_DONE] == 3.0 ? "face solve: no convergence within max_iter iterations"
                                                : "face solve: BiCGStab broke down";
            return HHO_ERR_UNSTABLE;
        }
        ++restarts;  // breakdown: restart from the current iterate with a fresh shadow residual
    }
    // true residual and the face rows of this stage
    SST(residual(ctx, ctx->x, ctx->rhs, ctx->r));
    SST(dots(ctx, ctx->r, ctx->r, nullptr, nullptr, F_TRUE));
    hipLaunchKernelGGL(k_face_rows, dim3(gr), dim3(kThreads), 0, ctx->stream, n, ctx->bF, ctx->r, ctx->dsc, Ei);
    SCK(hipGetLastError());
    SST(read_scalars(ctx));
    ctx->solves += 1;
    if (ctx->h_sc[S_BB] > 0.0)
        ctx->max_res = std::max(ctx->max_res, std::sqrt(ctx->h_sc[S_TRR] / ctx->h_sc[S_BB]));
    return HHO_OK;
}

hho_status add_sources(hho_sdirk *ctx, double *out, double t, double dt, int nw, const double *w, const double *c,
                       int final_update) {
    if (ctx->n_src == 0) return HHO_OK;
    hipLaunchKernelGGL(k_src_add, dim3((ctx->n_src + 63) / 64), dim3(64), 0, ctx->stream, ctx->n_src, ctx->src, t, dt, nw,
                       w[0], nw > 1 ? w[1] : 0.0, nw > 2 ? w[2] : 0.0, c[0], nw > 1 ? c[1] : 0.0, nw > 2 ? c[2] : 0.0,
                       final_update, out);
    SCK(hipGetLastError());
    return HHO_OK;
}

hho_status one_step(hho_sdirk *ctx, double t) {
    const auto &P = ctx->plan;
    const long long nd = P.n_dof;
    const int s = P.stages;
    const double dt = P.dt, ast = P.ast, adt = ast * dt;
    const unsigned gv = grid_for(nd);
    hipLaunchKernelGGL(k_copy, dim3(gv), dim3(kThreads), 0, ctx->stream, nd, ctx->U, ctx->U0);
    for (int i = 0; i < s; ++i) {
        // B_T
        hipLaunchKernelGGL(k_stage_rhs, dim3(gv), dim3(kThreads), 0, ctx->stream, ctx->gvec, nd, ctx->U0, ctx->Y, i,
                           i > 0 ? dt * P.A[i][0] : 0.0, i > 1 ? dt * P.A[i][1] : 0.0, ctx->mat, ctx->B);
        SCK(hipGetLastError());
        double w[3] = {P.A[i][0], P.A[i][1], P.A[i][2]};
        SST(add_sources(ctx, ctx->B, t, dt, i + 1, w, P.c, 0));
        // g = A^{-1} B, cf = V B
        hipLaunchKernelGGL(k_cell_apply, dim3(grid_for(mat_items(ctx))), dim3(kThreads), 0, ctx->stream, ctx->gmat,
                           mat_items(ctx), ctx->mats, ctx->B, ctx->gv, ctx->cf);
        // face right-hand side
        if (P.n_fdof > 0)
            hipLaunchKernelGGL(k_face_rhs, dim3(grid_for(P.n_fdof)), dim3(kThreads), 0, ctx->stream, P.n_fdof, ctx->feed,
                               ctx->cf, ctx->E, i, i > 0 ? P.A[i][0] / ast : 0.0, i > 1 ? P.A[i][1] / ast : 0.0, ctx->dsc,
                               ctx->bF, ctx->rhs);
        SCK(hipGetLastError());
        // initial guess: the face solution of this stage at the previous steps, extrapolated
        // linearly from two steps when there are two, else the last one, else the previous stage's
        const int nf = P.n_fdof;
        double *h_last = ctx->xhist + ((size_t)i * 2 + ((ctx->step_count - 1) & 1)) * nf;
        double *h_prev = ctx->xhist + ((size_t)i * 2 + (ctx->step_count & 1)) * nf;
        if (nf > 0 && ctx->hist_valid >= 2)
            hipLaunchKernelGGL(k_axpby, dim3(grid_for(nf)), dim3(kThreads), 0, ctx->stream, nf, 2.0, h_last, -1.0, h_prev,
                               ctx->x);
        else if (nf > 0 && ctx->hist_valid == 1)
            hipLaunchKernelGGL(k_copy, dim3(grid_for(nf)), dim3(kThreads), 0, ctx->stream, (long long)nf, h_last, ctx->x);
        SST(face_solve(ctx, ctx->E + (size_t)i * P.n_fdof));
        if (nf > 0)
            hipLaunchKernelGGL(k_copy, dim3(grid_for(nf)), dim3(kThreads), 0, ctx->stream, (long long)nf, ctx->x, h_prev);
        // cell recovery and the cell rows of K U^{n,i}
        hipLaunchKernelGGL(k_recover, dim3(gv), dim3(kThreads), 0, ctx->stream, ctx->gvec, nd, ctx->wmat, ctx->slot_dof,
                           ctx->x, ctx->dsc, ctx->gv, ctx->U);
        hipLaunchKernelGGL(k_stage_Y, dim3(gv), dim3(kThreads), 0, ctx->stream, ctx->gvec, nd, ctx->B, ctx->U, ctx->mat,
                           1.0 / adt, ctx->Y + (size_t)i * nd);
        SCK(hipGetLastError());
    }
    // U^{n+1} = U^n + dt M^{-1} sum_j b_j (F_j - Y_j)
    hipLaunchKernelGGL(k_combine_Y, dim3(gv), dim3(kThreads), 0, ctx->stream, nd, ctx->Y, s, P.b[0], P.b[1], P.b[2],
                       ctx->Z);
    hipLaunchKernelGGL(k_final, dim3(gv), dim3(kThreads), 0, ctx->stream, ctx->gvec, nd, ctx->U0, ctx->Z, ctx->mat, dt,
                       ctx->U);
    SCK(hipGetLastError());
    SST(add_sources(ctx, ctx->U, t, dt, s, P.b, P.c, 1));
    ctx->step_count += 1;
    ctx->hist_valid = std::min(ctx->hist_valid + 1, 2);
    return HHO_OK;
}

// external layout <-> group layout
void to_group(const hho::imp::Plan &P, const double *ext, std::vector<double> &grp) {
    grp.assign(P.n_dof, 0.0);
    for (int c = 0; c < P.n_cells; ++c) {
        const auto &g = P.groups[P.cell_group[c]];
        const int i = P.cell_index[c];
        for (int r = 0; r < g.nT; ++r) grp[g.vec_off + (int64_t)r * g.n + i] = ext[P.ext_off[c] + r];
    }
}

void from_group(const hho::imp::Plan &P, const std::vector<double> &grp, double *ext) {
    for (int c = 0; c < P.n_cells; ++c) {
        const auto &g = P.groups[P.cell_group[c]];
        const int i = P.cell_index[c];
        for (int r = 0; r < g.nT; ++r) ext[P.ext_off[c] + r] = grp[g.vec_off + (int64_t)r * g.n + i];
    }
}

}  // namespace

// Runs one C ABI call; a C++ exception (a failed host allocation, above all) becomes a status
// code and a message instead of crossing the ABI.
template <typename F>
hho_status guarded(std::string *err, F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        if (err) *err = "host memory allocation failed";
        return HHO_ERR_OOM;
    } catch (const std::exception &e) {
        if (err) *err = std::string("internal error: ") + e.what();
        return HHO_ERR_DEVICE;
    } catch (...) {
        if (err) *err = "internal error";
        return HHO_ERR_DEVICE;
    }
}

extern "C" {

const char *hho_sdirk_last_error(const hho_sdirk *ctx) { return ctx ? ctx->err.c_str() : g_sdirk_error.c_str(); }

hho_status hho_sdirk_setup(const hho_mesh *mesh, const hho_sdirk_params *prm, hho_sdirk **out) {
    return guarded(&g_sdirk_error, [&]() -> hho_status {
        g_sdirk_error.clear();
        if (!out) {
            g_sdirk_error = "null output pointer";
            return HHO_ERR_ARG;
        }
        *out = nullptr;
        if (prm && (!(prm->tol > 0.0) || !(prm->tol < 1.0) || prm->max_iter < 1)) {
            g_sdirk_error = "tol must lie in (0, 1) and max_iter be >= 1";
            return HHO_ERR_ARG;
        }
        hho_sdirk *ctx = new hho_sdirk();
        int code = 0;
        std::string msg = build_plan(mesh, prm, ctx->plan, &code);
        if (!msg.empty()) {
            g_sdirk_error = msg;
            delete ctx;
            return (hho_status)code;
        }
        if ((int)ctx->plan.groups.size() > kMaxGroups) {
            g_sdirk_error = "too many cell groups";
            delete ctx;
            return HHO_ERR_MESH;
        }
        ctx->device = prm->device;
        ctx->stream = (hipStream_t)prm->stream;
        ctx->tol = prm->tol;
        ctx->max_iter = prm->max_iter;
        auto fail = [&](hho_status st) {
            g_sdirk_error = ctx->err;
            hho_sdirk_destroy(ctx);
            return st;
        };
        if (hipSetDevice(ctx->device) != hipSuccess) {
            ctx->err = "hipSetDevice failed";
            return fail(HHO_ERR_DEVICE);
        }
        fill_groups(ctx);
        const auto &P = ctx->plan;
        hho_status st = HHO_OK;
    #define UP(ptr, vec)                                  \
        if ((st = upload(ctx, &ptr, vec)) != HHO_OK) return fail(st);
    #define AL(ptr, count)                                \
        if ((st = dev_alloc(ctx, &ptr, count)) != HHO_OK) return fail(st);
        UP(ctx->mats, P.mats);
        UP(ctx->wmat, P.wmat);
        UP(ctx->mat, P.mat);
        UP(ctx->slot_dof, P.slot_dof);
        UP(ctx->feed, P.feed);
        UP(ctx->S_ptr, P.S_ptr);
        {
            // shared column lists: a row reuses the previous row's list when it is the same
            std::vector<int> coff(std::max(P.n_fdof, 1), 0), cols;
            int last = -1;
            for (int d = 0; d < P.n_fdof; ++d) {
                const int a = P.S_ptr[d], len = P.S_ptr[d + 1] - a;
                bool same = last >= 0 && P.S_ptr[last + 1] - P.S_ptr[last] == len &&
                            std::equal(P.S_col.begin() + a, P.S_col.begin() + a + len, P.S_col.begin() + P.S_ptr[last]);
                if (same) {
                    coff[d] = coff[last];
                } else {
                    coff[d] = (int)cols.size();
                    cols.insert(cols.end(), P.S_col.begin() + a, P.S_col.begin() + a + len);
                }
                last = d;
            }
            ctx->n_shared_cols = (int64_t)cols.size();
            UP(ctx->S_coff, coff);
            UP(ctx->S_cols, cols);
        }
        {
            std::vector<double> scaled(P.S_val.size());
            for (int d = 0; d < P.n_fdof; ++d)
                for (int q = P.S_ptr[d]; q < P.S_ptr[d + 1]; ++q) scaled[q] = P.dscale[d] * P.S_val[q] * P.dscale[P.S_col[q]];
            UP(ctx->S_val, scaled);
        }
        UP(ctx->dsc, P.dscale);
        UP(ctx->P_ptr, P.P_ptr);
        {
            std::vector<int> start(P.n_fdof);
            std::vector<float> pv(P.P_val.size());
            for (int d = 0; d < P.n_fdof; ++d) start[d] = P.P_col[P.P_ptr[d]];
            for (size_t q = 0; q < pv.size(); ++q) pv[q] = (float)P.P_val[q];
            UP(ctx->P_start, start);
            UP(ctx->P_val, pv);
        }
        const size_t nd = (size_t)P.n_dof, nf = (size_t)P.n_fdof;
        AL(ctx->U, nd);
        AL(ctx->U0, nd);
        AL(ctx->B, nd);
        AL(ctx->gv, nd);
        AL(ctx->Z, nd);
        AL(ctx->Y, nd * P.stages);
        AL(ctx->cf, (size_t)P.n_slot);
        AL(ctx->E, nf * P.stages);
        AL(ctx->bF, nf);
    AL(ctx->xhist, nf * 2 * P.stages);
        AL(ctx->rhs, nf);
        AL(ctx->x, nf);
        AL(ctx->r, nf);
        AL(ctx->rh, nf);
        AL(ctx->pb[0], nf);
        AL(ctx->pb[1], nf);
        AL(ctx->v, nf);
        AL(ctx->s, nf);
        AL(ctx->t, nf);
        AL(ctx->ph, nf);
        AL(ctx->sh, nf);
        AL(ctx->part, 2 * (size_t)kDotBlocks);
        AL(ctx->partA, 2 * (size_t)grid_for(std::max<int>(P.n_fdof, 1)));
        AL(ctx->partB, 2 * (size_t)kSpmvBlocks);
        AL(ctx->partC, 2 * (size_t)kSpmvBlocks);
        AL(ctx->sc, kNumScalars);
    #undef UP
    #undef AL
        if (hipHostMalloc((void **)&ctx->h_sc, kNumScalars * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            ctx->err = "hipHostMalloc failed";
            return fail(HHO_ERR_OOM);
        }
        if (hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) ctx->cap = nullptr;
        const double tol2 = ctx->tol * ctx->tol;
        if (hipMemcpyAsync(ctx->sc + S_TOL2, &tol2, sizeof(double), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess) {
            ctx->err = "upload of the solver tolerance failed";
            return fail(HHO_ERR_DEVICE);
        }
        *out = ctx;
        return HHO_OK;
    });
}

void hho_sdirk_destroy(hho_sdirk *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->chunk) (void)hipGraphExecDestroy(ctx->chunk);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (void *p : ctx->allocs) (void)hipFree(p);
    if (ctx->h_sc) (void)hipHostFree(ctx->h_sc);
    delete ctx;
}

hho_status hho_sdirk_sizes(const hho_sdirk *ctx, int64_t *n_dof, int32_t *n_face_dof, int64_t *nnz) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n_dof) *n_dof = ctx->plan.n_dof;
        if (n_face_dof) *n_face_dof = ctx->plan.n_fdof;
        if (nnz) *nnz = (int64_t)ctx->plan.S_val.size();
        return HHO_OK;
    });
}

hho_status hho_sdirk_set_state(hho_sdirk *ctx, const double *U, int32_t on_device) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!U) {
            ctx->err = "null state";
            return HHO_ERR_ARG;
        }
        SCK(hipSetDevice(ctx->device));
        const auto &P = ctx->plan;
        std::vector<double> ext(P.n_dof), grp;
        if (on_device) {
            SCK(hipMemcpyAsync(ext.data(), U, P.n_dof * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            SCK(hipStreamSynchronize(ctx->stream));
        } else {
            std::memcpy(ext.data(), U, P.n_dof * sizeof(double));
        }
        to_group(P, ext.data(), grp);
        SCK(hipMemcpyAsync(ctx->U, grp.data(), P.n_dof * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        SCK(hipMemsetAsync(ctx->x, 0, std::max<size_t>(P.n_fdof, 1) * sizeof(double), ctx->stream));
        ctx->hist_valid = 0;
        ctx->step_count = 0;
        SCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_sdirk_set_ricker_ic(hho_sdirk *ctx, double xc, double yc, double theta, double lambda,
                                   int32_t field) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!(lambda > 0.0) || !std::isfinite(lambda) || !std::isfinite(xc) || !std::isfinite(yc) ||
            !std::isfinite(theta) || (field != 0 && field != 1)) {
            ctx->err = "set_ricker_ic: lambda <= 0, a non-finite value or field not 0 / 1";
            return HHO_ERR_ARG;
        }
        const auto &P = ctx->plan;
        const hho::RickerIC ic{xc, yc, theta, lambda, field};
        int px[16], py[16];
        for (int d = 0, m = 0; d <= P.kp; ++d)
            for (int a = d; a >= 0; --a, ++m) {
                px[m] = a;
                py[m] = d - a;
            }
        std::vector<double> U((size_t)P.n_dof, 0.0);
        for (int c = 0; c < P.n_cells; ++c) {
            const double h = P.hT[c], cx = P.centroid[2 * c], cy = P.centroid[2 * c + 1];
            const double *C = P.basisC.data() + (size_t)c * P.Np * P.Np;
            auto eval = [&](double x, double y, double *phi) {
                const double X = (x - cx) / h, Y = (y - cy) / h;
                double mu[16];
                for (int m = 0; m < P.Np; ++m) mu[m] = std::pow(X, px[m]) * std::pow(Y, py[m]);
                for (int a = 0; a < P.Np; ++a) {
                    double v = 0.0;
                    for (int m = 0; m <= a; ++m) v += C[a * P.Np + m] * mu[m];
                    phi[a] = v;
                }
            };
            // primal fields (p, v) of degree k', dual ones (m, s) of degree k: the first N functions
            const bool fluid = P.medium[c] == 0;
            const int b = P.cell_ptr[c];
            hho::project_ricker_cell(ic, P.xy.data(), P.cell_vtx.data() + b, P.cell_ptr[c + 1] - b, cx, cy, fluid, P.Np,
                                fluid ? P.N : P.Np, P.Np, eval, U.data() + P.ext_off[c]);
        }
        return hho_sdirk_set_state(ctx, U.data(), 0);
    });
}

hho_status hho_sdirk_get_state(hho_sdirk *ctx, double *U, int32_t on_device) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!U) {
            ctx->err = "null state";
            return HHO_ERR_ARG;
        }
        SCK(hipSetDevice(ctx->device));
        const auto &P = ctx->plan;
        std::vector<double> grp(P.n_dof), ext(P.n_dof);
        SCK(hipMemcpyAsync(grp.data(), ctx->U, P.n_dof * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        SCK(hipStreamSynchronize(ctx->stream));
        from_group(P, grp, ext.data());
        if (on_device) {
            SCK(hipMemcpyAsync(U, ext.data(), P.n_dof * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            SCK(hipStreamSynchronize(ctx->stream));
        } else {
            std::memcpy(U, ext.data(), P.n_dof * sizeof(double));
        }
        return HHO_OK;
    });
}

hho_status hho_sdirk_set_sources(hho_sdirk *ctx, int32_t n, const double *xy, const double *dir, const double *f0,
                                 const double *t0, const double *amp) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n < 0 || (n > 0 && (!xy || !dir || !f0 || !t0 || !amp))) {
            ctx->err = "invalid source arrays";
            return HHO_ERR_ARG;
        }
        SCK(hipSetDevice(ctx->device));
        const auto &P = ctx->plan;
        std::vector<SrcDev> v;
        std::vector<double> phi(P.Np);
        for (int q = 0; q < n; ++q) {
            const int c = hho::imp::locate(P, xy[2 * q], xy[2 * q + 1]);
            if (c < 0) {
                ctx->err = "source " + std::to_string(q) + " lies outside the mesh";
                return HHO_ERR_ARG;
            }
            hho::imp::eval_basis(P, c, xy[2 * q], xy[2 * q + 1], phi.data());
            const auto &g = P.groups[P.cell_group[c]];
            const int i = P.cell_index[c];
            const int ncomp = P.medium[c] == 0 ? 1 : 2;
            const double minv = P.medium[c] == 0 ? P.kappa[c] : 1.0 / P.rho[c];
            for (int cc = 0; cc < ncomp; ++cc)
                for (int a = 0; a < P.Np; ++a) {
                    const double coef = phi[a] * dir[2 * q + cc];
                    if (coef == 0.0) continue;
                    v.push_back({g.vec_off + (int64_t)(cc * P.Np + a) * g.n + i, coef, f0[q], t0[q], amp[q], minv});
                }
        }
        ctx->n_src = 0;
        release(ctx, ctx->src);
        ctx->src = nullptr;
        if (!v.empty()) {
            hho_status st = dev_alloc(ctx, &ctx->src, v.size());
            if (st != HHO_OK) return st;
            SCK(hipMemcpyAsync(ctx->src, v.data(), v.size() * sizeof(SrcDev), hipMemcpyHostToDevice, ctx->stream));
            SCK(hipStreamSynchronize(ctx->stream));
        }
        ctx->n_src = (int)v.size();
        return HHO_OK;
    });
}

hho_status hho_sdirk_step(hho_sdirk *ctx, double t0, int32_t n_steps) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n_steps < 0 || !std::isfinite(t0)) {
            ctx->err = "n_steps must be >= 0 and t0 finite";
            return HHO_ERR_ARG;
        }
        SCK(hipSetDevice(ctx->device));
        if (ctx->n_rec > 0) {
            const size_t need = (size_t)std::max(n_steps, 1) * ctx->n_rec * 2;
            if (need > ctx->trace_cap) {
                release(ctx, ctx->traces);
                ctx->traces = nullptr;
                ctx->trace_cap = 0;
                hho_status st = dev_alloc(ctx, &ctx->traces, need);
                if (st != HHO_OK) return st;
                ctx->trace_cap = need;
            }
        }
        ctx->last_steps = 0;
        for (int n = 0; n < n_steps; ++n) {
            hho_status st = one_step(ctx, t0 + n * ctx->plan.dt);
            if (st != HHO_OK) {
                // leave the state of the failing step's start
                hipLaunchKernelGGL(k_copy, dim3(grid_for(ctx->plan.n_dof)), dim3(kThreads), 0, ctx->stream,
                                   (long long)ctx->plan.n_dof, ctx->U0, ctx->U);
                (void)hipStreamSynchronize(ctx->stream);
                return st;
            }
            if (ctx->n_rec > 0) {
                hipLaunchKernelGGL(k_record, dim3((2 * ctx->n_rec + 63) / 64), dim3(64), 0, ctx->stream, 2 * ctx->n_rec,
                                   ctx->plan.Np, ctx->rec_idx, ctx->rec_coef, ctx->U,
                                   ctx->traces + (size_t)n * ctx->n_rec * 2);
                SCK(hipGetLastError());
            }
            ctx->last_steps = n + 1;
        }
        SCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_sdirk_receivers(hho_sdirk *ctx, int32_t n, const double *xy, const int32_t *field) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n < 0 || (n > 0 && (!xy || !field))) {
            ctx->err = "invalid receiver arrays";
            return HHO_ERR_ARG;
        }
        SCK(hipSetDevice(ctx->device));
        const auto &P = ctx->plan;
        const int Np = P.Np;
        std::vector<long long> idx((size_t)std::max(n, 1) * 2 * Np, -1);
        std::vector<double> coef((size_t)std::max(n, 1) * 2 * Np, 0.0), phi(Np);
        for (int q = 0; q < n; ++q) {
            const int c = hho::imp::locate(P, xy[2 * q], xy[2 * q + 1]);
            if (c < 0) {
                ctx->err = "receiver " + std::to_string(q) + " lies outside the mesh";
                return HHO_ERR_ARG;
            }
            if (field[q] != (int)P.medium[c] || (field[q] != 0 && field[q] != 1)) {
                ctx->err = "receiver " + std::to_string(q) + ": field 0 (p) needs a fluid cell, field 1 (v) a solid one";
                return HHO_ERR_ARG;
            }
            hho::imp::eval_basis(P, c, xy[2 * q], xy[2 * q + 1], phi.data());
            const auto &g = P.groups[P.cell_group[c]];
            const int i = P.cell_index[c];
            for (int comp = 0; comp < (field[q] == 0 ? 1 : 2); ++comp)
                for (int a = 0; a < Np; ++a) {
                    idx[((size_t)2 * q + comp) * Np + a] = g.vec_off + (int64_t)(comp * Np + a) * g.n + i;
                    coef[((size_t)2 * q + comp) * Np + a] = phi[a];
                }
        }
        release(ctx, ctx->rec_idx);
        release(ctx, ctx->rec_coef);
        ctx->rec_idx = nullptr;
        ctx->rec_coef = nullptr;
        ctx->n_rec = 0;
        ctx->last_steps = 0;
        if (n > 0) {
            hho_status st = dev_alloc(ctx, &ctx->rec_idx, idx.size());
            if (st != HHO_OK) return st;
            st = dev_alloc(ctx, &ctx->rec_coef, coef.size());
            if (st != HHO_OK) return st;
            SCK(hipMemcpyAsync(ctx->rec_idx, idx.data(), idx.size() * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
            SCK(hipMemcpyAsync(ctx->rec_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            SCK(hipStreamSynchronize(ctx->stream));
        }
        ctx->n_rec = n;
        return HHO_OK;
    });
}

hho_status hho_sdirk_get_traces(hho_sdirk *ctx, double *out) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx || !out) return HHO_ERR_ARG;
        if (ctx->n_rec == 0 || ctx->last_steps == 0) return HHO_OK;
        SCK(hipSetDevice(ctx->device));
        SCK(hipMemcpyAsync(out, ctx->traces, (size_t)ctx->last_steps * ctx->n_rec * 2 * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
        SCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_sdirk_energy(hho_sdirk *ctx, double *E) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx || !E) return HHO_ERR_ARG;
        SCK(hipSetDevice(ctx->device));
        const long long nd = ctx->plan.n_dof;
        const int nblk = std::min<int>(kDotBlocks, std::max<int>(1, (int)grid_for(nd)));
        hipLaunchKernelGGL(k_energy, dim3(nblk), dim3(kThreads), 0, ctx->stream, ctx->gvec, nd, ctx->U, ctx->mat, ctx->part);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, ctx->stream, nblk, ctx->part, ctx->sc, (int)F_TRUE,
                           ctx->partA, 0);
        SCK(hipGetLastError());
        SCK(hipMemcpyAsync(ctx->h_sc, ctx->sc, kNumScalars * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        SCK(hipStreamSynchronize(ctx->stream));
        *E = ctx->h_sc[S_TRR];
        return HHO_OK;
    });
}

hho_status hho_sdirk_footprint(const hho_sdirk *ctx, int64_t *sizes) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx || !sizes) return HHO_ERR_ARG;
        const auto &P = ctx->plan;
        sizes[0] = P.n_dof;
        sizes[1] = P.n_fdof;
        sizes[2] = (int64_t)P.S_val.size();
        sizes[3] = (int64_t)P.P_val.size();
        sizes[4] = (int64_t)(P.mats.size() + P.wmat.size());
        sizes[5] = P.n_slot;
        sizes[6] = ctx->n_shared_cols;
        return HHO_OK;
    });
}

hho_status hho_sdirk_stats(const hho_sdirk *ctx, int64_t *solves, int64_t *iterations, double *max_rel_residual) {
    return guarded(ctx ? &const_cast<hho_sdirk *>(ctx)->err : &g_sdirk_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (solves) *solves = ctx->solves;
        if (iterations) *iterations = ctx->iterations;
        if (max_rel_residual) *max_rel_residual = ctx->max_res;
        return HHO_OK;
    });
}

hho_status hho_sdirk_inspect_sizes(const hho_mesh *mesh, const hho_sdirk_params *prm, int64_t *sizes) {
    return guarded(&g_sdirk_error, [&]() -> hho_status {
        g_sdirk_error.clear();
        if (!sizes) return HHO_ERR_ARG;
        hho::imp::Plan P;
        int code = 0;
        std::string msg = build_plan(mesh, prm, P, &code);
        if (!msg.empty()) {
            g_sdirk_error = msg;
            return (hho_status)code;
        }
        sizes[0] = P.n_dof;
        sizes[1] = P.n_fdof;
        sizes[2] = (int64_t)P.S_val.size();
        sizes[3] = P.n_faces;
        sizes[4] = (int64_t)P.groups.size();
        return HHO_OK;
    });
}

hho_status hho_sdirk_inspect_face_matrix(const hho_mesh *mesh, const hho_sdirk_params *prm, int32_t *ptr, int32_t *col,
                                         double *val, int32_t *face) {
    return guarded(&g_sdirk_error, [&]() -> hho_status {
        g_sdirk_error.clear();
        hho::imp::Plan P;
        int code = 0;
        std::string msg = build_plan(mesh, prm, P, &code);
        if (!msg.empty()) {
            g_sdirk_error = msg;
            return (hho_status)code;
        }
        if (ptr) std::copy(P.S_ptr.begin(), P.S_ptr.end(), ptr);
        if (col) std::copy(P.S_col.begin(), P.S_col.end(), col);
        if (val) std::copy(P.S_val.begin(), P.S_val.end(), val);
        if (face) std::copy(P.fdof_face.begin(), P.fdof_face.end(), face);
        return HHO_OK;
    });
}

}  // extern "C"
