// Device-side argument blocks of the HHO ERK kernels and their host launchers.
// Shared by kernels.hip (device code) and api.cpp (host runtime); plain structs only.
#pragma once

#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace hho {

struct GroupDev {
    int medium, nF, tab_off, ic_begin, ncells, blk_begin, pooled;
};

constexpr int kMaxN = 10;  // (k+1)(k+2)/2 for k = 3

// Point source entry (sorted by internal cell; `next` chains the entries of one cell).
struct SrcDev {
    int ic, shot, next, pad;
    double dirx, diry, f0, t0, amp;
    double dirz;  // three-dimensional contexts
    double phi[kMaxN];
};

// Receiver entry (sorted by internal cell; `next` chains the entries of one cell).
struct RecDev {
    int ic, field, r, next;
    double phi[kMaxN];
};

// Device-resident time keeping of one context: the stage kernels derive the stage time, the
// time step and the step index from it, so a captured multi-step graph replays unchanged.
// Two clocks alternate: the steps of even index read the first and the last stage of such a
// step writes the advanced clock into the second, and the other way round.
struct Clock {
    double t0, dt;  // start time and time step of the current hho_erk_step call
    int step;       // steps completed since t0
    int pad;
};

template <typename R>
struct StageArgs {
    int dim;        // 2: polygons (kernels.hip), 3: tetrahedra and hexahedra (kernels3d.hip)
    const R *Yin;   // stage input: U^n (first stage) or the increment D_{i-1}  [rows][LT]
    R *Yout;        // stage output: the increment D_i   [rows][LT]  (unused on the last stage)
    R *U;           // U^n (read), U^{n+1} (written on the last stage)
    R *acc;         // adjoint stage: running sum of L^T mu_j (unused by the forward stages)
    const R *Tin;   // face-trace contributions of Y_i     [trace rows][LT]
    R *Tout;        // face-trace contributions of the output state
    const int32_t *link;  // [max_nf][n_ic]
    const R *c0;          // [max_nf][n_ic]
    const R *mat;         // [kNumMat][n_ic]
    const R *tab;         // class tables
    const int32_t *ic_tab;  // [n_ic] table offset of every cell (read by the pooled-group kernels)
    int has_pooled;         // some groups are pooled: the stage and trace launches come in pairs
    int all_pooled;         // every group is pooled: only the pooled launch runs (and advances the clock)
    const GroupDev *groups;
    const int32_t *blk_group;
    int n_ic, S, cpb;
    long long LT;         // lanes = n_ic * S
    const Clock *clock;   // t_n = t0 + step * dt
    Clock *clock_next;    // last stage: written with step + 1 (the clock the next step reads)
    double c;             // stage node: the stage time is t_n + c dt
    // The stage buffers hold increments D_i = Y_{i+1} - U (Yin = D_{i-1}, Yout = D_i; Yin = U on
    // the first stage).  Before the last stage D_i = cY D_{i-1} + ck dt k_i (cU = 1 - cY unused),
    // and with q_write the partial sum Q = qa D_{i-1} + qb D_i is stored to Yq; last stage:
    // U^{n+1} = U + [q_read] Q + cd D_{s-2} + cb dt k_s with Q read from Yq.
    R cU, cY, ck, cb;
    R qa, qb, cd;
    int q_write, q_read;
    R *Yq;
    int first, last;
    int nt_stores;        // stage outputs with the non-temporal cache policy (large working sets)
    // per-shot multiplier of the clock's dt ([S], float64; null: every shot steps with dt)
    const double *dt_scale;
    // point sources
    const int32_t *src_first;  // [n_ic], -1 = none
    const SrcDev *src;
    // separable dense loads, [term][rows][n_ic], time factors sin(omega t + phase)
    int nterms;
    const R *gload;
    double omega[4], phase[4];
    // last-stage diagnostics
    double *e_part;            // energy partials [n_blocks][S] (null = off)
    // with e_slots > 1 the partials of step n go to e_part + (n % e_slots) * e_stride, so that one
    // reduction after several steps sums all of them (e_stride = n_blocks * S)
    long long e_stride;
    int e_slots;
    const double *emat;        // [4][n_ic]
    const int32_t *rec_first;  // [n_ic], -1 = none (null = off)
    const RecDev *rec;
    double *rec_out;           // [S][rec_steps][nrec][rec_w]; steps beyond rec_steps are not recorded
    int nrec, rec_steps;
    int rec_w;                 // values per receiver and step: 2 (two dimensions; p or v_x, v_y), 3
    // Every per-lane and per-cell array above except gload lives in one device arena that the
    // kernels address through a single buffer resource: byte offsets of each array in it.
    const void *arena;
    unsigned arena_bytes;
    unsigned o_yin, o_yout, o_u, o_acc, o_tin, o_tout, o_link, o_c0, o_mat, o_yq;
    // forward recompute for the adjoint: the stage input Y_i, its derivative k_i ([rows][LT])
    // and its face values ([trace rows][LT], own faces) are stored when non-null
    R *ystore, *kstore, *fstore;
    // adjoint stage (adjoint.hip): Yin = z_i = D M^{-1} mu_i, Yout = z_{i-1}, U = lambda,
    // acc = the running sum of L^T mu_j, stored forward data of the same stage (read)
    const R *yfwd, *kfwd, *ffwd;
    double *gacc;              // gradient accumulator [3][LT], float64
    const double *gm;          // per-cell parameter derivative coefficients [8][n_ic], float64
    R mu_b, mu_a, zs_b;        // dt b_{i-1}, dt a_{i,i-1}, dt b_s
    int inject;                // the step n whose misfit derivative enters lambda^n is inject + clock->step
                               // (the adjoint clock's step holds a per-segment offset); 0 = none
    const double *dobs;        // observed data [S][nobs][nrec][2]
    int nobs;
};

// Launchers (kernels.hip).  K = polynomial degree, R = double or float.  The stage, trace and
// energy launchers forward arguments with dim = 3 to the three-dimensional kernels.
template <int K, typename R>
hipError_t launch_stage(const StageArgs<R> &a, int n_blocks, hipStream_t st);

template <int K, typename R>
hipError_t launch_traces(const StageArgs<R> &a, int n_blocks, hipStream_t st);

template <int K, typename R>
hipError_t launch_energy(const StageArgs<R> &a, const R *state, int n_blocks, hipStream_t st);

// Sum energy partials over blocks: out[s] = sum_b part[b * S + s]; with a clock, the sums go
// to out[clock->step * S + s] (an energy history), skipped past `cap` steps.
hipError_t launch_energy_reduce(const double *part, int n_blocks, int S, double *out, const Clock *clock, int cap,
                                hipStream_t st);

// The energy history of the `count` steps that end with the clock's step: step m = clock->step - j
// (j < count) sums part[(m % slots) * stride + b * S + s] over the blocks b into out[m * S + s],
// skipped past `cap` steps.
hipError_t launch_energy_reduce_steps(const double *part, int n_blocks, int S, long long stride, int slots,
                                      double *out, const Clock *clock, int count, int cap, hipStream_t st);

// Three-dimensional stage, trace and energy launches (kernels3d_k*.hip; energy of a.Yin), for
// k <= kMaxK3: at k = 3 a solid tetrahedron carries 180 unknowns, beyond one lane's registers.
constexpr int kMaxK3 = 2;
template <int K, typename R>
hipError_t launch_stage3(const StageArgs<R> &a, int n_blocks, hipStream_t st);
template <int K, typename R>
hipError_t launch_traces3(const StageArgs<R> &a, int n_blocks, hipStream_t st);
template <int K, typename R>
hipError_t launch_energy3(const StageArgs<R> &a, int n_blocks, hipStream_t st);

// Forward stage with the recompute stores (ystore / kstore / fstore non-null).
template <int K, typename R>
hipError_t launch_stage_store(const StageArgs<R> &a, int n_blocks, hipStream_t st);

// Adjoint stage (adjoint.hip): from z_i and its incoming traces, Ybar_i = L^T mu_i, the gradient
// contributions mu_i^T (dL/dtheta) Y_i, and z_{i-1} (or lambda^n and the next z on the last stage).
template <int K, typename R>
hipError_t launch_adjoint_stage(const StageArgs<R> &a, int n_blocks, hipStream_t st);

// lambda += dt R^T (R U - d^n) at the receivers (U = a.yfwd, lambda = a.U, n = a.inject + clock step), then
// z = D M^{-1} (a.zs_b lambda) and its outgoing traces (z = a.Yout, traces = a.Tout).
template <int K, typename R>
hipError_t launch_adjoint_start(const StageArgs<R> &a, int n_blocks, hipStream_t st);

// grad[c][q] = sum_shots gacc[q][ic_of_cell[c] * S + shot]  (adjoint.hip)
hipError_t launch_grad_reduce(const double *gacc, long long LT, int S, const int32_t *ic_of_cell, int n_cells,
                              double *out, hipStream_t st);

// External (per-cell contiguous, float64) <-> internal ([rows][lanes], R) state copies
// for one shot.  map[e] = internal row-major index (row * LT + ic * S) of external dof e.
template <typename R>
hipError_t launch_scatter(const double *ext, const int64_t *map, long long n, int shot, R *state,
                          hipStream_t st);
template <typename R>
hipError_t launch_gather(const R *state, const int64_t *map, long long n, int shot, double *ext,
                         hipStream_t st);

}  // namespace hho
