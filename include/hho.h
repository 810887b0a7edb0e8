/*
 * hho.h - C ABI of the MI355X HHO elasto-acoustic explicit Runge-Kutta engine.
 *
 * The engine advances the first-order hybrid high-order (HHO) semi-discretisation
 * of coupled acoustic / elastic waves (arXiv 2505.15771) with an explicit
 * Runge-Kutta method, eliminating the face unknowns at every stage so that every
 * solve is block-diagonal:
 *   model     Sec. 2.1, eq. continuous_acoustic (p, m), eq. continuous_elastic_eq (v, s),
 *             coupling eq. continuous_coupling imposed weakly (Sec. 2.2);
 *   space     Sec. 3.3, eq. HHO1 / HHO2 with the reconstructions eq. rec_a / rec_e, the
 *             least-squares stabilisation eq. stab (alpha = 0, equal order k' = k) scaled
 *             by the weights eta^f, eta^s of Sec. 5.1, and the face-local coupling block;
 *   time      Sec. 4.2, eq. ERK_compact / eq. ex_solve: K_F U_F = -K_FT U_T, then
 *             M U_T^{n,i} = M U_T^{n-1} + dt sum_j a_ij (F_T - K_T U_T - K_TF U_F)^{n,j},
 *             with the ERK(s) tableaux of eq. ERK (s = 2, 3, 4);
 *   energy    Sec. 5.1 (cell unknowns only).
 *
 * Conventions shared by every entry point
 *   - Every function returns hho_status; no C++ exception crosses the ABI.  After an
 *     error hho_last_error(ctx) returns a message (valid until the next call on ctx).
 *   - The caller owns every pointer it passes.  Input arrays are copied during the
 *     call and never retained.  "on_device" pointers are HIP device pointers (e.g.
 *     torch.Tensor.data_ptr() of a contiguous float64 cuda tensor); they are only
 *     accessed during the call, on params.stream.
 *   - A context is not thread-safe: use one context per host thread / stream.
 *   - State layout (external, "per cell contiguous", cells in input order, float64):
 *       fluid cell  [p (N) | m_x (N) | m_y (N)]
 *       solid cell  [v_x (N) | v_y (N) | s_1 (N) | s_2 (N) | s_3 (N)]
 *     N = (k+1)(k+2)/2 coefficients in the cell basis: the graded monomials
 *     ((x-x_T)/h_T)^a ((y-y_T)/h_T)^b (degree-major, decreasing power of x within a
 *     degree; x_T the centroid, h_T the largest vertex distance) orthonormalised in
 *     L2(T) by the inverse Cholesky factor of their Gram matrix (Sec. 3.3 uses
 *     barycentre-centred monomials; the orthonormal combination spans the same space).
 *     Stress coefficients refer to E_1 = e1 e1^T, E_2 = e2 e2^T, E_3 = (e1 e2^T + e2 e1^T)/sqrt(2),
 *     so s_3 = sqrt(2) * s_xy.
 */
#ifndef HHO_H
#define HHO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hho_ctx hho_ctx; /* opaque; owns every device buffer it allocates */

typedef enum {
    HHO_OK = 0,
    HHO_ERR_ARG = 1,      /* invalid argument (null pointer, out-of-range value)            */
    HHO_ERR_MESH = 2,     /* non-conforming / inconsistent mesh, clockwise or degenerate cell */
    HHO_ERR_SINGULAR = 3, /* a local Gram or face block is not invertible                 */
    HHO_ERR_DEVICE = 4,   /* HIP runtime or kernel launch failure                            */
    HHO_ERR_OOM = 5,      /* device allocation failed                                        */
    HHO_ERR_UNSTABLE = 6  /* recorded energy grew by more than 5 % or became non-finite
                             (energy criterion of Algorithm algo_CFL, Sec. 5.1)              */
} hho_status;

/* Polygonal mesh aligned with the fluid / solid partition (Sec. 3.1).
 *   xy[2*n_vertices]          vertex coordinates (x, y)
 *   cell_ptr[n_cells+1]       CSR offsets into cell_vtx
 *   cell_vtx[cell_ptr[n]]     counter-clockwise vertex ids of every cell; hanging nodes
 *                             are ordinary (collinear) vertices, so a face is one edge
 *   medium[n_cells]           0 = fluid (acoustic), 1 = solid (elastic)
 *   rho, a, b [n_cells]       piecewise-constant materials: fluid a = sound speed c
 *                             (kappa = rho c^2), b ignored; solid a = lambda, b = mu.
 * Every edge must be shared by at most two cells, traversed in opposite directions. */
typedef struct {
    int32_t n_vertices;
    const double *xy;
    int32_t n_cells;
    const int32_t *cell_ptr;
    const int32_t *cell_vtx;
    const uint8_t *medium;
    const double *rho;
    const double *a;
    const double *b;
} hho_mesh;

/* Discretisation and run parameters.
 *   k            polynomial degree, 1..3 (k >= 1 is needed in the solid, Sec. 3.2)
 *   rk_stages    ERK(s) of eq. ERK: 2 (midpoint), 3 (Kutta), 4 (classical)
 *   eta_f, eta_s stabilisation weights (0.8 and 1.5 in Sec. 5.1)
 *   stab_speed   speed c^s in tau^s = eta^s rho c^s (Sec. 3.3 leaves c^s undefined): 1 = S-wave
 *                speed, under which the stability-optimal solid weight is the paper's eta^s = 1.5
 *                (Sec. 5.1, Figure CFL_decoupled; the recommended setting), 0 = P-wave speed
 *   dtype        0 = float64 stepping; 1 = float32 stepping (float32 matvecs and
 *                accumulation, factors formed in float64 and rounded, float64 energy)
 *   n_shots      number of independent right-hand sides advanced together (1..256)
 *   record_energy 1 = record the float64 energy of every shot after every step
 *   device       HIP device ordinal
 *   stream       hipStream_t to run on (NULL = the null stream) */
typedef struct {
    int32_t k;
    int32_t rk_stages;
    double eta_f, eta_s;
    int32_t stab_speed;
    int32_t dtype;
    int32_t n_shots;
    int32_t record_energy;
    int32_t device;
    void *stream;
} hho_params;

/* Build the discretisation on the device: face extraction and tagging (Sec. 3.1),
 * local operators in float64 (Sec. 3.3), grouping of cells by (medium, shape class),
 * upload of SoA buffers.  State starts at zero.  Errors: ARG, MESH, SINGULAR, OOM, DEVICE. */
hho_status hho_setup(const hho_mesh *mesh, const hho_params *params, hho_ctx **out);

/* Three-dimensional mesh of tetrahedra, triangular prisms and hexahedra aligned with the fluid /
 * solid partition (the method of Sec. 2-3 with d = 3; Table tab::DOFS counts its unknowns):
 *   xyz[3*n_vertices]         vertex coordinates (x, y, z)
 *   cell_ptr[n_cells+1]       CSR offsets into cell_vtx: 4 ids (tetrahedron), 6 ids (triangular
 *                             prism: vertices 0-2 around the bottom triangle, 3-5 above vertices
 *                             0-2 in the same order) or 8 ids (hexahedron: vertices 0-3 around the
 *                             bottom face, 4-7 above vertices 0-3 in the same order); faces must
 *                             be planar and cells convex
 *   medium, rho, a, b         as in hho_mesh (solid: lambda, mu of 3D isotropic elasticity)
 * Every face (same vertex set) must be shared by at most two cells.  Local faces: tetrahedron
 * face j is opposite vertex j; prism faces (0 1 2), (3 4 5), (0 1 4 3), (1 2 5 4), (2 0 3 5);
 * hexahedron faces (0 1 2 3), (4 5 6 7), (0 1 5 4), (1 2 6 5), (2 3 7 6), (3 0 4 7). */
typedef struct {
    int32_t n_vertices;
    const double *xyz;
    int32_t n_cells;
    const int32_t *cell_ptr;
    const int32_t *cell_vtx;
    const uint8_t *medium;
    const double *rho;
    const double *a;
    const double *b;
} hho_mesh3d;

/* hho_setup for a three-dimensional mesh.  The returned context works with hho_sizes,
 * hho_set_state / hho_get_state, hho_set_sources, hho_receivers / hho_get_traces, hho_erk_step,
 * hho_energy, hho_energy_history, hho_energy_noalloc, hho_set_dt_scale, hho_cfl_search, the tuning
 * calls and hho_batch_*; separable loads, the Ricker initial field, the adjoint and hho_dt_cfl are
 * two-dimensional only (ARG).
 * State layout (external, per cell contiguous, float64), N = (k+1)(k+2)(k+3)/6:
 *   fluid cell  [p | m_x | m_y | m_z]
 *   solid cell  [v_x | v_y | v_z | s_1 | s_2 | s_3 | s_4 | s_5 | s_6]
 * in the orthonormalised graded monomials ((x-x_T)/h_T)^a ((y-y_T)/h_T)^b ((z-z_T)/h_T)^c (degree
 * major; within a degree decreasing a, then decreasing b; x_T the barycentre, h_T the largest
 * vertex distance); stress coefficients on E_1..E_3 = e_i e_i^T and E_4, E_5, E_6 =
 * (e_i e_j^T + e_j e_i^T)/sqrt(2) for ij = xy, xz, yz.  Face unknowns (eliminated at every stage)
 * live in a basis of P^k(F) fixed by the face: monomials in a frame whose origin is the face
 * centroid and whose first axis runs from the face's lowest-id vertex to its second-lowest-id
 * vertex, orthonormalised in L2(F).  Errors: ARG, MESH (vertex count, repeated vertex, non-planar
 * face, non-convex or degenerate cell, face shared by three cells), SINGULAR, OOM, DEVICE. */
hho_status hho_setup3d(const hho_mesh3d *mesh, const hho_params *params, hho_ctx **out);

/* Release every device buffer and the context (NULL is ignored). */
void hho_destroy(hho_ctx *ctx);

/* Message of the last error on ctx ("" if none); ctx NULL gives the last setup error. */
const char *hho_last_error(const hho_ctx *ctx);

/* Sizes: cell unknowns per shot (external layout), number of cells and faces. */
hho_status hho_sizes(const hho_ctx *ctx, int64_t *n_dof, int32_t *n_cells, int32_t *n_faces);

/* Copy one shot's state in / out (external layout above, float64, n_dof values).
 * on_device = 1: U is a device pointer.  Synchronous with respect to the host. */
hho_status hho_set_state(hho_ctx *ctx, int32_t shot, const double *U, int32_t on_device);
hho_status hho_get_state(hho_ctx *ctx, int32_t shot, double *U, int32_t on_device);

/* Initial state of eq. ricker_ic (Sec. 5.2) for one shot, replacing its state: the L2 projection
 * onto the cell bases of the Ricker-shaped field centred at (xc, yc) with
 * g = theta exp(-pi^2 r^2 / lambda^2), r the distance to the centre (the paper takes
 * lambda = c_P^f / f_c, f_c = 10 Hz, theta = 1 Hz):
 *   field 1  the printed initial velocity g (x - xc, y - yc): the m rows of fluid cells and the v
 *            rows of solid cells, every other unknown 0;
 *   field 0  the pressure pulse of the granite-water case (built, the paper says, from the same
 *            right-hand side; read as the scalar amplitude g): the p rows of fluid cells, every
 *            other unknown 0.
 * Computed on the host in float64: a fan of triangles from the cell centroid, each with a
 * 12 x 12 collapsed Gauss-Legendre rule; the coefficients are the moments (f, phi_a)_T of the
 * orthonormal basis.  Synchronous.  Errors: ARG (shot out of range, lambda <= 0, non-finite
 * values, field not 0 / 1). */
hho_status hho_set_ricker_ic(hho_ctx *ctx, int32_t shot, double xc, double yc, double theta, double lambda,
                             int32_t field);

/* Point sources of one shot (replaces earlier ones of that shot).  Source i is the load
 * vector of eq. rhs for the point force  amp_i R_i(t) d_i delta(x - x_i):  on the v rows of
 * the solid cell containing x_i (direction d_i = (dir[2i], dir[2i+1])), or on the p rows
 * of a fluid cell with weight dir[2i].  R_i is the Ricker wavelet
 * (1 - 2 a^2) exp(-a^2), a = pi f0_i (t - t0_i).  The containing cell is the lowest-id
 * cell whose closed polygon holds x_i.  On a three-dimensional context xy and dir hold three
 * values per source (x, y, z; d_x, d_y, d_z; a fluid source has weight d_x) and the cell is the
 * lowest-id cell that contains x_i.  Errors: ARG (point outside the mesh). */
hho_status hho_set_sources(hho_ctx *ctx, int32_t shot, int32_t n, const double *xy, const double *dir,
                           const double *f0, const double *t0, const double *amp);

/* Separable dense loads shared by every shot: F_T(t) += sum_m sin(omega_m t + phase_m) g_m,
 * g[m * n_dof + i] in the external layout (load vectors (f_m, phi_a)_T of eq. rhs).
 * At most 4 terms; n_terms = 0 removes them. */
hho_status hho_set_loads(hho_ctx *ctx, int32_t n_terms, const double *g, const double *omega,
                         const double *phase);

/* Register receivers (replaces earlier ones): field 0 records p (point must lie in the
 * fluid), field 1 records (v_x, v_y) (solid).  Values are point evaluations of the cell
 * polynomials (sensors of Sec. 5.2), recorded after every step of hho_erk_step.  On a
 * three-dimensional context xy holds (x, y, z) per receiver and field 1 records (v_x, v_y, v_z). */
hho_status hho_receivers(hho_ctx *ctx, int32_t n, const double *xy, const int32_t *field);

/* Advance every shot by n_steps steps of ERK(rk_stages) from time t0 with step dt.  Every step
 * runs from captured graphs: graphs of 32, 16, 8, 4, 2 and 1 steps are captured on first use
 * and kept while the configuration is unchanged; a call replays n_steps / 32 of the 32-step
 * graph and one graph per set binary digit of the remainder.  Enqueued on params.stream; returns
 * before completion unless record_energy = 1, in which case it synchronises and returns
 * HHO_ERR_UNSTABLE if the energy of a shot grew by more than 5 % over its initial value, or over
 * the previous step, or is not finite. */
hho_status hho_erk_step(hho_ctx *ctx, double t0, double dt, int32_t n_steps);

/* Size the per-call histories of ctx (receiver rows, energies when record_energy = 1) for calls
 * of up to n_steps steps.  A call longer than every earlier one grows them itself, and with them
 * the captured graphs are captured again inside that call; reserving first moves that work out of
 * a timed or latency-sensitive call.  Allocates device and pinned host memory (ERR_DEVICE when
 * that fails); changes no state; ARG for n_steps < 0. */
hho_status hho_reserve_steps(hho_ctx *ctx, int32_t n_steps);

/* Wait for all work enqueued by ctx. */
hho_status hho_synchronize(hho_ctx *ctx);

/* Receiver traces of the last hho_erk_step call for one shot: out[n_steps][n_rec][2]
 * (second slot 0 for p receivers), float64; out[n_steps][n_rec][3] on a three-dimensional
 * context (p, 0, 0 or v_x, v_y, v_z). */
hho_status hho_get_traces(hho_ctx *ctx, int32_t shot, double *out);

/* Energy of the current state of every shot, float64: E[n_shots]. */
hho_status hho_energy(hho_ctx *ctx, double *E);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the energies of hho_energy written to E[n_shots], a
 * device pointer (float64), enqueued on params.stream without synchronising.  The per-block
 * partial sums go to a static 2 MiB scratch array of the library on the context's device
 * (262144 doubles; resolved at hho_setup), so the call allocates nothing; ARG when the context
 * needs more than that (blocks of the launch shape x shots).  Every call on one device shares
 * that array: calls that overlap on one GPU (other host threads, other streams) race; calls in
 * one stream order are safe.  Results equal hho_energy's. */
hho_status hho_energy_noalloc(hho_ctx *ctx, double *E);

/* Energies recorded after each step of the last hho_erk_step call (record_energy = 1):
 * out[n_steps] for one shot. */
hho_status hho_energy_history(hho_ctx *ctx, int32_t shot, double *out);

/* Launch shape.  The stage kernel can run with workgroups of 64, 128 or 256 lanes (one lane per
 * cell and shot), and can store its outputs with the default or the non-temporal (streaming)
 * cache policy.  hho_autotune times one stage in every shape and policy on the current state,
 * keeps the fastest and returns its lane count; it changes no state.  hho_set_launch selects a
 * shape by lane count (ARG if none matches) and keeps the policy.  Results do not depend on the
 * shape or the policy except for the summation order of energies. */
hho_status hho_autotune(hho_ctx *ctx, int32_t *lanes);
hho_status hho_set_launch(hho_ctx *ctx, int32_t lanes);

/* Tuning flag of hho_set_tuning / hho_get_tuning: stage outputs with the non-temporal policy. */
#define HHO_TUNE_NT_STORES 1

/* Set the launch shape (by lane count, as hho_set_launch) and the tuning flags (ARG for a lane
 * count with no shape or for unknown flag bits; nothing changes then); get the current ones
 * (either output may be NULL). */
hho_status hho_set_tuning(hho_ctx *ctx, int32_t lanes, int32_t flags);
hho_status hho_get_tuning(const hho_ctx *ctx, int32_t *lanes, int32_t *flags);

/* Per-shot time steps: shot i advances with dt * scale[i] in every following hho_erk_step (and
 * batch step) of the context: stage times t0 + (n + c_i) dt scale[i], receivers and energies per
 * shot as before.  scale[S] (host, > 0 and finite, ARG otherwise); NULL resets every multiplier
 * to 1.  hho_adjoint_step refuses a context with multipliers set. */
hho_status hho_set_dt_scale(hho_ctx *ctx, const double *scale);

/* CFL stability limit by the energy criterion of Algorithm algo_CFL (Sec. 5.1), with the shots of
 * the context as simultaneous candidates.  Candidate step counts over [0, t_final]:
 * N_0 = n_start, N_{j+1} = N_j - max(1, floor(delta N_j)), each run with dt = t_final / N_j from
 * the states the shots hold on entry (set all shots to the same state for the paper's procedure),
 * sources and loads as set on ctx.  A round advances S candidates in one launch sequence: N_max
 * steps of the smallest dt, shot i with the multiplier N_max / N_i; candidate i is judged on the
 * energies after its first N_i steps.  It is unstable when the energy exceeds (1 + eps) times
 * the initial or the previous step's energy, or is not finite.  Rounds stop at the first
 * unstable candidate (in order) or after max_rounds.  Outputs: n_stable = the last stable N (0
 * if the first was unstable), n_unstable = the first unstable N (0 if none); tried[] and
 * growth[] (capacity cap, may be NULL when cap = 0) the candidates judged, in order, with their
 * largest relative energy increase (+inf when not finite); n_tried (may be NULL) their count.
 * CFL* brackets follow as c dt / h.  On return the entry states are restored, the multipliers
 * reset and the energy recording setting is as on entry. */
hho_status hho_cfl_search(hho_ctx *ctx, double t_final, int32_t n_start, double delta, double eps,
                          int32_t max_rounds, int32_t *n_stable, int32_t *n_unstable, int32_t *tried,
                          double *growth, int32_t cap, int32_t *n_tried);

/* Time step from the CFL condition (eq. CFL, Sec. 5.1): dt = factor * min over cells of
 * CFL*(s, k, shape) h_T / c_T, with c_T the largest wave speed of the cell (c, or c_P in the
 * solid), the shape from the cell's geometric corners (hanging nodes are not corners: 3 triangle,
 * 4 quadrilateral, 5 or more the hexagon column) and h_T the side of the generating square (sqrt
 * of the area, sqrt of twice the area for triangles).  CFL* is the paper's Table tab::ratio_geo
 * value, lowered to 0.9 times this discretisation's own stability limit for that shape where
 * that is smaller (with tau^s on c_S: triangles 0.90 and hexagons 0.66 of the paper's ERK(4) k = 1
 * value; with tau^s on c_P also squares), so factor 1 is a stable step for the weights
 * eta^f = 0.8, eta^s = 1.5 on the meshes tested (squares, triangles, hybrid, hanging nodes,
 * hexagons, moved vertices).  Other weights move the limit: measure it with hho_cfl_search. */
hho_status hho_dt_cfl(const hho_ctx *ctx, double factor, double *dt);

/* Receiver misfit and its gradient with respect to the cell materials, by the discrete adjoint
 * of the ERK time stepping of eq. ERK applied to the condensed semi-discretisation of eq. ex_solve
 * (the sensors of Sec. 5.2 as observations).  From the current state U^0 of every shot (time t0,
 * step dt, the sources and loads set on ctx), the call advances n_steps steps, recording the
 * receivers, and returns
 *   J = 1/2 dt sum_shots sum_{n=1..n_steps} sum_r |R_r U^n - d_obs[shot][n-1][r]|^2,
 *   grad[c][0..2] = dJ/d(rho, c, -) on fluid cells, dJ/d(rho, lambda, mu) on solid cells
 * (input cell order, float64, summed over shots; slot 2 is 0 on fluid cells).
 * d_obs[shot][n_steps][n_rec][2] (float64, host) in the layout of hho_get_traces; may be NULL
 * when no receivers are set (then J = 0 and grad = 0).  The reverse sweep keeps checkpoints of
 * the state every ckpt_every steps (0: about sqrt(n_steps)) and recomputes the stage data of one
 * segment while the adjoint stages of the following segment run (on a second stream the
 * context creates, default priority), so device memory grows as n_steps / ckpt_every states plus
 * 2 * ckpt_every * rk_stages stage records; the workspace is kept for later calls.
 * On return (synchronised) the state is U^{n_steps}, and hho_get_traces / hho_energy_history
 * report the forward run, as after hho_erk_step.  Only rk_stages 2 and 4 (subdiagonal
 * Runge-Kutta matrices) are supported: ARG otherwise; UNSTABLE as hho_erk_step. */
hho_status hho_adjoint_step(hho_ctx *ctx, double t0, double dt, int32_t n_steps, int32_t ckpt_every,
                            const double *d_obs, double *J, double *grad);

/* Batched stepping: several contexts (meshes of different sizes and degrees, each with its own
 * shots) advanced together.  The contexts' step chains are independent branches of captured
 * graphs of 32, 16, 8, 4, 2 and 1 steps, replayed as in hho_erk_step.
 * All contexts must live on one device; the batch launches on the first context's stream and
 * synchronises before returning.  t0[i], dt[i] per context.  The per-context results (state,
 * traces, energy history) are read with the per-context calls; HHO_ERR_UNSTABLE as hho_erk_step
 * for any context (message in hho_batch_last_error).  A batch does not own its contexts; destroy
 * it before them. */
typedef struct hho_batch hho_batch;
hho_status hho_batch_create(hho_ctx *const *ctxs, int32_t n, hho_batch **out);
void hho_batch_destroy(hho_batch *b);
const char *hho_batch_last_error(const hho_batch *b);
hho_status hho_batch_erk_step(hho_batch *b, const double *t0, const double *dt, int32_t n_steps);

/* Device time of the graph replays of the last hho_batch_erk_step, in milliseconds, measured
 * with HIP events recorded on the launch stream just before the first replay and after the last
 * (0 before the first step call). */
hho_status hho_batch_last_time(const hho_batch *b, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* HHO_H */
