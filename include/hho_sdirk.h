/*
 * hho_sdirk.h - C ABI of the MI355X SDIRK engine for the HHO elasto-acoustic semi-discretisation
 * (arXiv 2505.15771, implicit time stepping).
 *
 *   space  Sec. 3.3, eq. HHO1 / HHO2: cell unknowns of degree k' for the primal fields (p, v),
 *          degree k for the dual ones (m, s) and the faces.  mixed = 1 takes k' = k + 1 with the
 *          Lehrenfeld-Schoberl stabilisation (the L2(F) projection onto P^k(F) of the cell trace
 *          minus the face unknown), mixed = 0 takes k' = k with the plain least-squares one; the
 *          weights are tau^f = eta^f / (rho c_P), tau^s = eta^s rho c^s, times
 *          (h_T / l_Omega)^(-alpha) (eq. stab; alpha = 1 is the O(1/h) scaling the paper pairs
 *          with implicit schemes).
 *   time   Sec. 4.1, eq. SDIRK_compact with the SDIRK(s, s+1) tableaux of eq. SDIRK: s = 1 the
 *          implicit midpoint rule, s = 2 the order-3 tableau with a* = (3 + sqrt 3)/6 (the printed
 *          two-stage tableau, a* = 1/4, is of order 2 only), s = 3 the printed one (nu, xi).
 *          Every stage is solved by static condensation of the cell unknowns (the two solves
 *          following eq. cp_dirk): a cell-local elimination, a global solve for the face unknowns
 *          with the condensed matrix a* dt (K_F - a* dt K_FT (M + a* dt K_T)^{-1} K_TF), and the
 *          local recovery of the cell unknowns.  The condensed matrix is built once per context
 *          (the step dt is fixed at setup: the factor reuse of Sec. 4.1); the face system is
 *          solved by BiCGStab with a face-block Jacobi preconditioner to the relative residual
 *          tol (the paper pairs an ILU-preconditioned BiCG with a direct LU).
 *
 * Conventions as in hho.h: every function returns hho_status, the caller owns every pointer,
 * inputs are copied, a context is not thread-safe.  Float64 throughout.
 *
 * State layout (external, per cell contiguous, cells in input order):
 *   fluid cell  [p (N') | m_x (N) | m_y (N)]
 *   solid cell  [v_x (N') | v_y (N') | s_1 (N) | s_2 (N) | s_3 (N)]
 * N' = (k'+1)(k'+2)/2, N = (k+1)(k+2)/2; coefficients in the orthonormal cell basis of hho.h at
 * degree k' (the dual blocks use its first N functions, which are the degree-k basis).
 */
#ifndef HHO_SDIRK_H
#define HHO_SDIRK_H

#include "hho.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hho_sdirk hho_sdirk; /* opaque; owns its device buffers */

/* Parameters.
 *   k           face degree (and dual cell degree), 1..3
 *   mixed       1: primal cell degree k + 1, Lehrenfeld-Schoberl; 0: degree k, least squares
 *   alpha       0 or 1: stabilisation weights times (h_T / l_Omega)^(-alpha)
 *   eta_f/_s    stabilisation weights (> 0)
 *   stab_speed  c^s in tau^s: 1 = S-wave speed (the reading hho.h recommends), 0 = P-wave speed
 *   ell         l_Omega (> 0), or 0 for the diameter of the mesh (largest distance between two
 *               boundary vertices)
 *   stages      s of SDIRK(s, s+1): 1, 2 or 3
 *   dt          time step (> 0)
 *   tol         relative residual ||b - S x|| <= tol ||b|| of every face solve (> 0, < 1)
 *   max_iter    BiCGStab iterations per face solve before HHO_ERR_UNSTABLE
 *   device, stream as in hho.h */
typedef struct {
    int32_t k;
    int32_t mixed;
    int32_t alpha;
    double eta_f, eta_s;
    int32_t stab_speed;
    double ell;
    int32_t stages;
    double dt;
    double tol;
    int32_t max_iter;
    int32_t device;
    void *stream;
} hho_sdirk_params;

/* Build the local forms, the per-cell condensation and the face matrix in float64 on the host
 * (Sec. 3.3, Sec. 4.1), upload them.  State starts at zero.
 * Errors: ARG, MESH, SINGULAR (a Gram, stage or face block not invertible), OOM, DEVICE. */
hho_status hho_sdirk_setup(const hho_mesh *mesh, const hho_sdirk_params *params, hho_sdirk **out);
void hho_sdirk_destroy(hho_sdirk *ctx);
/* Message of the last error ("" if none); ctx NULL gives the last setup error. */
const char *hho_sdirk_last_error(const hho_sdirk *ctx);

/* Sizes: cell unknowns (external layout), face unknowns, nonzeros of the face matrix. */
hho_status hho_sdirk_sizes(const hho_sdirk *ctx, int64_t *n_dof, int32_t *n_face_dof, int64_t *nnz);

/* State in / out in the external layout (n_dof float64); on_device = 1 for a device pointer.
 * Synchronous with respect to the host. */
hho_status hho_sdirk_set_state(hho_sdirk *ctx, const double *U, int32_t on_device);

/* The initial state of eq. ricker_ic (Sec. 5.2), as hho_set_ricker_ic of hho.h: field 1 the
 * velocity g (x - xc, y - yc) on the m rows (degree k) of fluid cells and the v rows (degree k')
 * of solid cells, field 0 the pressure pulse g on the p rows (degree k') of fluid cells; L2
 * projections on the host in float64.  Errors: ARG. */
hho_status hho_sdirk_set_ricker_ic(hho_sdirk *ctx, double xc, double yc, double theta, double lambda,
                                   int32_t field);
hho_status hho_sdirk_get_state(hho_sdirk *ctx, double *U, int32_t on_device);

/* Point sources, as hho_set_sources of hho.h (Ricker time factor, v rows of a solid cell or
 * the p rows of a fluid cell with weight dir[2i]), evaluated with the degree-k' basis. */
hho_status hho_sdirk_set_sources(hho_sdirk *ctx, int32_t n, const double *xy, const double *dir,
                                 const double *f0, const double *t0, const double *amp);

/* Advance n_steps steps of SDIRK(stages, stages+1) from time t0 with the setup's dt.  Returns
 * when the steps are done (every face solve checks its residual on the host).
 * HHO_ERR_UNSTABLE: a face solve did not reach tol within max_iter iterations (or broke down
 * twice); the state is then that of the failing stage's step start. */
hho_status hho_sdirk_step(hho_sdirk *ctx, double t0, int32_t n_steps);

/* Receivers (replace earlier ones; n = 0 removes them): field 0 records p (the point must lie in
 * a fluid cell), field 1 records (v_x, v_y) (solid cell); point values of the degree-k' cell
 * polynomials (sensors of Sec. 5.2) recorded after every step of hho_sdirk_step.  The containing
 * cell is the lowest-id cell whose closed polygon holds the point.  Errors: ARG. */
hho_status hho_sdirk_receivers(hho_sdirk *ctx, int32_t n, const double *xy, const int32_t *field);

/* Traces of the last hho_sdirk_step call: out[n_steps][n_rec][2] (second slot 0 for p), float64. */
hho_status hho_sdirk_get_traces(hho_sdirk *ctx, double *out);

/* Energy of the current state (Sec. 5.1, cell unknowns only), float64. */
hho_status hho_sdirk_energy(hho_sdirk *ctx, double *E);

/* Footprint of the plan on the device: sizes[0..6] = cell unknowns, face unknowns, nonzeros of the
 * face matrix (float64 values), nonzeros of the face-block preconditioner (float32 values),
 * float64 values of the per-cell matrices ([A_T^{-1}; V_T] and W_T over all cells), face-slot
 * unknowns (sum over cells of the face unknowns each cell couples to), column indices stored for
 * the face matrix (rows with the same column list share one). */
hho_status hho_sdirk_footprint(const hho_sdirk *ctx, int64_t *sizes);

/* Counters since setup: face solves, BiCGStab iterations, largest final relative residual. */
hho_status hho_sdirk_stats(const hho_sdirk *ctx, int64_t *solves, int64_t *iterations, double *max_rel_residual);

/* Host-only inspection (no device touched): the plan hho_sdirk_setup would build.
 * sizes[0..4] = n_dof, n_face_dof, nnz of the face matrix, n_faces, number of cell groups.
 * hho_sdirk_inspect_face_matrix copies the face matrix in CSR (ptr[n_face_dof + 1], col[nnz],
 * val[nnz]) and, per face unknown, its face's two vertex ids (lower first) and its index inside
 * that face's block (face[3 * n_face_dof]); any output pointer may be NULL. */
hho_status hho_sdirk_inspect_sizes(const hho_mesh *mesh, const hho_sdirk_params *params, int64_t *sizes);
hho_status hho_sdirk_inspect_face_matrix(const hho_mesh *mesh, const hho_sdirk_params *params, int32_t *ptr,
                                         int32_t *col, double *val, int32_t *face);

#ifdef __cplusplus
}
#endif

#endif /* HHO_SDIRK_H */
