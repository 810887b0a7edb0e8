/*
 * hho_inspect.h - host-only inspection of the execution plan that hho_setup builds
 * (no device is touched).  Meant for tests and tools that check the local operators,
 * the cell grouping and the face links on a machine without a GPU.
 *
 * Plan contents (float64, structure of arrays over "internal cells" ic, which are the
 * input cells regrouped by (medium, shape class) and padded per group):
 *   tables   per shape class: B_x, B_y, S (N x N each, row-major), then for every local
 *            face j (counter-clockwise order, face j runs from vertex j to vertex j+1):
 *            G_j (N x F), then the outward unit normals n_j (2 values per face).
 *            B_c = D_c - sum_j n_{j,c} E_j with D_c[a][b] = (d_c phi_b, phi_a)_T,
 *            E_j[a][b] = (phi_b, phi_a)_F, S = sum_j E_j, G_j[a][i] = (phi_a, psi_i)_F.
 *            phi: orthonormal cell basis (see hho.h); psi_i = sqrt((2i+1)/|F|) P_i(xi),
 *            xi in [-1, 1] running along the counter-clockwise direction of the cell.
 *            These are the blocks of eq. rec_a / rec_e / stab (Sec. 3.3) in that basis.
 *   groups   [n_groups][6]: medium, n_faces, table offset (0 for a pooled group, see
 *            hho_inspect_cell_tables), first ic, cells, first block
 *   link     [max_nf][n_ic]: (ic' << 4) | (interface << 3) | j' of the neighbour across
 *            local face j, -1 on the boundary
 *   c0       [max_nf][n_ic]: 1 / (tau_T + tau_T') on same-medium faces,
 *            1 / (tau_f + 1 / tau_s) on interface faces (tau = eta * tau_T of eq. stab)
 *   mat      [6][n_ic]: 1/rho, kappa or lambda + 2 mu, eta tau, lambda, 2 mu, 1/(eta tau)
 *   ic_of_cell [n_cells]
 * Errors as hho_setup (ARG, MESH, SINGULAR).
 */
#ifndef HHO_INSPECT_H
#define HHO_INSPECT_H

#include "hho.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hho_inspect hho_inspect;

hho_status hho_inspect_create(const hho_mesh *mesh, const hho_params *params, hho_inspect **out);
/* Plan of a three-dimensional mesh (see hho_setup3d).  Table layout per shape class: B_x, B_y,
 * B_z, S (N x N each), then G_j (N x F, F = (k+1)(k+2)/2) for every local face, then the outward
 * unit normals n_j (3 values per face); mat holds 1/rho, kappa or lambda + 2 mu, eta tau, lambda,
 * 2 mu, 1/(eta tau). */
hho_status hho_inspect3d_create(const hho_mesh3d *mesh, const hho_params *params, hho_inspect **out);
void hho_inspect_destroy(hho_inspect *p);

/* sizes[0..9] = N, F, n_ic, max_nf, n_groups, n_table_values, n_cells, n_faces, cpb, n_blocks */
hho_status hho_inspect_sizes(const hho_inspect *p, int64_t *sizes);

/* Copy the plan arrays out (caller-allocated, sizes from hho_inspect_sizes); any
 * pointer may be NULL to skip that array. */
hho_status hho_inspect_arrays(const hho_inspect *p, double *tables, int32_t *groups, int32_t *link, double *c0,
                              double *mat, int32_t *ic_of_cell);

/* Class table of every internal cell: ic_tab[n_ic] = offset of its class's table in `tables`
 * (0 for padding), and pooled[n_groups] = 1 for the groups that hold the cells of small shape
 * classes (fewer than 32 cells of that shape, on meshes with more than 64 shape classes): their
 * lanes read the table at their own offset, laid out with the group's face count (faces beyond a
 * cell's own count hold zeros) and packed without structural zeros: the entries of B_x, then of
 * B_y, with deg(b) < deg(r) (row-major; deg the total degree of the graded basis function), the
 * upper triangle r <= b of S (row-major), per face the entries G_j[a][i] with i <= deg(a)
 * (row-major), then the normals.  Either output may be NULL. */
hho_status hho_inspect_cell_tables(const hho_inspect *p, int32_t *ic_tab, int32_t *pooled);

/* Material derivatives used by the adjoint gradient (hho_adjoint_step), gm[8][n_ic], float64:
 *   fluid (parameters rho, c; kappa = rho c^2, tau = eta / (rho c)):
 *     d(1/kappa)/drho, d(1/kappa)/dc, dtau/drho, dtau/dc, 0, 0, 0, 0
 *   solid (parameters rho, lambda, mu; tau = eta rho c_S with stab_speed 1, or eta rho c_P with stab_speed 0):
 *     dtau/drho, dtau/dlambda, dtau/dmu, dA/dlambda (= dB/dlambda), dA/dmu, dB/dmu, dC/dmu, 0
 *   with [[A, B, 0], [B, A, 0], [0, 0, C]] the compliance in the symmetric-tensor basis
 *   (the stress mass matrix of eq. mass); padding cells hold zeros. */
hho_status hho_inspect_grad_coefs(const hho_inspect *p, double *gm);

/* Coefficients the stage kernel uses for ERK(stages) of eq. ERK (stages 2, 3, 4; ARG otherwise),
 * coefs[stages][9] = c, cY, ck, cb, qa, qb, cd, q_write, q_read.  The stage buffers hold increments
 * D_i = Y_{i+1} - U^n: D_i = cY D_{i-1} + ck dt k_i before the last stage (with q_write, also
 * Q = qa D_{i-1} + qb D_i); the last stage forms U^{n+1} = U^n + [q_read] Q + cd D_{s-2} + cb dt k_s.
 * c is the stage node (stage time t_n + c dt). */
hho_status hho_inspect_erk(int32_t stages, double *coefs);

/* The time step of hho_dt_cfl for ERK(stages) (2, 3 or 4) on the inspected plan. */
hho_status hho_inspect_dt_cfl(const hho_inspect *p, int32_t stages, double factor, double *dt);

#ifdef __cplusplus
}
#endif

#endif /* HHO_INSPECT_H */
