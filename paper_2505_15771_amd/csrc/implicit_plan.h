// Host-side plan of the SDIRK engine (float64): faces and tags (Sec. 3.1), the local HHO forms of
// eq. HHO1 / HHO2 with cell degree k' = k + 1 and the Lehrenfeld-Schoberl stabilisation (or
// k' = k and plain least squares), the per-cell static condensation of the cell unknowns
// (Sec. 4.1, the two solves following eq. cp_dirk) and the global face matrix it leaves.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hho {
namespace imp {

constexpr int kMaxEdges = 8;
constexpr int kNumMat = 8;  // material slots per cell, see ImpPlan::mat

// Cells of one medium and one number of face-slot unknowns.  Cell vectors are stored
// [row][cell] per group: element (r, i) of group g at vec_off + r * n + i.
struct Group {
    int medium = 0;
    int nT = 0;   // cell unknowns
    int nFT = 0;  // face unknowns the cell couples to (non-boundary faces only)
    int n = 0;    // cells
    int64_t vec_off = 0;   // into cell vectors (n_dof long)
    int64_t cf_off = 0;    // into per-slot vectors (sum nFT * n long)
    int64_t mat_off = 0;   // into the stacked matrices [Ainv; V] ((nT + nFT) x nT per cell)
    int64_t w_off = 0;     // into W (nT x nFT per cell)
    int64_t m_off = 0;     // into material scalars (kNumMat * n)
};

struct Plan {
    int k = 1, kp = 2, N = 3, Np = 6, nf = 2;
    int stages = 3;
    double dt = 0.0, ast = 0.0;
    double A[3][3] = {}, b[3] = {}, c[3] = {};
    double ell = 0.0;
    int n_cells = 0, n_faces = 0;
    int64_t n_dof = 0;      // cell unknowns (external layout size)
    int64_t n_slot = 0;     // sum over cells of nFT
    int n_fdof = 0;         // face unknowns
    std::vector<Group> groups;
    std::vector<int> cell_group, cell_index;  // per input cell
    std::vector<int64_t> ext_off;             // [n_cells + 1] external layout offsets
    // stacked [Ainv; V] per cell, W per cell, both [row][col][cell] within a group:
    //   Ainv = (M_T + a* dt K_T)^{-1},  V = a* dt K_FT Ainv,  W = a* dt Ainv K_TF
    std::vector<double> mats, wmat;
    std::vector<int32_t> slot_dof;  // [g][q][i] global face unknown of slot q (per-slot layout)
    // material scalars [slot][cell] per group:
    //   fluid: 1/kappa, rho, kappa, 1/rho
    //   solid: rho, Ca, Cb, Cc, 1/rho, Ia, Ib, Ic  (compliance [[Ca, Cb, 0], [Cb, Ca, 0], [0, 0, Cc]]
    //          in the E basis and its inverse [[Ia, Ib, 0], [Ib, Ia, 0], [0, 0, Ic]])
    std::vector<double> mat;
    // condensed face matrix S = a* dt (K_F - a* dt K_FT (M + a* dt K_T)^{-1} K_TF), CSR
    std::vector<int32_t> S_ptr, S_col;
    std::vector<double> S_val;
    // symmetric scaling of the face system: it is solved as (D S D) y = D b, x = D y, with
    // D = diag(S)^(-1/2), so that fluid and solid face rows (weights 1/(rho c) against rho c)
    // weigh alike in the residual norm
    std::vector<double> dscale;  // [n_fdof]
    // block-Jacobi preconditioner: inverse of the diagonal block of every face of D S D, CSR
    std::vector<int32_t> P_ptr, P_col;
    std::vector<double> P_val;
    // for every face unknown the (at most two) per-slot entries that feed it, -1 if none
    std::vector<int32_t> feed;  // [n_fdof][2]
    // per face unknown: its face's vertex ids (lower first) and its index in the face block
    std::vector<int32_t> fdof_face;  // [n_fdof][3]
    // geometry kept for point location / evaluation
    std::vector<double> xy, centroid, hT, basisC;  // basisC: [n_cells][Np][Np] (lower)
    std::vector<int32_t> cell_ptr, cell_vtx;
    std::vector<uint8_t> medium;
    std::vector<double> rho, kappa;
};

struct Options {
    int k = 1;
    int mixed = 1;
    int alpha = 1;
    double eta_f = 1.0, eta_s = 1.0;
    int stab_speed = 0;
    double ell = 0.0;
    int stages = 3;
    double dt = 0.0;
};

// SDIRK(s, s+1) tableau (s = 1, 2, 3); false for another s.
bool sdirk_tableau(int s, double A[3][3], double b[3], double c[3]);

// Returns "" on success, otherwise a message; *code receives the hho_status value.
std::string build(int nv, const double *xy, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                  const uint8_t *medium, const double *rho, const double *pa, const double *pb,
                  const Options &opt, Plan &P, int *code);

// Orthonormal degree-k' basis of cell c at (x, y) -> phi[Np].
void eval_basis(const Plan &P, int c, double x, double y, double *phi);

// Lowest-id cell whose closed polygon holds (x, y), -1 if none.
int locate(const Plan &P, double x, double y);

}  // namespace imp
}  // namespace hho
