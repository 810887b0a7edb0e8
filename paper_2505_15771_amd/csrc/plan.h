// Host-side execution plan of the HHO elasto-acoustic ERK engine: the mesh turned
// into shape classes, cell groups and structure-of-arrays metadata, all in float64.
// Built once by hho_setup (Sec. 3.1 mesh and faces, Sec. 3.3 local operators).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hho {

constexpr int kMaxFaces = 8;     // faces per cell (hanging nodes raise the count)
constexpr int kBlock = 256;      // largest workgroup (lanes)
constexpr int kLanesTarget = 64; // preferred lanes per workgroup: one wavefront
constexpr int kPoolCells = 32;       // shape classes with fewer cells share pooled groups ...
constexpr int kPoolMinClasses = 64;  // ... when the mesh has more classes than this

enum Medium : int { kFluid = 0, kSolid = 1 };

// Per-class table layout (float64 on the host, rounded for float32 runs):
//   Bx, By, S   N x N each, row-major  (B_c = D_c - sum_j n_{j,c} E_j, S = sum_j E_j)
//   G_j         N x F for each local face j
//   n_j         2 values for each local face j (outward unit normal)
struct ClassInfo {
    int nF = 0;
    int offset = 0;  // into Plan::tables
    int rep_cell = 0;
    int ncells = 0;
    bool pooled = false;  // fewer than kPoolCells cells: its cells go to a pooled group
    int nF_layout = 0;    // faces in the table layout (pooled classes: the pooled group's count)
};

// A pooled group holds the cells of small shape classes of one medium and face-count bucket
// (at most 4 faces, or more): its lanes read their class tables at per-cell offsets (ic_tab).
struct Group {
    int medium = 0;
    int cls = 0;          // -1 for a pooled group
    bool pooled = false;
    int nF = 0;
    int tab_off = 0;
    int ic_begin = 0;  // first internal cell of the group
    int ncells = 0;    // real cells
    int blk_begin = 0;
    int nblk = 0;
};

// Material slots of Plan::mat (per internal cell, structure of arrays).
enum MatSlot : int {
    kInvRho = 0,  // 1 / rho
    kStiff = 1,   // fluid: kappa ; solid: lambda + 2 mu
    kTau = 2,     // eta * tau_T
    kLam = 3,     // solid: lambda
    kTwoMu = 4,   // solid: 2 mu
    kInvTau = 5,  // 1 / (eta * tau_T)
    kNumMat = 6
};

// Energy weights per internal cell (float64): fluid (rho, 1/kappa, 0, 0),
// solid (rho, a, b, c) with the compliance in the E basis [[a, b, 0], [b, a, 0], [0, 0, c]].
constexpr int kNumEnergyMat = 4;
constexpr int kNumGradCoef = 8;

struct Plan {
    // dim = 2: polygons, F = k + 1 face modes, cell rows 3N (fluid) / 5N (solid), 2 trace components
    // dim = 3: tetrahedra and hexahedra, F = (k+1)(k+2)/2, cell rows 4N / 9N, 3 trace components
    int dim = 2, tcomp = 2, rows_f = 3, rows_s = 5;
    int k = 1, N = 3, F = 2, S = 1;
    int stab_speed = 1;             // c^s in tau^s: 0 P-wave, 1 S-wave speed
    double eta_f = 0.8, eta_s = 1.5;
    int n_cells = 0, n_faces = 0, n_vertices = 0;
    int max_nf = 0;
    int cpb = 256;           // cells per block of the default launch shape
    int n_ic = 0;            // padded internal cells
    int64_t n_ext = 0;       // external dofs per shot
    std::vector<int64_t> ext_off;   // [n_cells+1]
    std::vector<int> ic_of_cell;    // [n_cells]
    std::vector<int> cell_of_ic;    // [n_ic], -1 = padding
    std::vector<uint8_t> medium;    // input media
    std::vector<ClassInfo> classes;
    std::vector<double> tables;
    std::vector<Group> groups;
    std::vector<int> blk_group;  // default launch shape
    // Launch shapes the autotuner can choose from: workgroups of `lanes` lanes, `cpb` cells
    // each; groups are padded to a multiple of the largest cpb so every shape fits.
    struct Launch {
        int lanes = 64, cpb = 64;
        std::vector<int> blk_group;  // group of every block
        std::vector<int> blk_begin;  // first block of every group
    };
    std::vector<Launch> launches;
    // per (j, ic): link = (ic' << 4) | (interface << 3) | j', -1 = boundary face
    std::vector<int32_t> link;  // [max_nf][n_ic]
    std::vector<double> c0;     // [max_nf][n_ic] face-solve coefficient
    std::vector<double> mat;    // [kNumMat][n_ic]
    std::vector<double> emat;   // [kNumEnergyMat][n_ic]
    // Material derivatives for the adjoint gradient, [kNumGradCoef][n_ic] (float64):
    //   fluid (rho, c):        d(1/kappa)/drho, d(1/kappa)/dc, dtau/drho, dtau/dc
    //   solid (rho, lam, mu):  dtau/drho, dtau/dlam, dtau/dmu, dA/dlam (= dB/dlam), dA/dmu, dB/dmu, dC/dmu
    // with tau the stabilisation weight and [[A, B, 0], [B, A, 0], [0, 0, C]] the compliance.
    std::vector<double> gm;
    // geometry needed for point location / evaluation
    std::vector<double> xy;   // dim 2: vertex coordinates [2 * n_vertices]
    std::vector<double> xyz;  // dim 3: [3 * n_vertices]
    std::vector<int32_t> cell_ptr, cell_vtx;
    std::vector<double> centroid;  // [dim * n_cells]
    std::vector<double> hT;        // [n_cells]
    std::vector<double> area;      // [n_cells] (dim 3: volume)
    std::vector<double> basisC;    // [n_classes][N][N] orthonormal basis coefficients (lower)
    std::vector<int> cell_class;   // [n_cells]
    std::vector<int32_t> ic_tab;   // [n_ic] class table offset of every internal cell (0: padding)
    bool has_pooled = false;
};

// Returns "" on success, otherwise an error message; *code receives the status code.
std::string build_plan(int nv, const double *xy, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                       const uint8_t *medium, const double *rho, const double *a, const double *b, int k,
                       double eta_f, double eta_s, int stab_speed, int n_shots, Plan &plan, int *code);

// Orthonormal cell basis of input cell c at (x, y) -> phi[N].
void eval_basis(const Plan &plan, int c, double x, double y, double *phi);

// Lowest-id cell whose closed polygon contains (x, y), -1 if none.
int locate_cell(const Plan &plan, double x, double y);

int trace_rows(const Plan &plan);  // rows of a trace buffer: max_nf * tcomp * F

// Three-dimensional plan: cells are tetrahedra (4 vertex ids) or hexahedra with planar faces
// (8 vertex ids, 0-3 around the bottom face, 4-7 above them); same status convention.
std::string build_plan3d(int nv, const double *xyz, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                         const uint8_t *medium, const double *rho, const double *a, const double *b, int k,
                         double eta_f, double eta_s, int stab_speed, int n_shots, Plan &plan, int *code);
// Orthonormal cell basis of input cell c at (x, y, z) -> phi[N] (three-dimensional plan).
void eval_basis3(const Plan &plan, int c, double x, double y, double z, double *phi);
// Lowest-id cell containing (x, y, z), -1 if none (three-dimensional plan).
int locate_cell3(const Plan &plan, double x, double y, double z);

}  // namespace hho
