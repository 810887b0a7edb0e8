// Host-side plan of the SDIRK engine (float64).
//
// Per cell: the orthonormal cell basis of degree k' (graded scaled monomials orthonormalised by
// the inverse Cholesky factor of their Gram matrix; the dual unknowns use its first dim P^k
// functions), the local forms of eq. HHO1 / HHO2 (Sec. 3.3: reconstructions eq. rec_a / rec_e,
// stabilisation eq. stab with the L2(F) projection onto P^k(F) of Lehrenfeld-Schoberl when
// k' = k + 1, weights tau (h_T / l_Omega)^(-alpha)), and the static condensation of its cell
// unknowns for the SDIRK stage matrix of eq. cp_dirk:
//   A_T = M_T + a* dt K_T,  V_T = a* dt K_FT A_T^{-1},  W_T = a* dt A_T^{-1} K_TF,
//   S_T = a* dt K_FF,T - a* dt K_FT W_T   (the cell's share of the global face matrix).
// The interface coupling blocks (face-local, Sec. 3.3) are added to the face matrix directly.
//
// Integrals are exact: cell moments of the scaled monomials by Green's formula with 5-point
// Gauss-Legendre on every edge (degree <= 2k' + 1 <= 9), face integrals by the same rule
// (degree <= k' + k <= 7).
#include "implicit_plan.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>
#include <map>

namespace hho {
namespace imp {

namespace {

struct GaussLegendre5 {
    double x[5], w[5];
    GaussLegendre5() {
        const double r = std::sqrt(10.0 / 7.0);
        const double p = std::sqrt(5.0 - 2.0 * r) / 3.0, q = std::sqrt(5.0 + 2.0 * r) / 3.0;
        const double wp = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0, wq = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
        const double xs[5] = {-q, -p, 0.0, p, q}, ws[5] = {wq, wp, 128.0 / 225.0, wp, wq};
        for (int i = 0; i < 5; ++i) { x[i] = xs[i]; w[i] = ws[i]; }
    }
};
const GaussLegendre5 kG5;

void graded_exponents(int k, std::vector<int> &ex, std::vector<int> &ey) {
    ex.clear();
    ey.clear();
    for (int d = 0; d <= k; ++d)
        for (int a = d; a >= 0; --a) { ex.push_back(a); ey.push_back(d - a); }
}

double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

double legendre_p(int n, double x) {
    if (n == 0) return 1.0;
    double a = 1.0, b = x;
    for (int m = 1; m < n; ++m) {
        const double c = ((2.0 * m + 1.0) * x * b - m * a) / (m + 1.0);
        a = b;
        b = c;
    }
    return b;
}

// lower Cholesky factor of an SPD matrix (row-major); false if not positive definite
bool chol(int n, const std::vector<double> &A, std::vector<double> &L) {
    L.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int m = 0; m < j; ++m) d -= L[j * n + m] * L[j * n + m];
        if (!(d > 0.0)) return false;
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int m = 0; m < j; ++m) s -= L[i * n + m] * L[j * n + m];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    return true;
}

void lower_inverse(int n, const std::vector<double> &L, std::vector<double> &Li) {
    Li.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            double s = i == j ? 1.0 : 0.0;
            for (int m = j; m < i; ++m) s -= L[i * n + m] * Li[m * n + j];
            Li[i * n + j] = s / L[i * n + i];
        }
}

// Gauss-Jordan inverse with partial pivoting; false if a pivot vanishes
bool gj_inverse(int n, std::vector<double> A, std::vector<double> &X) {
    X.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
        if (!(std::fabs(A[piv * n + col]) > 1e-300 + 1e-15 * scale)) return false;
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[piv * n + j], A[col * n + j]);
                std::swap(X[piv * n + j], X[col * n + j]);
            }
        const double inv = 1.0 / A[col * n + col];
        for (int j = 0; j < n; ++j) { A[col * n + j] *= inv; X[col * n + j] *= inv; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[col * n + j]; X[r * n + j] -= f * X[col * n + j]; }
        }
    }
    return true;
}

// Inverse after symmetric diagonal scaling D A D, D = diag(A_ii)^(-1/2) (every matrix inverted
// here has a positive diagonal: a mass matrix plus a term whose symmetric part is positive
// semi-definite), so that materials of very different magnitudes (1/kappa next to rho) do not
// trip the pivot test; A^{-1} = D (D A D)^{-1} D.
bool scaled_inverse(int n, const std::vector<double> &A, std::vector<double> &X) {
    std::vector<double> d(n), B((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        const double a = A[(size_t)i * n + i];
        if (!(a > 0.0) || !std::isfinite(a)) return false;
        d[i] = 1.0 / std::sqrt(a);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) B[(size_t)i * n + j] = d[i] * A[(size_t)i * n + j] * d[j];
    if (!gj_inverse(n, B, X)) return false;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) X[(size_t)i * n + j] *= d[i] * d[j];
    return true;
}

// (E_alpha)_{cd} of the symmetric tensor basis
double tensor_basis(int al, int c, int d) {
    if (al == 0) return (c == 0 && d == 0) ? 1.0 : 0.0;
    if (al == 1) return (c == 1 && d == 1) ? 1.0 : 0.0;
    return c != d ? 1.0 / std::sqrt(2.0) : 0.0;
}

}  // namespace

bool sdirk_tableau(int s, double A[3][3], double b[3], double c[3]) {
    for (int i = 0; i < 3; ++i) {
        b[i] = c[i] = 0.0;
        for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
    }
    if (s == 1) {  // implicit midpoint rule
        A[0][0] = 0.5; b[0] = 1.0; c[0] = 0.5;
    } else if (s == 2) {  // a* = (3 + sqrt 3) / 6: order 3
        const double g = (3.0 + std::sqrt(3.0)) / 6.0;
        A[0][0] = g; A[1][0] = 1.0 - 2.0 * g; A[1][1] = g;
        b[0] = b[1] = 0.5; c[0] = g; c[1] = 1.0 - g;
    } else if (s == 3) {  // eq. SDIRK with nu and xi
        const double pi = 3.14159265358979323846;
        const double nu = std::cos(pi / 18.0) / std::sqrt(3.0) + 0.5;
        const double xi = 1.0 / (6.0 * (2.0 * nu - 1.0) * (2.0 * nu - 1.0));
        A[0][0] = nu;
        A[1][0] = 0.5 - nu; A[1][1] = nu;
        A[2][0] = 2.0 * nu; A[2][1] = 1.0 - 4.0 * nu; A[2][2] = nu;
        b[0] = xi; b[1] = 1.0 - 2.0 * xi; b[2] = xi;
        c[0] = nu; c[1] = 0.5; c[2] = 1.0 - nu;
    } else {
        return false;
    }
    return true;
}

void eval_basis(const Plan &P, int c, double x, double y, double *phi) {
    std::vector<int> ex, ey;
    graded_exponents(P.kp, ex, ey);
    const double h = P.hT[c], X = (x - P.centroid[2 * c]) / h, Y = (y - P.centroid[2 * c + 1]) / h;
    const double *C = P.basisC.data() + (size_t)c * P.Np * P.Np;
    std::vector<double> mu(P.Np);
    for (int m = 0; m < P.Np; ++m) mu[m] = ipow(X, ex[m]) * ipow(Y, ey[m]);
    for (int a = 0; a < P.Np; ++a) {
        double s = 0.0;
        for (int m = 0; m <= a; ++m) s += C[a * P.Np + m] * mu[m];
        phi[a] = s;
    }
}

int locate(const Plan &P, double x, double y) {
    for (int c = 0; c < P.n_cells; ++c) {
        const int s = P.cell_ptr[c], n = P.cell_ptr[c + 1] - s;
        const double tol = 1e-12 * P.hT[c];
        bool in = true;
        for (int j = 0; j < n && in; ++j) {
            const int i0 = P.cell_vtx[s + j], i1 = P.cell_vtx[s + (j + 1) % n];
            const double ex = P.xy[2 * i1] - P.xy[2 * i0], ey = P.xy[2 * i1 + 1] - P.xy[2 * i0 + 1];
            if (ex * (y - P.xy[2 * i0 + 1]) - ey * (x - P.xy[2 * i0]) < -tol * std::hypot(ex, ey)) in = false;
        }
        if (in) return c;
    }
    return -1;
}

std::string build(int nv, const double *xy, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                  const uint8_t *medium, const double *rho, const double *pa, const double *pb,
                  const Options &o, Plan &P, int *code) {
    *code = 1;  // HHO_ERR_ARG
    if (o.k < 1 || o.k > 3) return "k must be 1, 2 or 3";
    if (o.mixed != 0 && o.mixed != 1) return "mixed must be 0 (k' = k) or 1 (k' = k + 1)";
    if (o.alpha != 0 && o.alpha != 1) return "alpha must be 0 or 1";
    if (!(o.eta_f > 0.0) || !(o.eta_s > 0.0)) return "eta_f and eta_s must be positive";
    if (o.stab_speed != 0 && o.stab_speed != 1) return "stab_speed must be 0 (P-wave) or 1 (S-wave)";
    if (!(o.ell >= 0.0) || !std::isfinite(o.ell)) return "ell must be >= 0 and finite (0 = diameter of the mesh)";
    if (!(o.dt > 0.0) || !std::isfinite(o.dt)) return "dt must be positive and finite";
    if (nv <= 0 || nc <= 0 || !xy || !cell_ptr || !cell_vtx || !medium || !rho || !pa || !pb)
        return "empty mesh or null mesh array";
    P = Plan();
    if (!sdirk_tableau(o.stages, P.A, P.b, P.c)) return "stages must be 1, 2 or 3";
    P.stages = o.stages;
    P.dt = o.dt;
    P.ast = P.A[0][0];
    P.k = o.k;
    P.kp = o.k + o.mixed;
    P.N = (o.k + 1) * (o.k + 2) / 2;
    P.Np = (P.kp + 1) * (P.kp + 2) / 2;
    P.nf = o.k + 1;
    P.n_cells = nc;
    const int N = P.N, Np = P.Np, nf = P.nf, kp = P.kp;
    const double adt = P.ast * P.dt;

    *code = 2;  // HHO_ERR_MESH
    if (cell_ptr[0] != 0) return "cell_ptr[0] must be 0";
    for (int c = 0; c < nc; ++c) {
        const int n = cell_ptr[c + 1] - cell_ptr[c];
        if (n < 3 || n > kMaxEdges) return "cell " + std::to_string(c) + " has " + std::to_string(n) + " vertices (3..8 supported)";
    }
    const int ne = cell_ptr[nc];
    for (int e = 0; e < ne; ++e)
        if (cell_vtx[e] < 0 || cell_vtx[e] >= nv) return "vertex id out of range";
    *code = 1;
    for (int c = 0; c < nc; ++c) {
        if (medium[c] > 1) return "medium must be 0 (fluid) or 1 (solid)";
        if (!(rho[c] > 0.0)) return "rho must be positive";
        if (medium[c] == 0 && !(pa[c] > 0.0)) return "fluid sound speed must be positive";
        if (medium[c] == 1 && (!(pb[c] > 0.0) || !(pa[c] + pb[c] > 0.0))) return "solid needs mu > 0 and lambda + mu > 0";
    }
    P.xy.assign(xy, xy + 2 * nv);
    P.cell_ptr.assign(cell_ptr, cell_ptr + nc + 1);
    P.cell_vtx.assign(cell_vtx, cell_vtx + ne);
    P.medium.assign(medium, medium + nc);
    P.rho.assign(rho, rho + nc);

    // geometry: centroid (shoelace), diameter h_T = largest vertex distance
    *code = 2;
    P.centroid.resize(2 * nc);
    P.hT.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        const double ox = xy[2 * cell_vtx[s]], oy = xy[2 * cell_vtx[s] + 1];
        double A2 = 0.0, sx = 0.0, sy = 0.0, h = 0.0;
        for (int j = 0; j < n; ++j) {
            const int i0 = cell_vtx[s + j], i1 = cell_vtx[s + (j + 1) % n];
            const double x0 = xy[2 * i0] - ox, y0 = xy[2 * i0 + 1] - oy, x1 = xy[2 * i1] - ox, y1 = xy[2 * i1 + 1] - oy;
            const double cr = x0 * y1 - x1 * y0;
            A2 += cr;
            sx += (x0 + x1) * cr;
            sy += (y0 + y1) * cr;
            for (int m = 0; m < n; ++m) {
                const int i2 = cell_vtx[s + m];
                h = std::max(h, std::hypot(xy[2 * i2] - xy[2 * i0], xy[2 * i2 + 1] - xy[2 * i0 + 1]));
            }
        }
        if (!(A2 > 0.0)) return "cell " + std::to_string(c) + " is clockwise or degenerate";
        P.centroid[2 * c] = ox + sx / (3.0 * A2);
        P.centroid[2 * c + 1] = oy + sy / (3.0 * A2);
        P.hT[c] = h;
    }

    // faces: edges matched by their vertex pair, traversed in opposite directions
    std::vector<int> edge_face(ne, -1), fcell, fedge;  // fcell/fedge: [2 * n_faces]
    std::vector<int> fv;                               // [2 * n_faces], lower id first
    {
        std::unordered_map<uint64_t, int> seen;
        seen.reserve(2 * ne);
        for (int c = 0; c < nc; ++c) {
            const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
            for (int j = 0; j < n; ++j) {
                const int va = cell_vtx[s + j], vb = cell_vtx[s + (j + 1) % n];
                if (va == vb) return "repeated vertex in cell " + std::to_string(c);
                const uint64_t key = (uint64_t)std::min(va, vb) * (uint64_t)nv + (uint64_t)std::max(va, vb);
                auto it = seen.find(key);
                if (it == seen.end()) {
                    const int f = (int)(fv.size() / 2);
                    seen.emplace(key, f);
                    fv.push_back(std::min(va, vb));
                    fv.push_back(std::max(va, vb));
                    fcell.push_back(c); fcell.push_back(-1);
                    fedge.push_back(j); fedge.push_back(-1);
                    edge_face[s + j] = f;
                    continue;
                }
                const int f = it->second;
                if (fcell[2 * f + 1] >= 0) return "edge shared by more than two cells";
                const int c0 = fcell[2 * f], j0 = fedge[2 * f], s0 = cell_ptr[c0], n0 = cell_ptr[c0 + 1] - s0;
                if (cell_vtx[s0 + j0] != vb || cell_vtx[s0 + (j0 + 1) % n0] != va)
                    return "edge traversed in the same direction by two cells (inconsistent orientation)";
                fcell[2 * f + 1] = c;
                fedge[2 * f + 1] = j;
                edge_face[s + j] = f;
            }
        }
    }
    const int nfc = (int)(fv.size() / 2);
    P.n_faces = nfc;
    // widths: boundary 0, fluid 1, solid 2, interface 3 (times nf); interface = [p | v_x | v_y]
    std::vector<int> fw(nfc), foff(nfc + 1, 0);
    for (int f = 0; f < nfc; ++f) {
        const int c0 = fcell[2 * f], c1 = fcell[2 * f + 1];
        if (c1 < 0) fw[f] = 0;
        else if (medium[c0] != medium[c1]) fw[f] = 3;
        else fw[f] = medium[c0] == 0 ? 1 : 2;
        foff[f + 1] = foff[f] + fw[f] * nf;
    }
    *code = 1;
    if (foff[nfc] > (1 << 30)) return "too many face unknowns";
    P.n_fdof = foff[nfc];
    P.fdof_face.resize(3 * (size_t)P.n_fdof);
    for (int f = 0; f < nfc; ++f)
        for (int i = 0; i < fw[f] * nf; ++i) {
            P.fdof_face[3 * (size_t)(foff[f] + i)] = fv[2 * f];
            P.fdof_face[3 * (size_t)(foff[f] + i) + 1] = fv[2 * f + 1];
            P.fdof_face[3 * (size_t)(foff[f] + i) + 2] = i;
        }

    // l_Omega: given, or the largest distance between two boundary vertices (= diam of the domain)
    if (o.ell > 0.0) {
        P.ell = o.ell;
    } else {
        std::vector<int> bv;
        for (int f = 0; f < nfc; ++f)
            if (fcell[2 * f + 1] < 0) { bv.push_back(fv[2 * f]); bv.push_back(fv[2 * f + 1]); }
        std::sort(bv.begin(), bv.end());
        bv.erase(std::unique(bv.begin(), bv.end()), bv.end());
        double d2 = 0.0;
        for (size_t i = 0; i < bv.size(); ++i)
            for (size_t j = i + 1; j < bv.size(); ++j) {
                const double dx = xy[2 * bv[i]] - xy[2 * bv[j]], dy = xy[2 * bv[i] + 1] - xy[2 * bv[j] + 1];
                d2 = std::max(d2, dx * dx + dy * dy);
            }
        P.ell = std::sqrt(d2);
        if (!(P.ell > 0.0)) { *code = 2; return "mesh has no boundary"; }
    }

    // groups by (medium, number of face-slot unknowns)
    std::vector<int> nFT(nc);
    std::map<std::pair<int, int>, int> gid;
    for (int c = 0; c < nc; ++c) {
        int nb = 0;
        for (int e = cell_ptr[c]; e < cell_ptr[c + 1]; ++e) nb += fw[edge_face[e]] > 0;
        nFT[c] = nb * nf * (medium[c] == 0 ? 1 : 2);
        gid.emplace(std::make_pair((int)medium[c], nFT[c]), 0);
    }
    for (auto &kv : gid) {
        kv.second = (int)P.groups.size();
        Group g;
        g.medium = kv.first.first;
        g.nFT = kv.first.second;
        g.nT = g.medium == 0 ? Np + 2 * N : 2 * Np + 3 * N;
        P.groups.push_back(g);
    }
    P.cell_group.resize(nc);
    P.cell_index.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const int g = gid[std::make_pair((int)medium[c], nFT[c])];
        P.cell_group[c] = g;
        P.cell_index[c] = P.groups[g].n++;
    }
    {
        int64_t vo = 0, co = 0, mo = 0, wo = 0, xo = 0;
        for (auto &g : P.groups) {
            g.vec_off = vo; vo += (int64_t)g.nT * g.n;
            g.cf_off = co; co += (int64_t)g.nFT * g.n;
            g.mat_off = mo; mo += (int64_t)(g.nT + g.nFT) * g.nT * g.n;
            g.w_off = wo; wo += (int64_t)g.nT * g.nFT * g.n;
            g.m_off = xo; xo += (int64_t)kNumMat * g.n;
        }
        P.n_dof = vo;
        P.n_slot = co;
        P.mats.assign(mo, 0.0);
        P.wmat.assign(wo, 0.0);
        P.slot_dof.assign(co, -1);
        P.mat.assign(xo, 0.0);
    }
    P.ext_off.resize(nc + 1);
    P.ext_off[0] = 0;
    for (int c = 0; c < nc; ++c) P.ext_off[c + 1] = P.ext_off[c] + P.groups[P.cell_group[c]].nT;
    P.kappa.assign(nc, 0.0);

    std::vector<int> ex, ey;
    graded_exponents(kp, ex, ey);
    P.basisC.assign((size_t)nc * Np * Np, 0.0);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(P.n_fdof);

    *code = 3;  // HHO_ERR_SINGULAR
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        const Group &G = P.groups[P.cell_group[c]];
        const int ic = P.cell_index[c], nT = G.nT, nS = G.nFT;
        const double h = P.hT[c], cx = P.centroid[2 * c], cy = P.centroid[2 * c + 1];
        std::vector<double> X(n), Y(n);
        for (int j = 0; j < n; ++j) {
            X[j] = (xy[2 * cell_vtx[s + j]] - cx) / h;
            Y[j] = (xy[2 * cell_vtx[s + j] + 1] - cy) / h;
        }
        // moments of X^p Y^q (p + q <= 2k') over the scaled cell, Green's formula
        const int pm = 2 * kp;
        std::vector<double> mom((pm + 2) * (pm + 2), 0.0);
        auto Mo = [&](int p, int q) -> double & { return mom[p * (pm + 2) + q]; };
        for (int p = 0; p <= pm; ++p)
            for (int q = 0; p + q <= pm; ++q) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j) {
                    const double X0 = X[j], Y0 = Y[j], X1 = X[(j + 1) % n], Y1 = Y[(j + 1) % n];
                    double e = 0.0;
                    for (int g = 0; g < 5; ++g) {
                        const double t = 0.5 * (1.0 + kG5.x[g]);
                        e += 0.5 * kG5.w[g] * ipow(X0 + t * (X1 - X0), p + 1) * ipow(Y0 + t * (Y1 - Y0), q);
                    }
                    acc += e * (Y1 - Y0);
                }
                Mo(p, q) = acc / (p + 1);
            }
        std::vector<double> gram((size_t)Np * Np), L, C;
        for (int a = 0; a < Np; ++a)
            for (int b = 0; b < Np; ++b) gram[a * Np + b] = h * h * Mo(ex[a] + ex[b], ey[a] + ey[b]);
        if (!chol(Np, gram, L)) return "Gram matrix of cell " + std::to_string(c) + " is not positive definite";
        lower_inverse(Np, L, C);
        std::copy(C.begin(), C.end(), P.basisC.begin() + (size_t)c * Np * Np);
        // D_d[a][b] = (d_d phi'_b, phi_a)_T, a < N, b < Np
        std::vector<double> Dm[2] = {std::vector<double>((size_t)Np * Np, 0.0), std::vector<double>((size_t)Np * Np, 0.0)};
        for (int a = 0; a < Np; ++a)
            for (int b = 0; b < Np; ++b) {
                if (ex[b] > 0) Dm[0][a * Np + b] = ex[b] * h * Mo(ex[b] - 1 + ex[a], ey[b] + ey[a]);
                if (ey[b] > 0) Dm[1][a * Np + b] = ey[b] * h * Mo(ex[b] + ex[a], ey[b] - 1 + ey[a]);
            }
        std::vector<double> D[2];
        for (int d = 0; d < 2; ++d) {
            D[d].assign((size_t)N * Np, 0.0);
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < Np; ++b) {
                    double acc = 0.0;
                    for (int m = 0; m <= a; ++m)
                        for (int l = 0; l <= b; ++l) acc += C[a * Np + m] * Dm[d][m * Np + l] * C[b * Np + l];
                    D[d][a * Np + b] = acc;
                }
        }
        // materials and weights
        const bool fluid = medium[c] == 0;
        double tau, Ca = 0, Cb = 0, Cc = 0;
        const double scale = o.alpha ? P.ell / h : 1.0;
        if (fluid) {
            P.kappa[c] = rho[c] * pa[c] * pa[c];
            tau = o.eta_f / (rho[c] * pa[c]) * scale;
        } else {
            const double lam = pa[c], mu = pb[c];
            const double cs = o.stab_speed == 0 ? std::sqrt((lam + 2.0 * mu) / rho[c]) : std::sqrt(mu / rho[c]);
            tau = o.eta_s * rho[c] * cs * scale;
            const double q = lam / (2.0 * (lam + mu));
            Ca = (1.0 - q) / (2.0 * mu);
            Cb = -q / (2.0 * mu);
            Cc = 1.0 / (2.0 * mu);
        }
        // local blocks: cell rows/cols [0, nT), slots [0, nS)
        std::vector<double> KT((size_t)nT * nT, 0.0), KTF((size_t)nT * nS, 0.0), KFT((size_t)nS * nT, 0.0),
            KFF((size_t)nS * nS, 0.0), MT((size_t)nT * nT, 0.0);
        auto kt = [&](int r, int q) -> double & { return KT[(size_t)r * nT + q]; };
        auto ktf = [&](int r, int q) -> double & { return KTF[(size_t)r * nS + q]; };
        auto kft = [&](int r, int q) -> double & { return KFT[(size_t)r * nT + q]; };
        const int rp = 0, rm = Np;           // fluid rows: p, m_c at rm + c N
        const int rv = 0, rs = 2 * Np;       // solid rows: v_c at c Np, s_al at rs + al N
        if (fluid) {
            for (int a = 0; a < Np; ++a) MT[(size_t)(rp + a) * nT + rp + a] = 1.0 / P.kappa[c];
            for (int a = 0; a < 2 * N; ++a) MT[(size_t)(rm + a) * nT + rm + a] = rho[c];
            for (int cc = 0; cc < 2; ++cc)
                for (int a = 0; a < N; ++a)
                    for (int b = 0; b < Np; ++b) {
                        kt(rm + cc * N + a, rp + b) -= D[cc][a * Np + b];   // m rows: -(d_c p_T, r)_T
                        kt(rp + b, rm + cc * N + a) += D[cc][a * Np + b];   // p rows: (d_c q_T, m_c)_T
                    }
        } else {
            for (int a = 0; a < 2 * Np; ++a) MT[(size_t)(rv + a) * nT + rv + a] = rho[c];
            const double Cm[3][3] = {{Ca, Cb, 0}, {Cb, Ca, 0}, {0, 0, Cc}};
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be)
                    if (Cm[al][be] != 0.0)
                        for (int a = 0; a < N; ++a) MT[(size_t)(rs + al * N + a) * nT + rs + be * N + a] = Cm[al][be];
            for (int al = 0; al < 3; ++al)
                for (int cc = 0; cc < 2; ++cc)
                    for (int d = 0; d < 2; ++d) {
                        const double e = tensor_basis(al, cc, d);
                        if (e == 0.0) continue;
                        for (int a = 0; a < N; ++a)
                            for (int b = 0; b < Np; ++b) {
                                kt(rs + al * N + a, rv + cc * Np + b) -= e * D[d][a * Np + b];
                                kt(rv + cc * Np + b, rs + al * N + a) += e * D[d][a * Np + b];
                            }
                    }
        }
        int slot = 0;
        for (int j = 0; j < n; ++j) {
            const int f = edge_face[s + j];
            const int va = cell_vtx[s + j], vb = cell_vtx[s + (j + 1) % n];
            const double dx = xy[2 * vb] - xy[2 * va], dy = xy[2 * vb + 1] - xy[2 * va + 1], len = std::hypot(dx, dy);
            const double nrm[2] = {dy / len, -dx / len};
            const int lo = fv[2 * f], hi = fv[2 * f + 1];
            // face moments on the 5 Gauss points, running from the lower to the higher vertex id
            std::vector<double> Ep((size_t)N * Np, 0.0), Gp((size_t)Np * nf, 0.0), MF((size_t)nf * nf, 0.0);
            for (int g = 0; g < 5; ++g) {
                const double t = 0.5 * (1.0 + kG5.x[g]), w = 0.5 * kG5.w[g] * len;
                const double x = xy[2 * lo] + t * (xy[2 * hi] - xy[2 * lo]), y = xy[2 * lo + 1] + t * (xy[2 * hi + 1] - xy[2 * lo + 1]);
                const double Xq = (x - cx) / h, Yq = (y - cy) / h;
                double mu[15], ph[15], psi[4];
                for (int m = 0; m < Np; ++m) mu[m] = ipow(Xq, ex[m]) * ipow(Yq, ey[m]);
                for (int a = 0; a < Np; ++a) {
                    double acc = 0.0;
                    for (int m = 0; m <= a; ++m) acc += C[a * Np + m] * mu[m];
                    ph[a] = acc;
                }
                for (int i = 0; i < nf; ++i) psi[i] = std::sqrt((2.0 * i + 1.0) / len) * legendre_p(i, kG5.x[g]);
                for (int a = 0; a < N; ++a)
                    for (int b = 0; b < Np; ++b) Ep[a * Np + b] += w * ph[a] * ph[b];
                for (int a = 0; a < Np; ++a)
                    for (int i = 0; i < nf; ++i) Gp[a * nf + i] += w * ph[a] * psi[i];
                for (int i = 0; i < nf; ++i)
                    for (int l = 0; l < nf; ++l) MF[i * nf + l] += w * psi[i] * psi[l];
            }
            std::vector<double> Pp((size_t)Np * Np, 0.0);  // (Pi phi'_b, Pi phi'_a)_F
            for (int a = 0; a < Np; ++a)
                for (int b = 0; b < Np; ++b) {
                    double acc = 0.0;
                    for (int i = 0; i < nf; ++i) acc += Gp[a * nf + i] * Gp[b * nf + i];
                    Pp[a * Np + b] = acc;
                }
            const bool bnd = fw[f] == 0;
            if (fluid) {
                for (int cc = 0; cc < 2; ++cc)
                    for (int a = 0; a < N; ++a)
                        for (int b = 0; b < Np; ++b) {
                            kt(rm + cc * N + a, rp + b) += nrm[cc] * Ep[a * Np + b];   // +(p_T, r n_c)_F
                            kt(rp + b, rm + cc * N + a) -= nrm[cc] * Ep[a * Np + b];   // -(q_T, m . n)_F
                        }
                for (int a = 0; a < Np; ++a)
                    for (int b = 0; b < Np; ++b) kt(rp + a, rp + b) += tau * Pp[a * Np + b];
                if (!bnd) {
                    for (int i = 0; i < nf; ++i) {
                        const int q = slot + i;
                        for (int cc = 0; cc < 2; ++cc)
                            for (int a = 0; a < N; ++a) {
                                ktf(rm + cc * N + a, q) -= nrm[cc] * Gp[a * nf + i];   // -(p_F, r n_c)_F
                                kft(q, rm + cc * N + a) += nrm[cc] * Gp[a * nf + i];   // +(q_F, m . n)_F
                            }
                        for (int a = 0; a < Np; ++a) {
                            ktf(rp + a, q) -= tau * Gp[a * nf + i];
                            kft(q, rp + a) -= tau * Gp[a * nf + i];
                        }
                        for (int l = 0; l < nf; ++l) KFF[(size_t)q * nS + slot + l] += tau * MF[i * nf + l];
                    }
                    const int base = foff[f];
                    for (int i = 0; i < nf; ++i) P.slot_dof[G.cf_off + (int64_t)(slot + i) * G.n + ic] = base + i;
                    slot += nf;
                }
            } else {
                for (int al = 0; al < 3; ++al)
                    for (int cc = 0; cc < 2; ++cc) {
                        const double en = tensor_basis(al, cc, 0) * nrm[0] + tensor_basis(al, cc, 1) * nrm[1];
                        if (en == 0.0) continue;
                        for (int a = 0; a < N; ++a)
                            for (int b = 0; b < Np; ++b) {
                                kt(rs + al * N + a, rv + cc * Np + b) += en * Ep[a * Np + b];
                                kt(rv + cc * Np + b, rs + al * N + a) -= en * Ep[a * Np + b];
                            }
                    }
                for (int cc = 0; cc < 2; ++cc)
                    for (int a = 0; a < Np; ++a)
                        for (int b = 0; b < Np; ++b) kt(rv + cc * Np + a, rv + cc * Np + b) += tau * Pp[a * Np + b];
                if (!bnd) {
                    for (int cc = 0; cc < 2; ++cc)
                        for (int i = 0; i < nf; ++i) {
                            const int q = slot + cc * nf + i;
                            for (int al = 0; al < 3; ++al) {
                                const double en = tensor_basis(al, cc, 0) * nrm[0] + tensor_basis(al, cc, 1) * nrm[1];
                                if (en == 0.0) continue;
                                for (int a = 0; a < N; ++a) {
                                    ktf(rs + al * N + a, q) -= en * Gp[a * nf + i];
                                    kft(q, rs + al * N + a) += en * Gp[a * nf + i];
                                }
                            }
                            for (int a = 0; a < Np; ++a) {
                                ktf(rv + cc * Np + a, q) -= tau * Gp[a * nf + i];
                                kft(q, rv + cc * Np + a) -= tau * Gp[a * nf + i];
                            }
                            for (int l = 0; l < nf; ++l) KFF[(size_t)q * nS + slot + cc * nf + l] += tau * MF[i * nf + l];
                        }
                    const int base = foff[f] + (fw[f] == 3 ? nf : 0);
                    for (int q = 0; q < 2 * nf; ++q) P.slot_dof[G.cf_off + (int64_t)(slot + q) * G.n + ic] = base + q;
                    if (fw[f] == 3) {
                        // coupling: fluid face rows +(v_F . n_G, q_F)_F, solid face rows -(p_F n_G, w_F)_F,
                        // n_G the outward normal of this (solid) cell
                        for (int i = 0; i < nf; ++i)
                            for (int cc = 0; cc < 2; ++cc)
                                for (int l = 0; l < nf; ++l) {
                                    const double v = adt * nrm[cc] * MF[i * nf + l];
                                    rows[foff[f] + i].push_back({foff[f] + nf + cc * nf + l, v});
                                    rows[foff[f] + nf + cc * nf + l].push_back({foff[f] + i, -v});
                                }
                    }
                    slot += 2 * nf;
                }
            }
        }
        // condensation of the cell unknowns
        std::vector<double> Amat((size_t)nT * nT), Ainv;
        for (size_t q = 0; q < Amat.size(); ++q) Amat[q] = MT[q] + adt * KT[q];
        if (!scaled_inverse(nT, Amat, Ainv)) return "stage matrix of cell " + std::to_string(c) + " is singular";
        std::vector<double> V((size_t)nS * nT, 0.0), W((size_t)nT * nS, 0.0), ST((size_t)nS * nS, 0.0);
        for (int q = 0; q < nS; ++q)
            for (int r = 0; r < nT; ++r) {
                double acc = 0.0;
                for (int m = 0; m < nT; ++m) acc += KFT[(size_t)q * nT + m] * Ainv[(size_t)m * nT + r];
                V[(size_t)q * nT + r] = adt * acc;
            }
        for (int r = 0; r < nT; ++r)
            for (int q = 0; q < nS; ++q) {
                double acc = 0.0;
                for (int m = 0; m < nT; ++m) acc += Ainv[(size_t)r * nT + m] * KTF[(size_t)m * nS + q];
                W[(size_t)r * nS + q] = adt * acc;
            }
        for (int q = 0; q < nS; ++q)
            for (int q2 = 0; q2 < nS; ++q2) {
                double acc = 0.0;
                for (int m = 0; m < nT; ++m) acc += KFT[(size_t)q * nT + m] * W[(size_t)m * nS + q2];
                ST[(size_t)q * nS + q2] = adt * (KFF[(size_t)q * nS + q2] - acc);
            }
        // store [Ainv; V] and W, [row][col][cell] within the group
        for (int r = 0; r < nT + nS; ++r)
            for (int q = 0; q < nT; ++q)
                P.mats[G.mat_off + ((int64_t)r * nT + q) * G.n + ic] =
                    r < nT ? Ainv[(size_t)r * nT + q] : V[(size_t)(r - nT) * nT + q];
        for (int r = 0; r < nT; ++r)
            for (int q = 0; q < nS; ++q) P.wmat[G.w_off + ((int64_t)r * nS + q) * G.n + ic] = W[(size_t)r * nS + q];
        const double m8[kNumMat] = {fluid ? 1.0 / P.kappa[c] : rho[c], fluid ? rho[c] : Ca, fluid ? P.kappa[c] : Cb,
                                    fluid ? 1.0 / rho[c] : Cc, fluid ? 0.0 : 1.0 / rho[c],
                                    fluid ? 0.0 : Ca / (Ca * Ca - Cb * Cb), fluid ? 0.0 : -Cb / (Ca * Ca - Cb * Cb),
                                    fluid ? 0.0 : 1.0 / Cc};
        for (int q = 0; q < kNumMat; ++q) P.mat[G.m_off + (int64_t)q * G.n + ic] = m8[q];
        for (int q = 0; q < nS; ++q) {
            const int dq = P.slot_dof[G.cf_off + (int64_t)q * G.n + ic];
            for (int q2 = 0; q2 < nS; ++q2)
                rows[dq].push_back({P.slot_dof[G.cf_off + (int64_t)q2 * G.n + ic], ST[(size_t)q * nS + q2]});
        }
    }

    // CSR of the face matrix (duplicates summed), block-Jacobi inverse per face
    P.S_ptr.assign(P.n_fdof + 1, 0);
    for (int d = 0; d < P.n_fdof; ++d) {
        auto &rw = rows[d];
        std::sort(rw.begin(), rw.end(), [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
            return x.first < y.first;
        });
        size_t m = 0;
        for (size_t q = 0; q < rw.size(); ++q) {
            if (m > 0 && rw[m - 1].first == rw[q].first) rw[m - 1].second += rw[q].second;
            else rw[m++] = rw[q];
        }
        rw.resize(m);
        P.S_ptr[d + 1] = P.S_ptr[d] + (int32_t)m;
    }
    P.S_col.resize(P.S_ptr[P.n_fdof]);
    P.S_val.resize(P.S_ptr[P.n_fdof]);
    for (int d = 0; d < P.n_fdof; ++d)
        for (int q = P.S_ptr[d]; q < P.S_ptr[d + 1]; ++q) {
            P.S_col[q] = rows[d][q - P.S_ptr[d]].first;
            P.S_val[q] = rows[d][q - P.S_ptr[d]].second;
        }
    P.dscale.assign(P.n_fdof, 1.0);
    for (int d = 0; d < P.n_fdof; ++d) {
        double dg = 0.0;
        for (int q = P.S_ptr[d]; q < P.S_ptr[d + 1]; ++q)
            if (P.S_col[q] == d) dg = P.S_val[q];
        if (!(dg > 0.0) || !std::isfinite(dg)) { *code = 3; return "face matrix has a non-positive diagonal entry"; }
        P.dscale[d] = 1.0 / std::sqrt(dg);
    }
    P.P_ptr.assign(P.n_fdof + 1, 0);
    for (int f = 0; f < nfc; ++f) {
        const int w = fw[f] * nf, d0 = foff[f];
        if (!w) continue;
        std::vector<double> B((size_t)w * w, 0.0), Bi;
        for (int i = 0; i < w; ++i)
            for (int q = P.S_ptr[d0 + i]; q < P.S_ptr[d0 + i + 1]; ++q) {
                const int col = P.S_col[q];
                if (col >= d0 && col < d0 + w)
                    B[(size_t)i * w + (col - d0)] = P.dscale[d0 + i] * P.S_val[q] * P.dscale[col];
            }
        if (!scaled_inverse(w, B, Bi)) return "diagonal block of face " + std::to_string(f) + " is singular";
        for (int i = 0; i < w; ++i) {
            P.P_ptr[d0 + i + 1] = w;
            for (int j = 0; j < w; ++j) { P.P_col.push_back(d0 + j); P.P_val.push_back(Bi[(size_t)i * w + j]); }
        }
    }
    for (int d = 0; d < P.n_fdof; ++d) P.P_ptr[d + 1] += P.P_ptr[d];
    P.feed.assign(2 * (size_t)P.n_fdof, -1);
    for (int64_t q = 0; q < P.n_slot; ++q) {
        const int d = P.slot_dof[q];
        if (d < 0) { *code = 2; return "internal: unassigned face slot"; }
        if (P.feed[2 * d] < 0) P.feed[2 * d] = (int32_t)q;
        else if (P.feed[2 * d + 1] < 0) P.feed[2 * d + 1] = (int32_t)q;
        else { *code = 2; return "internal: face unknown fed by more than two cells"; }
    }
    *code = 0;
    return "";
}

}  // namespace imp
}  // namespace hho
