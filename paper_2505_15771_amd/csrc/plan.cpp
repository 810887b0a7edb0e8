// Host-side construction of the execution plan (float64): mesh validation, face
// matching and tagging (Sec. 3.1), per-shape-class local operators in the
// orthonormal cell / face bases (Sec. 3.3, eq. rec_a, rec_e, stab), materials and
// stabilisation weights (eq. stab with alpha = 0, weights eta of Sec. 5.1), and the
// grouping of cells by (medium, shape class) into structure-of-arrays buffers.
//
// Integrals are exact for the polynomial integrands involved: cell moments of the
// scaled monomials come from Green's formula (a boundary integral of
// X^{p+1} Y^q / (p+1) dY) evaluated with 5-point Gauss-Legendre on every edge, and
// face integrals use the same 5-point rule (exact to degree 9 >= 2k + 1).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

namespace hho {

namespace {

// 5-point Gauss-Legendre rule on [-1, 1] in closed form.
struct GL5 {
    double x[5], w[5];
    GL5() {
        const double r = std::sqrt(10.0 / 7.0);
        const double a = std::sqrt(5.0 - 2.0 * r) / 3.0, b = std::sqrt(5.0 + 2.0 * r) / 3.0;
        const double wa = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0;
        const double wb = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
        x[0] = -b; w[0] = wb;
        x[1] = -a; w[1] = wa;
        x[2] = 0.0; w[2] = 128.0 / 225.0;
        x[3] = a; w[3] = wa;
        x[4] = b; w[4] = wb;
    }
};
const GL5 kGL;

// graded monomial exponents: degree-major, decreasing power of x within a degree
void exponents(int k, std::vector<int> &px, std::vector<int> &py) {
    px.clear();
    py.clear();
    for (int d = 0; d <= k; ++d)
        for (int a = d; a >= 0; --a) {
            px.push_back(a);
            py.push_back(d - a);
        }
}

double powi(double x, int e) {
    double r = 1.0;
    while (e-- > 0) r *= x;
    return r;
}

// Legendre polynomial P_i(x) by the three-term recurrence.
double legendre(int i, double x) {
    if (i == 0) return 1.0;
    double p0 = 1.0, p1 = x;
    for (int n = 1; n < i; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// Dense Cholesky A = L L^T (lower, row-major); false if not positive definite.
bool cholesky(int n, const std::vector<double> &A, std::vector<double> &L) {
    L.assign(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int m = 0; m < j; ++m) d -= L[j * n + m] * L[j * n + m];
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int m = 0; m < j; ++m) s -= L[i * n + m] * L[j * n + m];
            L[i * n + j] = s / ljj;
        }
    }
    return true;
}

// Inverse of a lower-triangular matrix by forward substitution on the unit columns.
void invert_lower(int n, const std::vector<double> &L, std::vector<double> &Li) {
    Li.assign(n * n, 0.0);
    for (int col = 0; col < n; ++col) {
        for (int i = col; i < n; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int m = col; m < i; ++m) s -= L[i * n + m] * Li[m * n + col];
            Li[i * n + col] = s / L[i * n + i];
        }
    }
}

struct CellGeom {
    double area, cx, cy, h;
};

}  // namespace

int trace_rows(const Plan &plan) { return plan.max_nf * plan.tcomp * plan.F; }

void eval_basis(const Plan &plan, int c, double x, double y, double *phi) {
    const int N = plan.N;
    std::vector<int> px, py;
    exponents(plan.k, px, py);
    const double h = plan.hT[c];
    const double X = (x - plan.centroid[2 * c]) / h, Y = (y - plan.centroid[2 * c + 1]) / h;
    const double *C = plan.basisC.data() + (size_t)plan.cell_class[c] * N * N;
    double mu[16];
    for (int m = 0; m < N; ++m) mu[m] = powi(X, px[m]) * powi(Y, py[m]);
    for (int a = 0; a < N; ++a) {
        double s = 0.0;
        for (int m = 0; m <= a; ++m) s += C[a * N + m] * mu[m];
        phi[a] = s;
    }
}

int locate_cell(const Plan &plan, double x, double y) {
    for (int c = 0; c < plan.n_cells; ++c) {
        const int s = plan.cell_ptr[c], n = plan.cell_ptr[c + 1] - s;
        const double tol = 1e-12 * plan.hT[c];
        bool inside = true;
        for (int j = 0; j < n && inside; ++j) {
            const int i0 = plan.cell_vtx[s + j], i1 = plan.cell_vtx[s + (j + 1) % n];
            const double ex = plan.xy[2 * i1] - plan.xy[2 * i0], ey = plan.xy[2 * i1 + 1] - plan.xy[2 * i0 + 1];
            const double cr = ex * (y - plan.xy[2 * i0 + 1]) - ey * (x - plan.xy[2 * i0]);
            if (cr < -tol * std::hypot(ex, ey)) inside = false;
        }
        if (inside) return c;
    }
    return -1;
}

std::string build_plan(int nv, const double *xy, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                       const uint8_t *medium, const double *rho, const double *pa, const double *pb, int k,
                       double eta_f, double eta_s, int stab_speed, int n_shots, Plan &P, int *code) {
    *code = 1;  // HHO_ERR_ARG
    if (k < 1 || k > 3) return "k must be 1, 2 or 3";
    if (nv <= 0 || nc <= 0 || !xy || !cell_ptr || !cell_vtx || !medium || !rho || !pa || !pb)
        return "empty mesh or null mesh array";
    if (n_shots < 1 || n_shots > kBlock) return "n_shots must be in 1..256";
    if (!(eta_f > 0.0) || !(eta_s > 0.0)) return "eta_f and eta_s must be positive";
    if (stab_speed != 0 && stab_speed != 1) return "stab_speed must be 0 (P-wave) or 1 (S-wave)";
    P = Plan();
    P.k = k;
    P.N = (k + 1) * (k + 2) / 2;
    P.F = k + 1;
    P.S = n_shots;
    P.stab_speed = stab_speed;
    P.eta_f = eta_f;
    P.eta_s = eta_s;
    P.n_cells = nc;
    P.n_vertices = nv;
    const int N = P.N, F = P.F;
    *code = 2;  // HHO_ERR_MESH
    if (cell_ptr[0] != 0) return "cell_ptr[0] must be 0";
    for (int c = 0; c < nc; ++c) {
        const int n = cell_ptr[c + 1] - cell_ptr[c];
        if (n < 3 || n > kMaxFaces) return "cell " + std::to_string(c) + " has " + std::to_string(n) +
                                            " vertices (3.." + std::to_string(kMaxFaces) + " supported)";
        P.max_nf = std::max(P.max_nf, n);
    }
    const int ne = cell_ptr[nc];
    for (int e = 0; e < ne; ++e)
        if (cell_vtx[e] < 0 || cell_vtx[e] >= nv) return "vertex id out of range";
    P.xy.assign(xy, xy + 2 * nv);
    P.cell_ptr.assign(cell_ptr, cell_ptr + nc + 1);
    P.cell_vtx.assign(cell_vtx, cell_vtx + ne);
    P.medium.assign(medium, medium + nc);

    // materials
    *code = 1;
    for (int c = 0; c < nc; ++c) {
        if (medium[c] > 1) return "medium must be 0 (fluid) or 1 (solid)";
        if (!(rho[c] > 0.0)) return "rho must be positive";
        if (medium[c] == kFluid && !(pa[c] > 0.0)) return "fluid sound speed must be positive";
        if (medium[c] == kSolid && (!(pb[c] > 0.0) || !(pa[c] + pb[c] > 0.0)))
            return "solid needs mu > 0 and lambda + mu > 0";
    }

    // geometry: shoelace area and centroid, diameter = largest vertex distance
    *code = 2;
    std::vector<CellGeom> geo(nc);
    P.centroid.resize(2 * nc);
    P.hT.resize(nc);
    P.area.resize(nc);
    double hsum = 0.0;
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        // shift by the first vertex for accuracy
        const double ox = xy[2 * cell_vtx[s]], oy = xy[2 * cell_vtx[s] + 1];
        double A2 = 0.0, sx = 0.0, sy = 0.0, h = 0.0;
        for (int j = 0; j < n; ++j) {
            const int i0 = cell_vtx[s + j], i1 = cell_vtx[s + (j + 1) % n];
            const double x0 = xy[2 * i0] - ox, y0 = xy[2 * i0 + 1] - oy;
            const double x1 = xy[2 * i1] - ox, y1 = xy[2 * i1 + 1] - oy;
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
        geo[c] = {0.5 * A2, ox + sx / (3.0 * A2), oy + sy / (3.0 * A2), h};
        P.centroid[2 * c] = geo[c].cx;
        P.centroid[2 * c + 1] = geo[c].cy;
        P.hT[c] = h;
        P.area[c] = 0.5 * A2;
        hsum += h;
    }

    // faces: each edge shared by at most two cells, traversed in opposite directions
    std::vector<int> nbr_cell(ne, -1), nbr_j(ne, -1), cell_of_edge(ne);
    for (int c = 0; c < nc; ++c)
        for (int e = cell_ptr[c]; e < cell_ptr[c + 1]; ++e) cell_of_edge[e] = c;
    {
        std::unordered_map<uint64_t, int> first;
        first.reserve(2 * ne);
        int nfaces = 0;
        for (int c = 0; c < nc; ++c) {
            const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
            for (int j = 0; j < n; ++j) {
                const uint64_t va = (uint64_t)cell_vtx[s + j], vb = (uint64_t)cell_vtx[s + (j + 1) % n];
                if (va == vb) return "repeated vertex in cell " + std::to_string(c);
                const uint64_t key = std::min(va, vb) * (uint64_t)nv + std::max(va, vb);
                auto it = first.find(key);
                if (it == first.end()) {
                    first.emplace(key, s + j);
                    ++nfaces;
                    continue;
                }
                const int e0 = it->second;
                if (e0 < 0) return "edge shared by more than two cells";
                const int c0 = cell_of_edge[e0];
                const int n0 = cell_ptr[c0 + 1] - cell_ptr[c0], j0 = e0 - cell_ptr[c0];
                if ((uint64_t)cell_vtx[cell_ptr[c0] + j0] != vb ||
                    (uint64_t)cell_vtx[cell_ptr[c0] + (j0 + 1) % n0] != va)
                    return "edge traversed in the same direction by two cells (inconsistent orientation)";
                nbr_cell[e0] = c;
                nbr_j[e0] = j;
                nbr_cell[s + j] = c0;
                nbr_j[s + j] = j0;
                it->second = -1;
            }
        }
        P.n_faces = nfaces;
    }

    // shape classes: cells equal up to translation (vertex offsets from the first vertex)
    std::vector<int> px, py;
    exponents(k, px, py);
    const double quantum = 1e-9 * hsum / nc;
    std::map<std::vector<int64_t>, int> class_of_key;
    P.cell_class.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        std::vector<int64_t> key;
        key.reserve(2 * n + 1);
        key.push_back(n);
        const double ox = xy[2 * cell_vtx[s]], oy = xy[2 * cell_vtx[s] + 1];
        for (int j = 1; j < n; ++j) {
            key.push_back(std::llround((xy[2 * cell_vtx[s + j]] - ox) / quantum));
            key.push_back(std::llround((xy[2 * cell_vtx[s + j] + 1] - oy) / quantum));
        }
        auto it = class_of_key.find(key);
        if (it == class_of_key.end()) {
            const int id = (int)P.classes.size();
            class_of_key.emplace(std::move(key), id);
            ClassInfo ci;
            ci.nF = n;
            ci.rep_cell = c;
            P.classes.push_back(ci);
            P.cell_class[c] = id;
        } else {
            P.cell_class[c] = it->second;
        }
    }

    // on a mesh with many shape classes (e.g. vertices moved at random: every cell its own shape),
    // the small classes (fewer than kPoolCells cells) are pooled: their tables use the face count
    // of their pooled group.  A few small classes (hanging nodes, cut cells) keep their groups.
    for (int c = 0; c < nc; ++c) P.classes[P.cell_class[c]].ncells += 1;
    const bool pool = (int)P.classes.size() > kPoolMinClasses;
    for (auto &ci : P.classes) {
        ci.pooled = pool && ci.ncells < kPoolCells;
        ci.nF_layout = !ci.pooled ? ci.nF : (ci.nF <= 4 ? std::min(4, P.max_nf) : P.max_nf);
    }

    // per-class tables in the orthonormal bases
    *code = 3;  // HHO_ERR_SINGULAR
    P.basisC.assign(P.classes.size() * N * N, 0.0);
    for (size_t cl = 0; cl < P.classes.size(); ++cl) {
        ClassInfo &ci = P.classes[cl];
        const int c = ci.rep_cell, s = cell_ptr[c], n = ci.nF;
        const double h = geo[c].h, h2 = h * h;
        std::vector<double> X(n), Y(n);
        for (int j = 0; j < n; ++j) {
            X[j] = (xy[2 * cell_vtx[s + j]] - geo[c].cx) / h;
            Y[j] = (xy[2 * cell_vtx[s + j] + 1] - geo[c].cy) / h;
        }
        // moments of X^p Y^q over the scaled cell by Green's formula
        const int pm = 2 * k + 1;
        std::vector<double> mom((pm + 1) * (pm + 1), 0.0);
        for (int p = 0; p <= pm; ++p)
            for (int q = 0; p + q <= 2 * k; ++q) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j) {
                    const double X0 = X[j], Y0 = Y[j], X1 = X[(j + 1) % n], Y1 = Y[(j + 1) % n];
                    double e = 0.0;
                    for (int g = 0; g < 5; ++g) {
                        const double t = 0.5 * (1.0 + kGL.x[g]);
                        e += 0.5 * kGL.w[g] * powi(X0 + t * (X1 - X0), p + 1) * powi(Y0 + t * (Y1 - Y0), q);
                    }
                    acc += e * (Y1 - Y0);
                }
                mom[p * (pm + 1) + q] = acc / (p + 1);
            }
        auto M = [&](int p, int q) { return mom[p * (pm + 1) + q]; };
        std::vector<double> gram(N * N), L, C;
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) gram[a * N + b] = h2 * M(px[a] + px[b], py[a] + py[b]);
        if (!cholesky(N, gram, L)) return "Gram matrix of cell " + std::to_string(c) + " is not positive definite";
        invert_lower(N, L, C);
        std::copy(C.begin(), C.end(), P.basisC.begin() + cl * N * N);
        // monomial derivative blocks Dm_c[a][b] = (d_c mu_b, mu_a)_T
        std::vector<double> Dmx(N * N, 0.0), Dmy(N * N, 0.0);
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
                if (px[b] > 0) Dmx[a * N + b] = px[b] * h * M(px[b] - 1 + px[a], py[b] + py[a]);
                if (py[b] > 0) Dmy[a * N + b] = py[b] * h * M(px[b] + px[a], py[b] - 1 + py[a]);
            }
        // D_c = C Dm_c C^T
        auto congr = [&](const std::vector<double> &Dm, std::vector<double> &D) {
            D.assign(N * N, 0.0);
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    double v = 0.0;
                    for (int i = 0; i <= a; ++i)
                        for (int j = 0; j <= b; ++j) v += C[a * N + i] * Dm[i * N + j] * C[b * N + j];
                    D[a * N + b] = v;
                }
        };
        std::vector<double> Dx, Dy;
        congr(Dmx, Dx);
        congr(Dmy, Dy);
        // faces: E_j = (phi_b, phi_a)_F, G_j = (phi_a, psi_i)_F in the local (counter-clockwise) face basis
        const int nl = ci.nF_layout;  // table layout: faces beyond n hold zeros
        std::vector<double> Bx = Dx, By = Dy, Ssum(N * N, 0.0), G(nl * N * F, 0.0), nrm(2 * nl, 0.0);
        for (int j = 0; j < n; ++j) {
            const double X0 = X[j], Y0 = Y[j], X1 = X[(j + 1) % n], Y1 = Y[(j + 1) % n];
            const double dX = X1 - X0, dY = Y1 - Y0, Ls = std::hypot(dX, dY), Lf = Ls * h;
            const double nx = dY / Ls, ny = -dX / Ls;
            nrm[2 * j] = nx;
            nrm[2 * j + 1] = ny;
            std::vector<double> E(N * N, 0.0);
            for (int g = 0; g < 5; ++g) {
                const double xi = kGL.x[g], t = 0.5 * (1.0 + xi), wq = 0.5 * kGL.w[g] * Lf;
                const double Xq = X0 + t * dX, Yq = Y0 + t * dY;
                double mu[16], phi[16], psi[8];
                for (int m = 0; m < N; ++m) mu[m] = powi(Xq, px[m]) * powi(Yq, py[m]);
                for (int a = 0; a < N; ++a) {
                    double v = 0.0;
                    for (int m = 0; m <= a; ++m) v += C[a * N + m] * mu[m];
                    phi[a] = v;
                }
                for (int i = 0; i < F; ++i) psi[i] = std::sqrt((2.0 * i + 1.0) / Lf) * legendre(i, xi);
                for (int a = 0; a < N; ++a) {
                    for (int b = 0; b < N; ++b) E[a * N + b] += wq * phi[a] * phi[b];
                    for (int i = 0; i < F; ++i) G[(j * N + a) * F + i] += wq * phi[a] * psi[i];
                }
            }
            for (int q = 0; q < N * N; ++q) {
                Bx[q] -= nx * E[q];
                By[q] -= ny * E[q];
                Ssum[q] += E[q];
            }
        }
        // B_c = -D_c^T vanishes where deg(b) >= deg(r) (the derivative of a graded orthonormal basis
        // function is orthogonal to all functions of its degree and above): store exact zeros there,
        // after checking that the computed values are round-off
        {
            const int deg[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
            double bmax = 0.0, zmax = 0.0;
            for (int q = 0; q < N * N; ++q) bmax = std::max({bmax, std::fabs(Bx[q]), std::fabs(By[q])});
            for (int r = 0; r < N; ++r)
                for (int b = 0; b < N; ++b)
                    if (deg[b] >= deg[r]) {
                        zmax = std::max({zmax, std::fabs(Bx[r * N + b]), std::fabs(By[r * N + b])});
                        Bx[r * N + b] = By[r * N + b] = 0.0;
                    }
            // G_j[a][i] = (phi_a, psi_i)_F vanishes where i > deg(a)
            double gmax = 0.0, gzero = 0.0;
            for (double v : G) gmax = std::max(gmax, std::fabs(v));
            for (int j = 0; j < n; ++j)
                for (int a2 = 0; a2 < N; ++a2)
                    for (int i = 0; i < F; ++i)
                        if (i > deg[a2]) {
                            double &g = G[(j * N + a2) * F + i];
                            gzero = std::max(gzero, std::fabs(g));
                            g = 0.0;
                        }
            if (zmax > 1e-9 * bmax || gzero > 1e-9 * gmax) {
                *code = 3;  // HHO_ERR_SINGULAR
                return "cell " + std::to_string(c) + ": local gradient operator lost its degree structure "
                       "(ill-conditioned cell basis)";
            }
        }
        ci.offset = (int)P.tables.size();
        if (!ci.pooled) {
            P.tables.insert(P.tables.end(), Bx.begin(), Bx.end());
            P.tables.insert(P.tables.end(), By.begin(), By.end());
            P.tables.insert(P.tables.end(), Ssum.begin(), Ssum.end());
            P.tables.insert(P.tables.end(), G.begin(), G.end());
            P.tables.insert(P.tables.end(), nrm.begin(), nrm.end());
        } else {
            // packed (read per lane): the structurally nonzero entries of B_x and B_y, the upper
            // triangle of the symmetric S, the structurally nonzero entries of every G_j, the normals
            const int deg[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
            for (const std::vector<double> *Bc : {&Bx, &By})
                for (int r = 0; r < N; ++r)
                    for (int b = 0; b < N; ++b)
                        if (deg[b] < deg[r]) P.tables.push_back((*Bc)[r * N + b]);
            for (int r = 0; r < N; ++r)
                for (int b = r; b < N; ++b) P.tables.push_back(Ssum[r * N + b]);
            for (int j = 0; j < nl; ++j)
                for (int a2 = 0; a2 < N; ++a2)
                    for (int i = 0; i < F; ++i)
                        if (i <= deg[a2]) P.tables.push_back(G[(j * N + a2) * F + i]);
            P.tables.insert(P.tables.end(), nrm.begin(), nrm.end());
        }
    }

    // per-cell stabilisation weight eta * tau_T (alpha = 0) and elastic constants
    std::vector<double> tau(nc);
    for (int c = 0; c < nc; ++c) {
        if (medium[c] == kFluid) {
            tau[c] = eta_f / (rho[c] * pa[c]);
        } else {
            const double lam = pa[c], mu = pb[c];
            const double cs = stab_speed == 0 ? std::sqrt((lam + 2.0 * mu) / rho[c]) : std::sqrt(mu / rho[c]);
            tau[c] = eta_s * rho[c] * cs;
        }
    }

    // groups (medium, class) in order of first appearance; cells of a group in input order
    std::map<std::pair<int, int>, int> gid;
    std::vector<std::vector<int>> members;
    for (int c = 0; c < nc; ++c) {
        const ClassInfo &cc = P.classes[P.cell_class[c]];
        auto key = cc.pooled ? std::make_pair((int)medium[c], -1 - cc.nF_layout) : std::make_pair((int)medium[c], P.cell_class[c]);
        auto it = gid.find(key);
        int g;
        if (it == gid.end()) {
            g = (int)P.groups.size();
            gid.emplace(key, g);
            Group G;
            G.medium = medium[c];
            G.pooled = cc.pooled;
            G.cls = cc.pooled ? -1 : P.cell_class[c];
            G.nF = cc.nF_layout;
            G.tab_off = cc.pooled ? 0 : cc.offset;
            P.groups.push_back(G);
            members.emplace_back();
        } else {
            g = it->second;
        }
        members[g].push_back(c);
    }
    // within a group, cells in Z (Morton) order of their centroids: the cells of one workgroup
    // are close in space, so the neighbour slots their face contributions are written to fall
    // in few cache lines
    {
        double x0 = P.centroid[0], x1 = x0, y0 = P.centroid[1], y1 = y0;
        for (int c = 0; c < nc; ++c) {
            x0 = std::min(x0, P.centroid[2 * c]), x1 = std::max(x1, P.centroid[2 * c]);
            y0 = std::min(y0, P.centroid[2 * c + 1]), y1 = std::max(y1, P.centroid[2 * c + 1]);
        }
        const double sx = 65535.0 / std::max(x1 - x0, 1e-300), sy = 65535.0 / std::max(y1 - y0, 1e-300);
        auto spread = [](uint32_t v) {  // 16 bits -> even bits of 32
            v &= 0xffffu;
            v = (v | (v << 8)) & 0x00ff00ffu;
            v = (v | (v << 4)) & 0x0f0f0f0fu;
            v = (v | (v << 2)) & 0x33333333u;
            v = (v | (v << 1)) & 0x55555555u;
            return v;
        };
        std::vector<uint32_t> key(nc);
        for (int c = 0; c < nc; ++c) {
            const uint32_t qx = (uint32_t)std::lround((P.centroid[2 * c] - x0) * sx);
            const uint32_t qy = (uint32_t)std::lround((P.centroid[2 * c + 1] - y0) * sy);
            key[c] = spread(qx) | (spread(qy) << 1);
        }
        for (auto &m : members)
            std::stable_sort(m.begin(), m.end(), [&](int a, int b) { return key[a] < key[b]; });
    }
    // launch shapes: 64, 128 and 256 lanes per workgroup (one shape when shots fill a block)
    for (int lanes : {kLanesTarget, 2 * kLanesTarget, kBlock}) {
        const int cpb = std::max(1, lanes / P.S);
        bool dup = false;
        for (const auto &L : P.launches) dup |= L.cpb == cpb;
        if (dup) continue;
        Plan::Launch L;
        L.cpb = cpb;
        L.lanes = cpb * P.S;
        P.launches.push_back(L);
    }
    int cpb_max = 1;
    for (const auto &L : P.launches) cpb_max = std::max(cpb_max, L.cpb);
    int ic = 0;
    P.ic_of_cell.assign(nc, -1);
    for (size_t g = 0; g < P.groups.size(); ++g) {
        Group &G = P.groups[g];
        G.ic_begin = ic;
        G.ncells = (int)members[g].size();
        for (int l = 0; l < G.ncells; ++l) P.ic_of_cell[members[g][l]] = ic + l;
        ic += (G.ncells + cpb_max - 1) / cpb_max * cpb_max;
    }
    P.n_ic = ic;
    for (auto &L : P.launches) {
        int blk = 0;
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const int nblk = (P.groups[g].ncells + L.cpb - 1) / L.cpb;
            L.blk_begin.push_back(blk);
            for (int b = 0; b < nblk; ++b) L.blk_group.push_back((int)g);
            blk += nblk;
        }
    }
    P.cpb = P.launches[0].cpb;
    P.blk_group = P.launches[0].blk_group;
    for (size_t g = 0; g < P.groups.size(); ++g) {
        P.groups[g].blk_begin = P.launches[0].blk_begin[g];
        P.groups[g].nblk = (P.groups[g].ncells + P.cpb - 1) / P.cpb;
    }
    P.cell_of_ic.assign(P.n_ic, -1);
    for (int c = 0; c < nc; ++c) P.cell_of_ic[P.ic_of_cell[c]] = c;
    P.ic_tab.assign(P.n_ic, 0);
    for (int c = 0; c < nc; ++c) P.ic_tab[P.ic_of_cell[c]] = P.classes[P.cell_class[c]].offset;
    for (const auto &G : P.groups) P.has_pooled |= G.pooled;

    // face links, face-solve coefficients and materials (structure of arrays over internal cells)
    const int nic = P.n_ic;
    P.link.assign((size_t)P.max_nf * nic, -1);
    P.c0.assign((size_t)P.max_nf * nic, 0.0);
    P.mat.assign((size_t)kNumMat * nic, 0.0);
    P.emat.assign((size_t)kNumEnergyMat * nic, 0.0);
    P.gm.assign((size_t)kNumGradCoef * nic, 0.0);
    for (int c = 0; c < nc; ++c) {
        const int i = P.ic_of_cell[c], s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        for (int j = 0; j < n; ++j) {
            const int cn = nbr_cell[s + j];
            if (cn < 0) continue;
            const int iface = medium[cn] != medium[c] ? 1 : 0;
            P.link[(size_t)j * nic + i] = (P.ic_of_cell[cn] << 4) | (iface << 3) | nbr_j[s + j];
            if (!iface) {
                P.c0[(size_t)j * nic + i] = 1.0 / (tau[c] + tau[cn]);
            } else {
                const double tf = medium[c] == kFluid ? tau[c] : tau[cn];
                const double ts = medium[c] == kFluid ? tau[cn] : tau[c];
                P.c0[(size_t)j * nic + i] = 1.0 / (tf + 1.0 / ts);
            }
        }
        auto m = [&](int slot) -> double & { return P.mat[(size_t)slot * nic + i]; };
        auto em = [&](int slot) -> double & { return P.emat[(size_t)slot * nic + i]; };
        m(kInvRho) = 1.0 / rho[c];
        m(kTau) = tau[c];
        m(kInvTau) = 1.0 / tau[c];
        em(0) = rho[c];
        auto gd = [&](int slot) -> double & { return P.gm[(size_t)slot * nic + i]; };
        const double t = tau[c];
        if (medium[c] == kFluid) {
            const double kap = rho[c] * pa[c] * pa[c];
            m(kStiff) = kap;
            em(1) = 1.0 / kap;
            // kappa = rho c^2, tau = eta / (rho c)
            gd(0) = -1.0 / (rho[c] * kap);
            gd(1) = -2.0 / (pa[c] * kap);
            gd(2) = -t / rho[c];
            gd(3) = -t / pa[c];
        } else {
            const double lam = pa[c], mu = pb[c], lpm = lam + mu, l2m = lam + 2.0 * mu;
            m(kStiff) = l2m;
            m(kLam) = lam;
            m(kTwoMu) = 2.0 * mu;
            em(1) = l2m / (4.0 * mu * lpm);
            em(2) = -lam / (4.0 * mu * lpm);
            em(3) = 1.0 / (2.0 * mu);
            // tau = eta rho c_P = eta sqrt(rho (lam + 2 mu))  or  eta rho c_S = eta sqrt(rho mu)
            gd(0) = t / (2.0 * rho[c]);
            gd(1) = stab_speed == 0 ? t / (2.0 * l2m) : 0.0;
            gd(2) = stab_speed == 0 ? t / l2m : t / (2.0 * mu);
            gd(3) = -1.0 / (4.0 * lpm * lpm);
            gd(4) = -(lam * lam + 2.0 * lam * mu + 2.0 * mu * mu) / (4.0 * mu * mu * lpm * lpm);
            gd(5) = lam * l2m / (4.0 * mu * mu * lpm * lpm);
            gd(6) = -1.0 / (2.0 * mu * mu);
        }
    }
    P.ext_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) P.ext_off[c + 1] = P.ext_off[c] + (medium[c] == kFluid ? 3 : 5) * N;
    P.n_ext = P.ext_off[nc];
    *code = 0;
    return "";
}

}  // namespace hho
