// Host-side execution plan of the three-dimensional engine (float64): mesh validation for
// tetrahedra, triangular prisms and hexahedra with planar faces, face matching and tagging, per-shape-class local
// operators in orthonormal cell and face bases (Sec. 3.3, eq. rec_a, rec_e, stab in d = 3),
// materials and stabilisation weights, and the grouping of cells by (medium, shape class) into
// the same structure-of-arrays layout as the two-dimensional plan.
//
// Integrals are exact for the polynomial integrands involved: every cell is cut into
// tetrahedra (one per fan triangle of each face, apex at the vertex average; exact for convex
// cells with planar faces) and every face into fan triangles, and each simplex is integrated
// with a Grundmann-Moeller rule (Grundmann and Moeller, SIAM J. Numer. Anal. 15, 1978) of
// degree 2k + 3, above the 2k of the Gram, derivative and face-mass integrands.
//
// Face bases are defined by the face alone, so that the two cells of a face use one basis:
// origin at the face centroid, first tangent from the face's lowest-id vertex to its
// second-lowest-id vertex, normal from the three lowest-id vertices.  A shape class is a cell
// geometry up to translation together with the order of its vertex ids, which fixes every face
// frame relative to the geometry.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "plan.h"

namespace hho {

namespace {

struct V3 {
    double x, y, z;
};
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }

// Local faces, every face a cycle of its vertices: tetrahedron face j opposite vertex j; triangular
// prism with vertices 0-2 around the bottom and 3-5 above them; hexahedron with vertices 0-3 around
// the bottom and 4-7 above them.
const int kTetFace[4][4] = {{1, 2, 3, -1}, {0, 2, 3, -1}, {0, 1, 3, -1}, {0, 1, 2, -1}};
const int kPrismFace[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
const int kHexFace[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};

int n_local_faces(int nv) { return nv == 4 ? 4 : nv == 6 ? 5 : 6; }
const int *local_face_table(int nv, int j) { return nv == 4 ? kTetFace[j] : nv == 6 ? kPrismFace[j] : kHexFace[j]; }
int face_size(int nv, int j) { return local_face_table(nv, j)[3] < 0 ? 3 : 4; }
int face_vertex(int nv, int j, int m) { return local_face_table(nv, j)[m]; }

double factorial(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// Grundmann-Moeller rule on the n-simplex (n = 2 or 3) exact for degree 2s + 1: barycentric
// points (n + 1 per point) and weights scaled to sum to 1 (to be multiplied by the measure).
struct SimplexRule {
    int n = 0;
    std::vector<double> bary, w;
};

void compositions(int total, int parts, std::vector<int> &cur, std::vector<std::vector<int>> &out) {
    if (parts == 1) {
        cur.push_back(total);
        out.push_back(cur);
        cur.pop_back();
        return;
    }
    for (int v = total; v >= 0; --v) {
        cur.push_back(v);
        compositions(total - v, parts - 1, cur, out);
        cur.pop_back();
    }
}

SimplexRule gm_rule(int n, int s) {
    SimplexRule R;
    R.n = n;
    const int d = 2 * s + 1;
    double sum = 0.0;
    for (int i = 0; i <= s; ++i) {
        const double base = d + n - 2 * i;
        double p = 1.0;
        for (int e = 0; e < d; ++e) p *= base;
        const double w = ((i & 1) ? -1.0 : 1.0) * std::ldexp(1.0, -2 * s) * p / (factorial(i) * factorial(d + n - i));
        std::vector<std::vector<int>> betas;
        std::vector<int> cur;
        compositions(s - i, n + 1, cur, betas);
        for (const auto &b : betas) {
            for (int m = 0; m <= n; ++m) R.bary.push_back((2.0 * b[m] + 1.0) / base);
            R.w.push_back(w);
            sum += w;
        }
    }
    for (double &w : R.w) w /= sum;
    return R;
}

// Quadrature points (physical coordinates) and weights.
struct Quad {
    std::vector<V3> x;
    std::vector<double> w;
};

void add_simplex(const SimplexRule &R, const V3 *P, double measure, Quad &q) {
    const int np = (int)R.w.size();
    for (int p = 0; p < np; ++p) {
        V3 x{0, 0, 0};
        for (int m = 0; m <= R.n; ++m) x = x + R.bary[p * (R.n + 1) + m] * P[m];
        q.x.push_back(x);
        q.w.push_back(R.w[p] * measure);
    }
}

// graded monomial exponents in three variables: degree-major; within a degree decreasing power
// of x, then decreasing power of y
void exponents3(int k, std::vector<std::array<int, 3>> &e) {
    e.clear();
    for (int d = 0; d <= k; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b) e.push_back({a, b, d - a - b});
}
// in two variables (face coordinates): degree-major, decreasing power of the first
void exponents2(int k, std::vector<std::array<int, 2>> &e) {
    e.clear();
    for (int d = 0; d <= k; ++d)
        for (int a = d; a >= 0; --a) e.push_back({a, d - a});
}

double powi(double x, int e) {
    double r = 1.0;
    while (e-- > 0) r *= x;
    return r;
}

bool cholesky(int n, const std::vector<double> &A, std::vector<double> &L) {
    L.assign((size_t)n * n, 0.0);
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

void invert_lower(int n, const std::vector<double> &L, std::vector<double> &Li) {
    Li.assign((size_t)n * n, 0.0);
    for (int col = 0; col < n; ++col)
        for (int i = col; i < n; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int m = col; m < i; ++m) s -= L[i * n + m] * Li[m * n + col];
            Li[i * n + col] = s / L[i * n + i];
        }
}

// Coefficients C (lower triangular) of the basis orthonormal in the weighted inner product of
// the monomial values V [q][n]: C = L^{-1} with L L^T the Gram matrix.
bool orthonormal_coefs(int n, const std::vector<double> &V, const std::vector<double> &w, std::vector<double> &C) {
    const int nq = (int)w.size();
    std::vector<double> G((size_t)n * n, 0.0), L;
    for (int q = 0; q < nq; ++q)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b <= a; ++b) G[a * n + b] += w[q] * V[(size_t)q * n + a] * V[(size_t)q * n + b];
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) G[a * n + b] = G[b * n + a];
    if (!cholesky(n, G, L)) return false;
    invert_lower(n, L, C);
    return true;
}

struct Geo3 {
    V3 bary;
    double vol, h;
};

// One face of a cell as a polygon (cycle of input vertex ids).
struct FaceRef {
    int nv;
    int v[4];
};

FaceRef local_face(const int32_t *cv, int nv, int j) {
    FaceRef f;
    f.nv = face_size(nv, j);
    for (int m = 0; m < f.nv; ++m) f.v[m] = cv[face_vertex(nv, j, m)];
    return f;
}

// Face frame: centroid, tangents t1, t2, unit normal (from the lowest ids), diameter.
struct Frame {
    V3 c, t1, t2, n;
    double h, area;
};

Frame face_frame(const std::vector<V3> &X, const FaceRef &f) {
    Frame F;
    int ids[4];
    for (int m = 0; m < f.nv; ++m) ids[m] = f.v[m];
    std::sort(ids, ids + f.nv);
    const V3 a = X[ids[0]], b = X[ids[1]], c = X[ids[2]];
    F.n = cross(b - a, c - a);
    F.n = (1.0 / norm(F.n)) * F.n;
    F.t1 = (1.0 / norm(b - a)) * (b - a);
    F.t2 = cross(F.n, F.t1);
    // centroid and area from the fan triangles of the cycle
    double A = 0.0;
    V3 s{0, 0, 0};
    for (int t = 1; t + 1 < f.nv; ++t) {
        const V3 p0 = X[f.v[0]], p1 = X[f.v[t]], p2 = X[f.v[t + 1]];
        const double at = 0.5 * norm(cross(p1 - p0, p2 - p0));
        A += at;
        s = s + (at / 3.0) * (p0 + p1 + p2);
    }
    F.area = A;
    F.c = (1.0 / A) * s;
    F.h = 0.0;
    for (int m = 0; m < f.nv; ++m)
        for (int l = 0; l < f.nv; ++l) F.h = std::max(F.h, norm(X[f.v[m]] - X[f.v[l]]));
    return F;
}

void face_quad(const SimplexRule &R2, const std::vector<V3> &X, const FaceRef &f, Quad &q) {
    for (int t = 1; t + 1 < f.nv; ++t) {
        const V3 P[3] = {X[f.v[0]], X[f.v[t]], X[f.v[t + 1]]};
        add_simplex(R2, P, 0.5 * norm(cross(P[1] - P[0], P[2] - P[0])), q);
    }
}

void cell_quad(const SimplexRule &R3, const std::vector<V3> &X, const int32_t *cv, int nv, Quad &q) {
    V3 apex{0, 0, 0};
    for (int m = 0; m < nv; ++m) apex = apex + X[cv[m]];
    apex = (1.0 / nv) * apex;
    for (int j = 0; j < n_local_faces(nv); ++j) {
        const FaceRef f = local_face(cv, nv, j);
        for (int t = 1; t + 1 < f.nv; ++t) {
            const V3 P[4] = {apex, X[f.v[0]], X[f.v[t]], X[f.v[t + 1]]};
            const double vol = std::fabs(dot(P[1] - P[0], cross(P[2] - P[0], P[3] - P[0]))) / 6.0;
            add_simplex(R3, P, vol, q);
        }
    }
}

}  // namespace

void eval_basis3(const Plan &P, int c, double x, double y, double z, double *phi) {
    const int N = P.N;
    std::vector<std::array<int, 3>> e;
    exponents3(P.k, e);
    const double h = P.hT[c];
    const double X = (x - P.centroid[3 * c]) / h, Y = (y - P.centroid[3 * c + 1]) / h,
                 Z = (z - P.centroid[3 * c + 2]) / h;
    const double *C = P.basisC.data() + (size_t)P.cell_class[c] * N * N;
    std::vector<double> mu(N);
    for (int m = 0; m < N; ++m) mu[m] = powi(X, e[m][0]) * powi(Y, e[m][1]) * powi(Z, e[m][2]);
    for (int a = 0; a < N; ++a) {
        double s = 0.0;
        for (int m = 0; m <= a; ++m) s += C[(size_t)a * N + m] * mu[m];
        phi[a] = s;
    }
}

int locate_cell3(const Plan &P, double x, double y, double z) {
    std::vector<V3> X(P.n_vertices);
    for (int v = 0; v < P.n_vertices; ++v) X[v] = {P.xyz[3 * v], P.xyz[3 * v + 1], P.xyz[3 * v + 2]};
    const V3 p{x, y, z};
    for (int c = 0; c < P.n_cells; ++c) {
        const int s = P.cell_ptr[c], nv = P.cell_ptr[c + 1] - s;
        const V3 bc{P.centroid[3 * c], P.centroid[3 * c + 1], P.centroid[3 * c + 2]};
        bool inside = true;
        for (int j = 0; j < n_local_faces(nv) && inside; ++j) {
            const FaceRef f = local_face(P.cell_vtx.data() + s, nv, j);
            V3 n = cross(X[f.v[1]] - X[f.v[0]], X[f.v[2]] - X[f.v[0]]);
            n = (1.0 / norm(n)) * n;
            if (dot(n, X[f.v[0]] - bc) < 0.0) n = -1.0 * n;
            if (dot(n, p - X[f.v[0]]) > 1e-12 * P.hT[c]) inside = false;
        }
        if (inside) return c;
    }
    return -1;
}

std::string build_plan3d(int nv, const double *xyz, int nc, const int32_t *cell_ptr, const int32_t *cell_vtx,
                         const uint8_t *medium, const double *rho, const double *pa, const double *pb, int k,
                         double eta_f, double eta_s, int stab_speed, int n_shots, Plan &P, int *code) {
    *code = 1;  // HHO_ERR_ARG
    if (k < 1 || k > 2) return "k must be 1 or 2 in three dimensions (a solid cell of degree 3 carries 180 unknowns)";
    if (nv <= 0 || nc <= 0 || !xyz || !cell_ptr || !cell_vtx || !medium || !rho || !pa || !pb)
        return "empty mesh or null mesh array";
    if (n_shots < 1 || n_shots > kBlock) return "n_shots must be in 1..256";
    if (!(eta_f > 0.0) || !(eta_s > 0.0)) return "eta_f and eta_s must be positive";
    if (stab_speed != 0 && stab_speed != 1) return "stab_speed must be 0 (P-wave) or 1 (S-wave)";
    P = Plan();
    P.dim = 3;
    P.tcomp = 3;
    P.rows_f = 4;
    P.rows_s = 9;
    P.k = k;
    P.N = (k + 1) * (k + 2) * (k + 3) / 6;
    P.F = (k + 1) * (k + 2) / 2;
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
        if (n != 4 && n != 6 && n != 8)
            return "cell " + std::to_string(c) + " has " + std::to_string(n) +
                   " vertices (4: tetrahedron, 6: triangular prism, 8: hexahedron)";
        P.max_nf = std::max(P.max_nf, n_local_faces(n));
    }
    const int ne = cell_ptr[nc];
    for (int e = 0; e < ne; ++e)
        if (cell_vtx[e] < 0 || cell_vtx[e] >= nv) return "vertex id out of range";
    for (int c = 0; c < nc; ++c)
        for (int m = cell_ptr[c]; m < cell_ptr[c + 1]; ++m)
            for (int l = m + 1; l < cell_ptr[c + 1]; ++l)
                if (cell_vtx[m] == cell_vtx[l]) return "repeated vertex in cell " + std::to_string(c);
    P.xyz.assign(xyz, xyz + 3 * (size_t)nv);
    P.cell_ptr.assign(cell_ptr, cell_ptr + nc + 1);
    P.cell_vtx.assign(cell_vtx, cell_vtx + ne);
    P.medium.assign(medium, medium + nc);
    std::vector<V3> X(nv);
    for (int v = 0; v < nv; ++v) X[v] = {xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]};

    *code = 1;
    for (int c = 0; c < nc; ++c) {
        if (medium[c] > 1) return "medium must be 0 (fluid) or 1 (solid)";
        if (!(rho[c] > 0.0)) return "rho must be positive";
        if (medium[c] == kFluid && !(pa[c] > 0.0)) return "fluid sound speed must be positive";
        if (medium[c] == kSolid && (!(pb[c] > 0.0) || !(3.0 * pa[c] + 2.0 * pb[c] > 0.0)))
            return "solid needs mu > 0 and 3 lambda + 2 mu > 0";
    }

    // geometry: volume, barycentre, diameter; planar faces and convexity
    *code = 2;
    const SimplexRule R3 = gm_rule(3, k + 1), R2 = gm_rule(2, k + 1);
    std::vector<Geo3> geo(nc);
    P.centroid.resize(3 * (size_t)nc);
    P.hT.resize(nc);
    P.area.resize(nc);
    double hsum = 0.0;
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        const int32_t *cv = cell_vtx + s;
        double h = 0.0;
        for (int m = 0; m < n; ++m)
            for (int l = 0; l < n; ++l) h = std::max(h, norm(X[cv[m]] - X[cv[l]]));
        V3 avg{0, 0, 0};
        for (int m = 0; m < n; ++m) avg = avg + X[cv[m]];
        avg = (1.0 / n) * avg;
        for (int j = 0; j < n_local_faces(n); ++j) {
            const FaceRef f = local_face(cv, n, j);
            V3 nn = cross(X[f.v[1]] - X[f.v[0]], X[f.v[2]] - X[f.v[0]]);
            const double ln = norm(nn);
            if (!(ln > 1e-14 * h * h)) return "cell " + std::to_string(c) + " has a degenerate face";
            nn = (1.0 / ln) * nn;
            if (f.nv == 4 && std::fabs(dot(nn, X[f.v[3]] - X[f.v[0]])) > 1e-10 * h)
                return "cell " + std::to_string(c) + " has a non-planar face";
            const double side = dot(nn, avg - X[f.v[0]]);
            for (int m = 0; m < n; ++m) {
                const double sm = dot(nn, X[cv[m]] - X[f.v[0]]);
                if (sm * side < 0.0 && std::fabs(sm) > 1e-10 * h)
                    return "cell " + std::to_string(c) + " is not convex or its vertices are out of order";
            }
            if (std::fabs(side) < 1e-10 * h) return "cell " + std::to_string(c) + " is degenerate";
        }
        Quad q;
        cell_quad(R3, X, cv, n, q);
        double vol = 0.0;
        V3 b{0, 0, 0};
        for (size_t p = 0; p < q.w.size(); ++p) {
            vol += q.w[p];
            b = b + q.w[p] * q.x[p];
        }
        if (!(vol > 0.0)) return "cell " + std::to_string(c) + " has no volume";
        geo[c] = {(1.0 / vol) * b, vol, h};
        P.centroid[3 * c] = geo[c].bary.x;
        P.centroid[3 * c + 1] = geo[c].bary.y;
        P.centroid[3 * c + 2] = geo[c].bary.z;
        P.hT[c] = h;
        P.area[c] = vol;
        hsum += h;
    }

    // faces: matched by their sorted vertex ids, at most two cells per face
    std::vector<int> nbr_cell((size_t)nc * 6, -1), nbr_j((size_t)nc * 6, -1);
    {
        std::map<std::array<int, 4>, std::pair<int, int>> first;
        int nfaces = 0;
        for (int c = 0; c < nc; ++c) {
            const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
            for (int j = 0; j < n_local_faces(n); ++j) {
                const FaceRef f = local_face(cell_vtx + s, n, j);
                std::array<int, 4> key{-1, -1, -1, -1};
                for (int m = 0; m < f.nv; ++m) key[m] = f.v[m];
                std::sort(key.begin(), key.begin() + f.nv);
                auto it = first.find(key);
                if (it == first.end()) {
                    first.emplace(key, std::make_pair(c, j));
                    ++nfaces;
                    continue;
                }
                const int c0 = it->second.first, j0 = it->second.second;
                if (c0 < 0) return "face shared by more than two cells";
                nbr_cell[(size_t)c0 * 6 + j0] = c;
                nbr_j[(size_t)c0 * 6 + j0] = j;
                nbr_cell[(size_t)c * 6 + j] = c0;
                nbr_j[(size_t)c * 6 + j] = j0;
                it->second.first = -1;
            }
        }
        P.n_faces = nfaces;
    }

    // shape classes: vertex offsets from the first vertex, and the order of the vertex ids
    const double quantum = 1e-9 * hsum / nc;
    std::map<std::vector<int64_t>, int> class_of_key;
    P.cell_class.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const int s = cell_ptr[c], n = cell_ptr[c + 1] - s;
        std::vector<int64_t> key;
        key.push_back(n);
        const V3 o = X[cell_vtx[s]];
        for (int j = 1; j < n; ++j) {
            const V3 d = X[cell_vtx[s + j]] - o;
            key.push_back(std::llround(d.x / quantum));
            key.push_back(std::llround(d.y / quantum));
            key.push_back(std::llround(d.z / quantum));
        }
        for (int j = 0; j < n; ++j) {
            int rank = 0;
            for (int l = 0; l < n; ++l) rank += cell_vtx[s + l] < cell_vtx[s + j];
            key.push_back(rank);
        }
        auto it = class_of_key.find(key);
        if (it == class_of_key.end()) {
            const int id = (int)P.classes.size();
            class_of_key.emplace(std::move(key), id);
            ClassInfo ci;
            ci.nF = n_local_faces(n);
            ci.rep_cell = c;
            P.classes.push_back(ci);
            P.cell_class[c] = id;
        } else {
            P.cell_class[c] = it->second;
        }
    }
    for (int c = 0; c < nc; ++c) P.classes[P.cell_class[c]].ncells += 1;
    const bool pool = (int)P.classes.size() > kPoolMinClasses;
    for (auto &ci : P.classes) {
        ci.pooled = pool && ci.ncells < kPoolCells;
        ci.nF_layout = ci.nF;  // pooled groups are bucketed by face count (4 or 6)
    }

    // per-class tables: Bx, By, Bz, S (N x N), G_j (N x F), n_j (3)
    *code = 3;  // HHO_ERR_SINGULAR
    std::vector<std::array<int, 3>> ec;
    std::vector<std::array<int, 2>> ef;
    exponents3(k, ec);
    exponents2(k, ef);
    const int degc[20] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3};
    const int degf[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
    P.basisC.assign(P.classes.size() * (size_t)N * N, 0.0);
    for (size_t cl = 0; cl < P.classes.size(); ++cl) {
        ClassInfo &ci = P.classes[cl];
        const int c = ci.rep_cell, s = cell_ptr[c], n = cell_ptr[c + 1] - s, nF = ci.nF;
        const int32_t *cv = cell_vtx + s;
        const double h = geo[c].h;
        const V3 bc = geo[c].bary;
        auto mono = [&](V3 x, double *v, double *dx, double *dy, double *dz) {
            const V3 y = (1.0 / h) * (x - bc);
            for (int m = 0; m < N; ++m) {
                const int a = ec[m][0], b = ec[m][1], e = ec[m][2];
                v[m] = powi(y.x, a) * powi(y.y, b) * powi(y.z, e);
                if (dx) {
                    dx[m] = a ? a * powi(y.x, a - 1) * powi(y.y, b) * powi(y.z, e) / h : 0.0;
                    dy[m] = b ? b * powi(y.x, a) * powi(y.y, b - 1) * powi(y.z, e) / h : 0.0;
                    dz[m] = e ? e * powi(y.x, a) * powi(y.y, b) * powi(y.z, e - 1) / h : 0.0;
                }
            }
        };
        Quad q;
        cell_quad(R3, X, cv, n, q);
        const int nq = (int)q.w.size();
        std::vector<double> V((size_t)nq * N), Dx((size_t)nq * N), Dy((size_t)nq * N), Dz((size_t)nq * N), C;
        for (int p = 0; p < nq; ++p) mono(q.x[p], &V[(size_t)p * N], &Dx[(size_t)p * N], &Dy[(size_t)p * N], &Dz[(size_t)p * N]);
        if (!orthonormal_coefs(N, V, q.w, C))
            return "Gram matrix of cell " + std::to_string(c) + " is not positive definite";
        std::copy(C.begin(), C.end(), P.basisC.begin() + cl * (size_t)N * N);
        // basis values and derivatives at the points: phi = C mu
        auto apply = [&](const double *mu, double *out) {
            for (int a = 0; a < N; ++a) {
                double v = 0.0;
                for (int m = 0; m <= a; ++m) v += C[(size_t)a * N + m] * mu[m];
                out[a] = v;
            }
        };
        std::vector<double> B[3], Ssum((size_t)N * N, 0.0);
        for (int d = 0; d < 3; ++d) B[d].assign((size_t)N * N, 0.0);
        {
            std::vector<double> phi(N), g(N);
            for (int p = 0; p < nq; ++p) {
                apply(&V[(size_t)p * N], phi.data());
                const std::vector<double> *Dm[3] = {&Dx, &Dy, &Dz};
                for (int d = 0; d < 3; ++d) {
                    apply(&(*Dm[d])[(size_t)p * N], g.data());
                    // D_d[a][b] = (d_d phi_b, phi_a)_T
                    for (int a = 0; a < N; ++a)
                        for (int b = 0; b < N; ++b) B[d][(size_t)a * N + b] += q.w[p] * phi[a] * g[b];
                }
            }
        }
        std::vector<double> G((size_t)nF * N * F, 0.0), nrm(3 * (size_t)nF, 0.0);
        for (int j = 0; j < nF; ++j) {
            const FaceRef f = local_face(cv, n, j);
            const Frame fr = face_frame(X, f);
            V3 nout = fr.n;
            if (dot(nout, fr.c - bc) < 0.0) nout = -1.0 * nout;
            nrm[3 * j] = nout.x;
            nrm[3 * j + 1] = nout.y;
            nrm[3 * j + 2] = nout.z;
            Quad fq;
            face_quad(R2, X, f, fq);
            const int nfq = (int)fq.w.size();
            std::vector<double> Vf((size_t)nfq * F), Cf;
            for (int p = 0; p < nfq; ++p) {
                const V3 y = fq.x[p] - fr.c;
                const double sx = dot(y, fr.t1) / fr.h, ty = dot(y, fr.t2) / fr.h;
                for (int i = 0; i < F; ++i) Vf[(size_t)p * F + i] = powi(sx, ef[i][0]) * powi(ty, ef[i][1]);
            }
            if (!orthonormal_coefs(F, Vf, fq.w, Cf))
                return "face Gram matrix of cell " + std::to_string(c) + " is not positive definite";
            std::vector<double> mu(N), phi(N), psi(F);
            for (int p = 0; p < nfq; ++p) {
                mono(fq.x[p], mu.data(), nullptr, nullptr, nullptr);
                apply(mu.data(), phi.data());
                for (int i = 0; i < F; ++i) {
                    double v = 0.0;
                    for (int m = 0; m <= i; ++m) v += Cf[(size_t)i * F + m] * Vf[(size_t)p * F + m];
                    psi[i] = v;
                }
                const double w = fq.w[p];
                for (int a = 0; a < N; ++a) {
                    for (int b = 0; b < N; ++b) {
                        const double e = w * phi[a] * phi[b];  // E_j[a][b] = (phi_b, phi_a)_F
                        Ssum[(size_t)a * N + b] += e;
                        B[0][(size_t)a * N + b] -= nout.x * e;
                        B[1][(size_t)a * N + b] -= nout.y * e;
                        B[2][(size_t)a * N + b] -= nout.z * e;
                    }
                    for (int i = 0; i < F; ++i) G[((size_t)j * N + a) * F + i] += w * phi[a] * psi[i];
                }
            }
        }
        // degree structure: B_d[r][b] = 0 unless deg(b) < deg(r); G_j[a][i] = 0 unless
        // deg(psi_i) <= deg(phi_a) (planar faces); checked as round-off, then stored as exact zeros
        double bmax = 0.0, zmax = 0.0, gmax = 0.0, gzero = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int r = 0; r < N; ++r)
                for (int b = 0; b < N; ++b) {
                    double &v = B[d][(size_t)r * N + b];
                    bmax = std::max(bmax, std::fabs(v));
                    if (degc[b] >= degc[r]) {
                        zmax = std::max(zmax, std::fabs(v));
                        v = 0.0;
                    }
                }
        for (int j = 0; j < nF; ++j)
            for (int a = 0; a < N; ++a)
                for (int i = 0; i < F; ++i) {
                    double &g = G[((size_t)j * N + a) * F + i];
                    gmax = std::max(gmax, std::fabs(g));
                    if (degf[i] > degc[a]) {
                        gzero = std::max(gzero, std::fabs(g));
                        g = 0.0;
                    }
                }
        if (zmax > 1e-9 * bmax || gzero > 1e-9 * gmax)
            return "cell " + std::to_string(c) + ": local operators lost their degree structure "
                   "(ill-conditioned basis)";
        ci.offset = (int)P.tables.size();
        if (!ci.pooled) {
            for (int d = 0; d < 3; ++d) P.tables.insert(P.tables.end(), B[d].begin(), B[d].end());
            P.tables.insert(P.tables.end(), Ssum.begin(), Ssum.end());
            P.tables.insert(P.tables.end(), G.begin(), G.end());
        } else {
            // packed (read per lane): the structurally nonzero entries of B_x, B_y, B_z, the upper
            // triangle of the symmetric S, the structurally nonzero entries of every G_j, the normals
            for (int d = 0; d < 3; ++d)
                for (int r = 0; r < N; ++r)
                    for (int b = 0; b < N; ++b)
                        if (degc[b] < degc[r]) P.tables.push_back(B[d][(size_t)r * N + b]);
            for (int r = 0; r < N; ++r)
                for (int b = r; b < N; ++b) P.tables.push_back(Ssum[(size_t)r * N + b]);
            for (int j = 0; j < nF; ++j)
                for (int a = 0; a < N; ++a)
                    for (int i = 0; i < F; ++i)
                        if (degf[i] <= degc[a]) P.tables.push_back(G[((size_t)j * N + a) * F + i]);
        }
        P.tables.insert(P.tables.end(), nrm.begin(), nrm.end());
    }

    // stabilisation weights eta tau_T
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

    // groups (medium, class), pooled groups by (medium, face count)
    std::map<std::pair<int, int>, int> gid;
    std::vector<std::vector<int>> members;
    for (int c = 0; c < nc; ++c) {
        const ClassInfo &cc = P.classes[P.cell_class[c]];
        auto key = cc.pooled ? std::make_pair((int)medium[c], -1 - cc.nF) : std::make_pair((int)medium[c], P.cell_class[c]);
        auto it = gid.find(key);
        int g;
        if (it == gid.end()) {
            g = (int)P.groups.size();
            gid.emplace(key, g);
            Group Gr;
            Gr.medium = medium[c];
            Gr.pooled = cc.pooled;
            Gr.cls = cc.pooled ? -1 : P.cell_class[c];
            Gr.nF = cc.nF;
            Gr.tab_off = cc.pooled ? 0 : cc.offset;
            P.groups.push_back(Gr);
            members.emplace_back();
        } else {
            g = it->second;
        }
        members[g].push_back(c);
    }
    // cells of a group in Morton order of their barycentres (10 bits per axis)
    {
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = P.centroid[d];
        for (int c = 0; c < nc; ++c)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], P.centroid[3 * c + d]);
                hi[d] = std::max(hi[d], P.centroid[3 * c + d]);
            }
        auto spread3 = [](uint32_t v) {  // 10 bits -> every third bit of 30
            v &= 0x3ffu;
            v = (v | (v << 16)) & 0x030000ffu;
            v = (v | (v << 8)) & 0x0300f00fu;
            v = (v | (v << 4)) & 0x030c30c3u;
            v = (v | (v << 2)) & 0x09249249u;
            return v;
        };
        std::vector<uint32_t> key(nc);
        for (int c = 0; c < nc; ++c) {
            uint32_t kk = 0;
            for (int d = 0; d < 3; ++d) {
                const double sc = 1023.0 / std::max(hi[d] - lo[d], 1e-300);
                kk |= spread3((uint32_t)std::lround((P.centroid[3 * c + d] - lo[d]) * sc)) << d;
            }
            key[c] = kk;
        }
        for (auto &m : members) std::stable_sort(m.begin(), m.end(), [&](int a, int b) { return key[a] < key[b]; });
    }
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
        Group &Gr = P.groups[g];
        Gr.ic_begin = ic;
        Gr.ncells = (int)members[g].size();
        for (int l = 0; l < Gr.ncells; ++l) P.ic_of_cell[members[g][l]] = ic + l;
        ic += (Gr.ncells + cpb_max - 1) / cpb_max * cpb_max;
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
    for (const auto &Gr : P.groups) P.has_pooled |= Gr.pooled;

    // links, face-solve coefficients, materials, energy weights
    const int nic = P.n_ic;
    P.link.assign((size_t)P.max_nf * nic, -1);
    P.c0.assign((size_t)P.max_nf * nic, 0.0);
    P.mat.assign((size_t)kNumMat * nic, 0.0);
    P.emat.assign((size_t)kNumEnergyMat * nic, 0.0);
    P.gm.assign((size_t)kNumGradCoef * nic, 0.0);
    for (int c = 0; c < nc; ++c) {
        const int i = P.ic_of_cell[c], n = cell_ptr[c + 1] - cell_ptr[c];
        for (int j = 0; j < n_local_faces(n); ++j) {
            const int cn = nbr_cell[(size_t)c * 6 + j];
            if (cn < 0) continue;
            const int iface = medium[cn] != medium[c] ? 1 : 0;
            P.link[(size_t)j * nic + i] = (P.ic_of_cell[cn] << 4) | (iface << 3) | nbr_j[(size_t)c * 6 + j];
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
        if (medium[c] == kFluid) {
            const double kap = rho[c] * pa[c] * pa[c];
            m(kStiff) = kap;
            em(1) = 1.0 / kap;
        } else {
            // stiffness 2 mu I + lambda 1 1^T on the diagonal tensor components, 2 mu on the
            // off-diagonal ones; compliance (I - t 1 1^T) / (2 mu), t = lambda / (3 lambda + 2 mu)
            const double lam = pa[c], mu = pb[c], t = lam / (3.0 * lam + 2.0 * mu);
            m(kStiff) = lam + 2.0 * mu;
            m(kLam) = lam;
            m(kTwoMu) = 2.0 * mu;
            em(1) = (1.0 - t) / (2.0 * mu);
            em(2) = -t / (2.0 * mu);
            em(3) = 1.0 / (2.0 * mu);
        }
    }
    P.ext_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) P.ext_off[c + 1] = P.ext_off[c] + (medium[c] == kFluid ? P.rows_f : P.rows_s) * N;
    P.n_ext = P.ext_off[nc];
    *code = 0;
    return "";
}

}  // namespace hho
