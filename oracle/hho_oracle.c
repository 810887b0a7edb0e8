/*
 * FP64 CPU oracle for the HHO elasto-acoustic semi-discretisation advanced by
 * explicit Runge-Kutta with the face unknowns condensed out.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the HIP
 * path: its own quadrature (Gauss-Legendre + Duffy-collapsed triangle fans), its
 * own bases (Cholesky orthonormalisation of graded monomials, evaluated at
 * quadrature points), its own general LU solves for the mass and face blocks.
 *
 * What it computes (paper references are to arXiv 2505.15771):
 *   - Model: acoustic (p, m) eq. continuous_acoustic, elastic (v, s)
 *     eq. continuous_elastic_eq, coupling eq. continuous_coupling imposed weakly
 *     as in eq. weak_form_acoustic_eq / weak_form_elastic_eq (Sec. 2.2).
 *   - HHO space semi-discretisation eq. HHO1 / HHO2 (Sec. 3.3) with the
 *     gradient and symmetric-gradient reconstructions eq. rec_a / rec_e, the
 *     plain least-squares stabilisation eq. stab with alpha = 0 (equal order),
 *     weights eta^f, eta^s (Sec. 5.1) and the face-local coupling block.
 *     Signs follow the weak form (the printed block matrix eq. algebraic_system
 *     flips the sign of the dual variables; the primal dynamics are identical).
 *   - Face condensation and cell update, eq. ex_solve (Sec. 4.2):
 *     K_F U_F = -K_FT U_T, then M dU_T/dt = F_T - K_T U_T - K_TF U_F.
 *   - ERK(s) Butcher tableaux of eq. ERK (s = 2, 3, 4).
 *   - Energy of Sec. 5.1 (cell unknowns only).
 *   - Point sources: load vectors (eq. rhs) of a point force with a Ricker time factor; the
 *     time factor is parity unpinned (no values in the paper for a time-domain wavelet).
 * Bases (Sec. 3.3 "local modal basis composed of monomials centred at the
 * barycentre"): graded monomials ((x-xT)/hT)^a ((y-yT)/hT)^b, degree-major and,
 * within a degree, decreasing power of x, orthonormalised in L2(T) by the
 * Cholesky factor of their Gram matrix (positive leading coefficients).  Face
 * basis: powers of the face coordinate running from the lower to the higher
 * global vertex id, orthonormalised in L2(F).  Symmetric tensors use
 * E1 = e1(x)e1, E2 = e2(x)e2, E3 = (e1(x)e2 + e2(x)e1)/sqrt(2).
 *
 * Cell unknown layout: fluid [p | m_x | m_y], solid [v_x | v_y | s_1 | s_2 | s_3],
 * each block N = (k+1)(k+2)/2 coefficients; cells concatenated in input order.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define FLUID 0
#define SOLID 1
enum { T_INT_F = 0, T_INT_S = 1, T_GAMMA = 2, T_BND_F = 3, T_BND_S = 4 };

typedef struct {
    int k, N, nf;
    int nv, nc, nfc;
    double *xy;
    int *cptr, *cvtx;
    unsigned char *med;
    double *rho, *pa, *pb;
    double eta_f, eta_s;
    int stab_speed;
    /* faces */
    int *fv;   /* [nfc][2] vertex ids, fv[0] < fv[1] */
    int *fc;   /* [nfc][2] adjacent cells (second = -1 on the boundary) */
    int *fj;   /* [nfc][2] local edge index in each adjacent cell */
    int *ftag; /* [nfc] */
    int *cf;   /* [cptr[nc]] face id of each local edge */
    double *flen, *fmid, *ftan; /* [nfc], [nfc][2], [nfc][2] */
    double *fC;                 /* [nfc][nf][nf] face basis coefficients */
    double *MF;                 /* [nfc][nf][nf] face mass */
    /* cells */
    double *area, *bary, *hT;
    double *C;   /* [nc][N][N] phi_a = sum_b C[a][b] mono_b */
    double *M0;  /* [nc][N][N] */
    double *L0;  /* [nc][N][N] Cholesky factor of M0 */
    double *D;   /* [nc][2][N][N] D_c[a][b] = (d_c phi_b, phi_a)_T */
    double *E;   /* [cptr[nc]][N][N] (phi_b, phi_a)_F */
    double *G;   /* [cptr[nc]][N][nf] (psi_i, phi_a)_F, face basis of the face */
    double *nrm; /* [cptr[nc]][2] outward unit normal */
    double *tau; /* [nc] eta * tau_T */
    double *Cinv;    /* [nc][3][3] compliance in the E-basis (solid) */
    double *Cinv_iv; /* [nc][3][3] inverse of Cinv (solid) */
    int *off;    /* [nc+1] dof offsets */
    int *foff;   /* [nfc+1] face unknown offsets */
    /* loads */
    int nsrc;
    int *src_cell;
    double *src_phi; /* [nsrc][N] */
    double *src_par; /* [nsrc][5]: dir_x, dir_y, f0, t0, amp */
    int nterm;
    double *dload;   /* [nterm][ndof] */
    double *domega, *dphase;
    /* workspace */
    double *UF;
    /* explicit local blocks of the weak form (built on demand for the adjoint) */
    double *KT, *KTF, *KF, *KFT;
    size_t *kt_off, *ktf_off, *kf_off, *kft_off;
} orc_t;

/* ---------------------------------------------------------------- small dense algebra */

/* Solve A x = b in place (b overwritten by x), A n x n row-major overwritten; partial pivoting. */
static int lu_solve(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > best) { best = fabs(A[r * n + c]); p = r; }
        if (best == 0.0) return -1;
        if (p != c) {
            for (int j = 0; j < n; ++j) { double t = A[c * n + j]; A[c * n + j] = A[p * n + j]; A[p * n + j] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* Cholesky A = L L^T (lower), returns -1 if not SPD. */
static int cholesky(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int m = 0; m < j; ++m) s -= L[i * n + m] * L[j * n + m];
            if (i == j) {
                if (s <= 0.0) return -1;
                L[i * n + i] = sqrt(s);
            } else
                L[i * n + j] = s / L[j * n + j];
        }
    return 0;
}

/* Inverse of a lower-triangular matrix. */
static void lower_inverse(int n, const double *L, double *Li)
{
    memset(Li, 0, sizeof(double) * n * n);
    for (int c = 0; c < n; ++c) {
        Li[c * n + c] = 1.0 / L[c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double s = 0.0;
            for (int m = c; m < r; ++m) s += L[r * n + m] * Li[m * n + c];
            Li[r * n + c] = -s / L[r * n + r];
        }
    }
}

/* Solve (L L^T) x = b with a Cholesky factor. */
static void chol_solve(int n, const double *L, double *b)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int m = 0; m < i; ++m) s -= L[i * n + m] * b[m];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int m = i + 1; m < n; ++m) s -= L[m * n + i] * b[m];
        b[i] = s / L[i * n + i];
    }
}

/* ---------------------------------------------------------------- quadrature */

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) { double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m; p0 = p1; p1 = p2; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) { double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m; p0 = p1; p1 = p2; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Quadrature on a polygon: fan of triangles (xT, v_i, v_{i+1}), each mapped
 * from the unit square by the Duffy collapse x = A + u(B-A) + uv(C-B). */
static int cell_quad(const orc_t *o, int c, int n, double *px, double *py, double *pw)
{
    double gx[32], gw[32];
    gauss_legendre(n, gx, gw);
    int s = o->cptr[c], m = o->cptr[c + 1] - s, q = 0;
    double Ax = o->bary[2 * c], Ay = o->bary[2 * c + 1];
    for (int t = 0; t < m; ++t) {
        int i0 = o->cvtx[s + t], i1 = o->cvtx[s + (t + 1) % m];
        double Bx = o->xy[2 * i0], By = o->xy[2 * i0 + 1], Cx = o->xy[2 * i1], Cy = o->xy[2 * i1 + 1];
        double det = fabs((Bx - Ax) * (Cy - By) - (By - Ay) * (Cx - Bx));
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double u = 0.5 * (1 + gx[a]), v = 0.5 * (1 + gx[b]);
                px[q] = Ax + u * (Bx - Ax) + u * v * (Cx - Bx);
                py[q] = Ay + u * (By - Ay) + u * v * (Cy - By);
                pw[q] = 0.25 * gw[a] * gw[b] * u * det;
                ++q;
            }
    }
    return q;
}

/* Gauss points on face f (ordered along its global tangent). */
static int face_quad(const orc_t *o, int f, int n, double *px, double *py, double *pw)
{
    double gx[32], gw[32];
    gauss_legendre(n, gx, gw);
    int a = o->fv[2 * f], b = o->fv[2 * f + 1];
    double L = o->flen[f];
    for (int q = 0; q < n; ++q) {
        double t = 0.5 * (1 + gx[q]);
        px[q] = o->xy[2 * a] + t * (o->xy[2 * b] - o->xy[2 * a]);
        py[q] = o->xy[2 * a + 1] + t * (o->xy[2 * b + 1] - o->xy[2 * a + 1]);
        pw[q] = 0.5 * gw[q] * L;
    }
    return n;
}

/* ---------------------------------------------------------------- bases */

static void mono_exps(int k, int *ea, int *eb)
{
    int m = 0;
    for (int d = 0; d <= k; ++d)
        for (int a = d; a >= 0; --a) { ea[m] = a; eb[m] = d - a; ++m; }
}

static double ipow(double x, int e) { double r = 1.0; for (int i = 0; i < e; ++i) r *= x; return r; }

/* monomial values and gradients at (x, y) for cell c */
static void mono_eval(const orc_t *o, int c, double x, double y, double *mu, double *mux, double *muy)
{
    int ea[64], eb[64];
    mono_exps(o->k, ea, eb);
    double h = o->hT[c], X = (x - o->bary[2 * c]) / h, Y = (y - o->bary[2 * c + 1]) / h;
    for (int m = 0; m < o->N; ++m) {
        mu[m] = ipow(X, ea[m]) * ipow(Y, eb[m]);
        if (mux) mux[m] = ea[m] ? ea[m] * ipow(X, ea[m] - 1) * ipow(Y, eb[m]) / h : 0.0;
        if (muy) muy[m] = eb[m] ? eb[m] * ipow(X, ea[m]) * ipow(Y, eb[m] - 1) / h : 0.0;
    }
}

/* orthonormal cell basis (and gradient) at (x, y) */
static void basis_eval(const orc_t *o, int c, double x, double y, double *phi, double *phx, double *phy)
{
    double mu[64], mux[64], muy[64];
    mono_eval(o, c, x, y, mu, mux, muy);
    const double *C = o->C + (size_t)c * o->N * o->N;
    for (int a = 0; a < o->N; ++a) {
        double s = 0, sx = 0, sy = 0;
        for (int b = 0; b <= a; ++b) { s += C[a * o->N + b] * mu[b]; sx += C[a * o->N + b] * mux[b]; sy += C[a * o->N + b] * muy[b]; }
        phi[a] = s;
        if (phx) phx[a] = sx;
        if (phy) phy[a] = sy;
    }
}

/* orthonormal face basis at (x, y) on face f */
static void face_basis_eval(const orc_t *o, int f, double x, double y, double *psi)
{
    double xi = 2.0 * ((x - o->fmid[2 * f]) * o->ftan[2 * f] + (y - o->fmid[2 * f + 1]) * o->ftan[2 * f + 1]) / o->flen[f];
    const double *C = o->fC + (size_t)f * o->nf * o->nf;
    for (int i = 0; i < o->nf; ++i) {
        double s = 0;
        for (int m = 0; m <= i; ++m) s += C[i * o->nf + m] * ipow(xi, m);
        psi[i] = s;
    }
}

/* symmetric tensor basis E_alpha, entries (E_alpha)_{cd} */
static double Eten(int al, int c, int d)
{
    const double r = 1.0 / sqrt(2.0);
    if (al == 0) return (c == 0 && d == 0) ? 1.0 : 0.0;
    if (al == 1) return (c == 1 && d == 1) ? 1.0 : 0.0;
    return (c != d) ? r : 0.0;
}

/* ---------------------------------------------------------------- setup */

static int cmp_edge(const void *a, const void *b)
{
    const long long *x = a, *y = b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

void orc_destroy(orc_t *o);

orc_t *orc_create(int nv, const double *xy, int nc, const int *cptr, const int *cvtx,
                  const unsigned char *med, const double *rho, const double *pa, const double *pb,
                  int k, double eta_f, double eta_s, int stab_speed)
{
    if (k < 1 || k > 5 || nc <= 0) return NULL;
    orc_t *o = calloc(1, sizeof(orc_t));
    o->k = k; o->N = (k + 1) * (k + 2) / 2; o->nf = k + 1;
    o->nv = nv; o->nc = nc;
    o->eta_f = eta_f; o->eta_s = eta_s; o->stab_speed = stab_speed;
    int N = o->N, nf = o->nf, ne = cptr[nc];
    o->xy = malloc(sizeof(double) * 2 * nv); memcpy(o->xy, xy, sizeof(double) * 2 * nv);
    o->cptr = malloc(sizeof(int) * (nc + 1)); memcpy(o->cptr, cptr, sizeof(int) * (nc + 1));
    o->cvtx = malloc(sizeof(int) * ne); memcpy(o->cvtx, cvtx, sizeof(int) * ne);
    o->med = malloc(nc); memcpy(o->med, med, nc);
    o->rho = malloc(sizeof(double) * nc); memcpy(o->rho, rho, sizeof(double) * nc);
    o->pa = malloc(sizeof(double) * nc); memcpy(o->pa, pa, sizeof(double) * nc);
    o->pb = malloc(sizeof(double) * nc); memcpy(o->pb, pb, sizeof(double) * nc);

    /* faces: sort the (min, max, cell, local) edge records and pair equal keys */
    long long *rec = malloc(sizeof(long long) * 2 * ne);
    for (int c = 0; c < nc; ++c) {
        int s = cptr[c], m = cptr[c + 1] - s;
        for (int t = 0; t < m; ++t) {
            long long a = cvtx[s + t], b = cvtx[s + (t + 1) % m];
            long long lo = a < b ? a : b, hi = a < b ? b : a;
            rec[2 * (s + t)] = lo * (long long)nv + hi;
            rec[2 * (s + t) + 1] = s + t;
        }
    }
    qsort(rec, ne, 2 * sizeof(long long), cmp_edge);
    o->cf = malloc(sizeof(int) * ne);
    int *cell_of = malloc(sizeof(int) * ne);
    for (int c = 0; c < nc; ++c) for (int e = cptr[c]; e < cptr[c + 1]; ++e) cell_of[e] = c;
    o->fv = malloc(sizeof(int) * 2 * ne); o->fc = malloc(sizeof(int) * 2 * ne);
    o->fj = malloc(sizeof(int) * 2 * ne); o->ftag = malloc(sizeof(int) * ne);
    int nfc = 0;
    for (int i = 0; i < ne;) {
        int j = i + 1;
        while (j < ne && rec[2 * j] == rec[2 * i]) ++j;
        if (j - i > 2) { fprintf(stderr, "oracle: edge shared by >2 cells\n"); free(rec); free(cell_of); orc_destroy(o); return NULL; }
        long long key = rec[2 * i];
        o->fv[2 * nfc] = (int)(key / nv); o->fv[2 * nfc + 1] = (int)(key % nv);
        for (int r = 0; r < 2; ++r) {
            if (i + r < j) {
                int e = (int)rec[2 * (i + r) + 1];
                o->fc[2 * nfc + r] = cell_of[e];
                o->fj[2 * nfc + r] = e - cptr[cell_of[e]];
                o->cf[e] = nfc;
            } else { o->fc[2 * nfc + r] = -1; o->fj[2 * nfc + r] = -1; }
        }
        int c0 = o->fc[2 * nfc], c1 = o->fc[2 * nfc + 1];
        if (c1 < 0) o->ftag[nfc] = med[c0] == FLUID ? T_BND_F : T_BND_S;
        else if (med[c0] != med[c1]) o->ftag[nfc] = T_GAMMA;
        else o->ftag[nfc] = med[c0] == FLUID ? T_INT_F : T_INT_S;
        ++nfc;
        i = j;
    }
    free(rec); free(cell_of);
    o->nfc = nfc;

    /* face geometry and orthonormal face bases */
    o->flen = malloc(sizeof(double) * nfc); o->fmid = malloc(sizeof(double) * 2 * nfc);
    o->ftan = malloc(sizeof(double) * 2 * nfc);
    o->fC = malloc(sizeof(double) * nfc * nf * nf); o->MF = malloc(sizeof(double) * nfc * nf * nf);
    for (int f = 0; f < nfc; ++f) {
        int a = o->fv[2 * f], b = o->fv[2 * f + 1];
        double dx = xy[2 * b] - xy[2 * a], dy = xy[2 * b + 1] - xy[2 * a + 1];
        double L = sqrt(dx * dx + dy * dy);
        o->flen[f] = L; o->ftan[2 * f] = dx / L; o->ftan[2 * f + 1] = dy / L;
        o->fmid[2 * f] = 0.5 * (xy[2 * a] + xy[2 * b]); o->fmid[2 * f + 1] = 0.5 * (xy[2 * a + 1] + xy[2 * b + 1]);
        double px[32], py[32], pw[32], Gm[64], Lc[64];
        int nq = face_quad(o, f, k + 2, px, py, pw);
        memset(Gm, 0, sizeof(Gm));
        for (int q = 0; q < nq; ++q) {
            double xi = 2.0 * ((px[q] - o->fmid[2 * f]) * o->ftan[2 * f] + (py[q] - o->fmid[2 * f + 1]) * o->ftan[2 * f + 1]) / L;
            for (int i = 0; i < nf; ++i) for (int l = 0; l < nf; ++l) Gm[i * nf + l] += pw[q] * ipow(xi, i) * ipow(xi, l);
        }
        cholesky(nf, Gm, Lc);
        lower_inverse(nf, Lc, o->fC + (size_t)f * nf * nf);
        double *MF = o->MF + (size_t)f * nf * nf;
        memset(MF, 0, sizeof(double) * nf * nf);
        for (int q = 0; q < nq; ++q) {
            double psi[16];
            face_basis_eval(o, f, px[q], py[q], psi);
            for (int i = 0; i < nf; ++i) for (int l = 0; l < nf; ++l) MF[i * nf + l] += pw[q] * psi[i] * psi[l];
        }
    }

    /* cell geometry: shoelace area and centroid, diameter = max vertex distance */
    o->area = malloc(sizeof(double) * nc); o->bary = malloc(sizeof(double) * 2 * nc); o->hT = malloc(sizeof(double) * nc);
    for (int c = 0; c < nc; ++c) {
        int s = cptr[c], m = cptr[c + 1] - s;
        double A = 0, cx = 0, cy = 0, h = 0;
        for (int t = 0; t < m; ++t) {
            int i0 = cvtx[s + t], i1 = cvtx[s + (t + 1) % m];
            double x0 = xy[2 * i0], y0 = xy[2 * i0 + 1], x1 = xy[2 * i1], y1 = xy[2 * i1 + 1];
            double cr = x0 * y1 - x1 * y0;
            A += cr; cx += (x0 + x1) * cr; cy += (y0 + y1) * cr;
            for (int u = 0; u < m; ++u) {
                int i2 = cvtx[s + u];
                double d = hypot(xy[2 * i2] - x0, xy[2 * i2 + 1] - y0);
                if (d > h) h = d;
            }
        }
        A *= 0.5;
        if (!(A > 0)) { fprintf(stderr, "oracle: cell %d not counter-clockwise or degenerate\n", c); orc_destroy(o); return NULL; }
        o->area[c] = A; o->bary[2 * c] = cx / (6 * A); o->bary[2 * c + 1] = cy / (6 * A); o->hT[c] = h;
    }

    /* orthonormal cell bases and local operators by quadrature */
    o->C = calloc((size_t)nc * N * N, sizeof(double));
    o->M0 = calloc((size_t)nc * N * N, sizeof(double));
    o->L0 = calloc((size_t)nc * N * N, sizeof(double));
    o->D = calloc((size_t)nc * 2 * N * N, sizeof(double));
    o->E = calloc((size_t)ne * N * N, sizeof(double));
    o->G = calloc((size_t)ne * N * nf, sizeof(double));
    o->nrm = calloc((size_t)ne * 2, sizeof(double));
    o->tau = calloc(nc, sizeof(double));
    o->Cinv = calloc((size_t)nc * 9, sizeof(double));
    o->Cinv_iv = calloc((size_t)nc * 9, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < nc; ++c) {
        double px[4096], py[4096], pw[4096];
        int nq = cell_quad(o, c, k + 2, px, py, pw);
        double Gm[256], Lc[256], mu[64];
        memset(Gm, 0, sizeof(Gm));
        for (int q = 0; q < nq; ++q) {
            mono_eval(o, c, px[q], py[q], mu, NULL, NULL);
            for (int a = 0; a < N; ++a) for (int b = 0; b < N; ++b) Gm[a * N + b] += pw[q] * mu[a] * mu[b];
        }
        if (cholesky(N, Gm, Lc)) { bad = 1; continue; }
        lower_inverse(N, Lc, o->C + (size_t)c * N * N);
        double *M0 = o->M0 + (size_t)c * N * N, *Dx = o->D + (size_t)c * 2 * N * N, *Dy = Dx + N * N;
        for (int q = 0; q < nq; ++q) {
            double ph[64], phx[64], phy[64];
            basis_eval(o, c, px[q], py[q], ph, phx, phy);
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    M0[a * N + b] += pw[q] * ph[a] * ph[b];
                    Dx[a * N + b] += pw[q] * phx[b] * ph[a];
                    Dy[a * N + b] += pw[q] * phy[b] * ph[a];
                }
        }
        cholesky(N, M0, o->L0 + (size_t)c * N * N);
        int s = cptr[c], m = cptr[c + 1] - s;
        for (int t = 0; t < m; ++t) {
            int e = s + t, f = o->cf[e];
            int i0 = cvtx[s + t], i1 = cvtx[s + (t + 1) % m];
            double dx = xy[2 * i1] - xy[2 * i0], dy = xy[2 * i1 + 1] - xy[2 * i0 + 1], L = hypot(dx, dy);
            o->nrm[2 * e] = dy / L; o->nrm[2 * e + 1] = -dx / L;
            double fx[32], fy[32], fw[32];
            int nfq = face_quad(o, f, k + 2, fx, fy, fw);
            double *E = o->E + (size_t)e * N * N, *G = o->G + (size_t)e * N * nf;
            for (int q = 0; q < nfq; ++q) {
                double ph[64], psi[16];
                basis_eval(o, c, fx[q], fy[q], ph, NULL, NULL);
                face_basis_eval(o, f, fx[q], fy[q], psi);
                for (int a = 0; a < N; ++a) {
                    for (int b = 0; b < N; ++b) E[a * N + b] += fw[q] * ph[a] * ph[b];
                    for (int i = 0; i < nf; ++i) G[a * nf + i] += fw[q] * ph[a] * psi[i];
                }
            }
        }
        /* materials: stabilisation weight eta * tau (alpha = 0) and compliance */
        double r = rho[c];
        if (med[c] == FLUID) {
            double cf = pa[c];
            o->tau[c] = eta_f / (r * cf);
        } else {
            double lam = pa[c], muL = pb[c];
            double cs = stab_speed == 0 ? sqrt((lam + 2 * muL) / r) : sqrt(muL / r);
            o->tau[c] = eta_s * r * cs;
            /* Cinv[al][be] = (C^{-1} E_be) : E_al, C^{-1} X = (X - lam/(2(lam+mu)) tr(X) I) / (2 mu) */
            double *Ci = o->Cinv + (size_t)c * 9;
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) {
                    double tr = Eten(be, 0, 0) + Eten(be, 1, 1), sacc = 0;
                    for (int i = 0; i < 2; ++i)
                        for (int j = 0; j < 2; ++j) {
                            double X = (Eten(be, i, j) - lam / (2 * (lam + muL)) * tr * (i == j)) / (2 * muL);
                            sacc += X * Eten(al, i, j);
                        }
                    Ci[al * 3 + be] = sacc;
                }
            /* its inverse, column by column */
            for (int be = 0; be < 3; ++be) {
                double A9[9], rhs[3] = {0, 0, 0};
                memcpy(A9, Ci, sizeof(A9));
                rhs[be] = 1.0;
                lu_solve(3, A9, rhs);
                for (int al = 0; al < 3; ++al) o->Cinv_iv[(size_t)c * 9 + al * 3 + be] = rhs[al];
            }
        }
    }
    if (bad) { fprintf(stderr, "oracle: Gram matrix not SPD\n"); orc_destroy(o); return NULL; }
    o->off = malloc(sizeof(int) * (nc + 1));
    o->off[0] = 0;
    for (int c = 0; c < nc; ++c) o->off[c + 1] = o->off[c] + (med[c] == FLUID ? 3 : 5) * N;
    o->foff = malloc(sizeof(int) * (nfc + 1));
    o->foff[0] = 0;
    for (int f = 0; f < nfc; ++f) {
        int w = o->ftag[f] == T_INT_F ? 1 : o->ftag[f] == T_INT_S ? 2 : o->ftag[f] == T_GAMMA ? 3 : 0;
        o->foff[f + 1] = o->foff[f] + w * nf;
    }
    o->UF = calloc(o->foff[nfc] + 1, sizeof(double));
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    void *p[] = {o->xy, o->cptr, o->cvtx, o->med, o->rho, o->pa, o->pb, o->fv, o->fc, o->fj, o->ftag, o->cf,
                 o->flen, o->fmid, o->ftan, o->fC, o->MF, o->area, o->bary, o->hT, o->C, o->M0, o->L0, o->D,
                 o->E, o->G, o->nrm, o->tau, o->Cinv, o->Cinv_iv, o->off, o->foff, o->src_cell, o->src_phi,
                 o->src_par, o->dload, o->domega, o->dphase, o->UF, o->KT, o->KTF, o->KF, o->KFT,
                 o->kt_off, o->ktf_off, o->kf_off, o->kft_off};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    free(o);
}

/* ---------------------------------------------------------------- queries */

int orc_ndof(const orc_t *o) { return o->off[o->nc]; }
int orc_nfaces(const orc_t *o) { return o->nfc; }
int orc_nface_dofs(const orc_t *o) { return o->foff[o->nfc]; }
void orc_offsets(const orc_t *o, int *off) { memcpy(off, o->off, sizeof(int) * (o->nc + 1)); }
void orc_face_offsets(const orc_t *o, int *off) { memcpy(off, o->foff, sizeof(int) * (o->nfc + 1)); }
void orc_face_info(const orc_t *o, int *fv, int *fc, int *ftag)
{
    memcpy(fv, o->fv, sizeof(int) * 2 * o->nfc);
    memcpy(fc, o->fc, sizeof(int) * 2 * o->nfc);
    memcpy(ftag, o->ftag, sizeof(int) * o->nfc);
}
void orc_cell_geom(const orc_t *o, double *area, double *bary, double *h, double *tau)
{
    memcpy(area, o->area, sizeof(double) * o->nc);
    memcpy(bary, o->bary, sizeof(double) * 2 * o->nc);
    memcpy(h, o->hT, sizeof(double) * o->nc);
    memcpy(tau, o->tau, sizeof(double) * o->nc);
}

/* local operator blocks of cell c: M0 [N][N], D [2][N][N], and per local edge E, G, n */
void orc_cell_ops(const orc_t *o, int c, double *M0, double *D, double *E, double *G, double *nrm, int *faces)
{
    int N = o->N, nf = o->nf, s = o->cptr[c], m = o->cptr[c + 1] - s;
    memcpy(M0, o->M0 + (size_t)c * N * N, sizeof(double) * N * N);
    memcpy(D, o->D + (size_t)c * 2 * N * N, sizeof(double) * 2 * N * N);
    memcpy(E, o->E + (size_t)s * N * N, sizeof(double) * m * N * N);
    memcpy(G, o->G + (size_t)s * N * nf, sizeof(double) * m * N * nf);
    memcpy(nrm, o->nrm + (size_t)s * 2, sizeof(double) * m * 2);
    memcpy(faces, o->cf + s, sizeof(int) * m);
}

void orc_face_mass(const orc_t *o, int f, double *MF) { memcpy(MF, o->MF + (size_t)f * o->nf * o->nf, sizeof(double) * o->nf * o->nf); }

/* cell basis values at a point (no containment check) */
void orc_basis(const orc_t *o, int c, double x, double y, double *phi, double *phx, double *phy)
{
    basis_eval(o, c, x, y, phi, phx, phy);
}

/* cell basis values at many points (cells given per point) */
void orc_basis_many(const orc_t *o, int n, const int *cells, const double *x, const double *y, double *phi)
{
#pragma omp parallel for schedule(static)
    for (int q = 0; q < n; ++q) basis_eval(o, cells[q], x[q], y[q], phi + (size_t)q * o->N, NULL, NULL);
}

/* face basis values at a point of face f */
void orc_face_basis(const orc_t *o, int f, double x, double y, double *psi) { face_basis_eval(o, f, x, y, psi); }

/* lowest-id cell whose closed polygon contains (x, y); -1 if none */
int orc_locate(const orc_t *o, double x, double y)
{
    for (int c = 0; c < o->nc; ++c) {
        int s = o->cptr[c], m = o->cptr[c + 1] - s, in = 1;
        double tol = 1e-12 * o->hT[c];
        for (int t = 0; t < m && in; ++t) {
            int i0 = o->cvtx[s + t], i1 = o->cvtx[s + (t + 1) % m];
            double ex = o->xy[2 * i1] - o->xy[2 * i0], ey = o->xy[2 * i1 + 1] - o->xy[2 * i0 + 1];
            double cr = ex * (y - o->xy[2 * i0 + 1]) - ey * (x - o->xy[2 * i0]);
            if (cr < -tol * hypot(ex, ey)) in = 0;
        }
        if (in) return c;
    }
    return -1;
}

/* quadrature points of all cells (nq Gauss points per direction per fan triangle) */
int orc_quad_count(const orc_t *o, int nq) { return (o->cptr[o->nc]) * nq * nq; }
void orc_quad_points(const orc_t *o, int nq, double *px, double *py, double *pw, int *pc)
{
    int q = 0;
    for (int c = 0; c < o->nc; ++c) {
        int n = cell_quad(o, c, nq, px + q, py + q, pw + q);
        for (int i = 0; i < n; ++i) pc[q + i] = c;
        q += n;
    }
}

/* ---------------------------------------------------------------- loads */

void orc_set_point_sources(orc_t *o, int n, const double *xy, const double *dir, const double *f0,
                           const double *t0, const double *amp)
{
    free(o->src_cell); free(o->src_phi); free(o->src_par);
    o->nsrc = n;
    o->src_cell = malloc(sizeof(int) * (n + 1));
    o->src_phi = malloc(sizeof(double) * (n + 1) * o->N);
    o->src_par = malloc(sizeof(double) * (n + 1) * 5);
    for (int s = 0; s < n; ++s) {
        int c = orc_locate(o, xy[2 * s], xy[2 * s + 1]);
        o->src_cell[s] = c;
        if (c >= 0) basis_eval(o, c, xy[2 * s], xy[2 * s + 1], o->src_phi + (size_t)s * o->N, NULL, NULL);
        o->src_par[5 * s] = dir[2 * s]; o->src_par[5 * s + 1] = dir[2 * s + 1];
        o->src_par[5 * s + 2] = f0[s]; o->src_par[5 * s + 3] = t0[s]; o->src_par[5 * s + 4] = amp[s];
    }
}

void orc_set_dense_load(orc_t *o, int nterm, const double *g, const double *omega, const double *phase)
{
    free(o->dload); free(o->domega); free(o->dphase);
    size_t nd = (size_t)o->off[o->nc];
    o->nterm = nterm;
    o->dload = malloc(sizeof(double) * (nterm * nd + 1));
    o->domega = malloc(sizeof(double) * (nterm + 1));
    o->dphase = malloc(sizeof(double) * (nterm + 1));
    if (nterm) {
        memcpy(o->dload, g, sizeof(double) * nterm * nd);
        memcpy(o->domega, omega, sizeof(double) * nterm);
        memcpy(o->dphase, phase, sizeof(double) * nterm);
    }
}

/* Ricker wavelet (second derivative of a Gaussian) with peak frequency f0, delay t0, as the time
 * factor of a point force.  Parity unpinned: the paper's "Ricker" is a spatial initial field
 * (eq. ricker_ic), it prints no values for a time-domain wavelet; the formula is the textbook
 * (1 - 2a^2) exp(-a^2), a = pi f0 (t - t0). */
static double ricker(double t, double f0, double t0)
{
    double a = M_PI * f0 * (t - t0);
    return (1.0 - 2.0 * a * a) * exp(-a * a);
}

/* ---------------------------------------------------------------- operator */

/* Face system of face f (eq. ex_solve, first line): A = K_F (n x n, the face block of the weak
 * form), r = -K_FT U_T built from the dofs of the adjacent cells (u_side[0], u_side[1]).
 * Returns n = number of face unknowns (0 on the boundary). */
static int face_system(const orc_t *o, int f, const double *const *u_side, double *A, double *r)
{
    int N = o->N, nf = o->nf;
    int tag = o->ftag[f];
    if (tag == T_BND_F || tag == T_BND_S) return 0;
    int w = tag == T_INT_F ? 1 : tag == T_INT_S ? 2 : 3, n = w * nf;
    memset(A, 0, sizeof(double) * n * n);
    memset(r, 0, sizeof(double) * n);
    const double *MF = o->MF + (size_t)f * nf * nf;
    for (int side = 0; side < 2; ++side) {
        int c = o->fc[2 * f + side];
        int e = o->cptr[c] + o->fj[2 * f + side];
        const double *G = o->G + (size_t)e * N * nf, *nv = o->nrm + 2 * e, *u = u_side[side];
        double tau = o->tau[c];
        if (o->med[c] == FLUID) {
            /* rows q_F: tau (p_T - p_F, q_F)_F - (m_T . n_T, q_F)_F   (eq. stab_a, rec_a tested with q_F) */
            int r0 = 0;  /* fluid face unknowns first */
            for (int i = 0; i < nf; ++i) {
                double t = 0, q = 0;
                for (int a = 0; a < N; ++a) {
                    t += G[a * nf + i] * u[a];
                    q += G[a * nf + i] * (nv[0] * u[N + a] + nv[1] * u[2 * N + a]);
                }
                r[r0 + i] += tau * t - q;
                for (int l = 0; l < nf; ++l) A[(r0 + i) * n + r0 + l] += tau * MF[i * nf + l];
            }
        } else {
            int r0 = (tag == T_GAMMA) ? nf : 0;
            for (int cc = 0; cc < 2; ++cc)
                for (int i = 0; i < nf; ++i) {
                    double t = 0, q = 0;
                    for (int a = 0; a < N; ++a) {
                        t += G[a * nf + i] * u[cc * N + a];
                        double sn = 0;  /* (s n)_cc = sum_al (E_al n)_cc s_al */
                        for (int al = 0; al < 3; ++al)
                            sn += (Eten(al, cc, 0) * nv[0] + Eten(al, cc, 1) * nv[1]) * u[(2 + al) * N + a];
                        q += G[a * nf + i] * sn;
                    }
                    r[r0 + cc * nf + i] += tau * t - q;
                    for (int l = 0; l < nf; ++l) A[(r0 + cc * nf + i) * n + r0 + cc * nf + l] += tau * MF[i * nf + l];
                }
        }
    }
    if (tag == T_GAMMA) {
        /* coupling block C[i][(c,l)] = (n_G,c psi_l, psi_i)_F with n_G pointing from solid to fluid:
         * fluid rows +C v_F, solid rows -C^T p_F (eq. HHO1 / HHO2 coupling terms) */
        int cs = o->med[o->fc[2 * f]] == SOLID ? 0 : 1;
        int es = o->cptr[o->fc[2 * f + cs]] + o->fj[2 * f + cs];
        const double *ng = o->nrm + 2 * es;
        for (int i = 0; i < nf; ++i)
            for (int cc = 0; cc < 2; ++cc)
                for (int l = 0; l < nf; ++l) {
                    double Cv = ng[cc] * MF[i * nf + l];
                    A[i * n + nf + cc * nf + l] += Cv;
                    A[(nf + cc * nf + l) * n + i] -= Cv;
                }
    }
    return n;
}

/* Face solves K_F U_F = -K_FT U_T for every non-boundary face (eq. ex_solve, first line). */
void orc_face_values(orc_t *o, const double *U, double *UF)
{
#pragma omp parallel for schedule(static)
    for (int f = 0; f < o->nfc; ++f) {
        double A[576], r[24];
        const double *us[2] = {U + o->off[o->fc[2 * f]], o->fc[2 * f + 1] >= 0 ? U + o->off[o->fc[2 * f + 1]] : NULL};
        int n = face_system(o, f, us, A, r);
        if (!n) continue;
        if (lu_solve(n, A, r)) fprintf(stderr, "oracle: singular face block %d\n", f);
        memcpy(UF + o->foff[f], r, sizeof(double) * n);
    }
}

/* face unknown block of face f as seen from a cell of the given medium (NULL-safe zero on the boundary) */
static const double *face_slice(const orc_t *o, const double *UF, int f, int medium, const double *zero)
{
    int tag = o->ftag[f];
    if (tag == T_BND_F || tag == T_BND_S) return zero;
    if (tag == T_GAMMA && medium == SOLID) return UF + o->foff[f] + o->nf;
    return UF + o->foff[f];
}

/* Cell residual without loads, R = -(K_T u + K_TF u_F) (eq. ex_solve, second line, weak form of
 * eq. HHO1 / HHO2): u = the cell's dofs, uf[t] = its face unknowns on local face t (the fluid slice
 * for a fluid cell, the solid slice for a solid cell; zeros on boundary faces). */
static void cell_residual(const orc_t *o, int c, const double *u, const double *const *uf, double *R)
{
    int N = o->N, nf = o->nf;
    const double *Dx = o->D + (size_t)c * 2 * N * N, *Dd[2] = {Dx, Dx + N * N};
    int s = o->cptr[c], m = o->cptr[c + 1] - s;
    double tau = o->tau[c];
    int nd = o->off[c + 1] - o->off[c];
    memset(R, 0, sizeof(double) * nd);
    if (o->med[c] == FLUID) {
        const double *p = u, *mc[2] = {u + N, u + 2 * N};
        for (int a = 0; a < N; ++a) {
            /* m rows: (grad p_T, r)_T - (p_T - p_F, r . n)_dT      (eq. rec_a) */
            for (int cc = 0; cc < 2; ++cc) {
                double v = 0;
                for (int b = 0; b < N; ++b) v += Dd[cc][a * N + b] * p[b];
                R[(1 + cc) * N + a] = v;
            }
            /* p row: -(m, g_T(q_T, 0))_T = -(grad q, m)_T + (q, m . n)_dT */
            double v = 0;
            for (int cc = 0; cc < 2; ++cc)
                for (int b = 0; b < N; ++b) v -= Dd[cc][b * N + a] * mc[cc][b];
            R[a] = v;
        }
        for (int t2 = 0; t2 < m; ++t2) {
            int e = s + t2, f = o->cf[e];
            const double *E = o->E + (size_t)e * N * N, *G = o->G + (size_t)e * N * nf, *nv = o->nrm + 2 * e;
            const double *pF = uf[t2];
            for (int a = 0; a < N; ++a) {
                double jump = 0, mn = 0;  /* (p_T - p_F, phi_a)_F and (m . n, phi_a)_F */
                for (int b = 0; b < N; ++b) { jump += E[a * N + b] * p[b]; mn += E[a * N + b] * (nv[0] * mc[0][b] + nv[1] * mc[1][b]); }
                for (int i = 0; i < nf; ++i) jump -= G[a * nf + i] * pF[i];
                R[N + a] -= nv[0] * jump;
                R[2 * N + a] -= nv[1] * jump;
                R[a] += mn - tau * jump;   /* + (q, m.n)_F - tau (p_T - p_F, q)_F */
            }
        }
    } else {
        const double *vc[2] = {u, u + N}, *sa[3] = {u + 2 * N, u + 3 * N, u + 4 * N};
        for (int a = 0; a < N; ++a) {
            /* s rows: (grad_sym v_T, E_al phi_a)_T */
            for (int al = 0; al < 3; ++al) {
                double v = 0;
                for (int cc = 0; cc < 2; ++cc)
                    for (int d = 0; d < 2; ++d) {
                        double q = Eten(al, cc, d);
                        if (q == 0) continue;
                        for (int b = 0; b < N; ++b) v += q * Dd[d][a * N + b] * vc[cc][b];
                    }
                R[(2 + al) * N + a] = v;
            }
            /* v rows: -(s, grad_sym(e_cc phi_a))_T */
            for (int cc = 0; cc < 2; ++cc) {
                double v = 0;
                for (int al = 0; al < 3; ++al)
                    for (int d = 0; d < 2; ++d) {
                        double q = Eten(al, cc, d);
                        if (q == 0) continue;
                        for (int b = 0; b < N; ++b) v -= q * Dd[d][b * N + a] * sa[al][b];
                    }
                R[cc * N + a] = v;
            }
        }
        for (int t2 = 0; t2 < m; ++t2) {
            int e = s + t2, f = o->cf[e];
            const double *E = o->E + (size_t)e * N * N, *G = o->G + (size_t)e * N * nf, *nv = o->nrm + 2 * e;
            const double *vF = uf[t2];
            for (int a = 0; a < N; ++a) {
                double jump[2], sn[2] = {0, 0};
                for (int cc = 0; cc < 2; ++cc) {
                    double j = 0;
                    for (int b = 0; b < N; ++b) j += E[a * N + b] * vc[cc][b];
                    for (int i = 0; i < nf; ++i) j -= G[a * nf + i] * vF[cc * nf + i];
                    jump[cc] = j;
                    for (int al = 0; al < 3; ++al) {
                        double En = Eten(al, cc, 0) * nv[0] + Eten(al, cc, 1) * nv[1];
                        if (En == 0) continue;
                        for (int b = 0; b < N; ++b) sn[cc] += En * E[a * N + b] * sa[al][b];
                    }
                }
                /* s rows: - (v_T - v_F, E_al n)_F */
                for (int al = 0; al < 3; ++al) {
                    double v = 0;
                    for (int cc = 0; cc < 2; ++cc) v += (Eten(al, cc, 0) * nv[0] + Eten(al, cc, 1) * nv[1]) * jump[cc];
                    R[(2 + al) * N + a] -= v;
                }
                /* v rows: + (s n, w)_F - tau (v_T - v_F, w)_F */
                for (int cc = 0; cc < 2; ++cc) R[cc * N + a] += sn[cc] - tau * jump[cc];
            }
        }
    }
}

/* out = M_T^{-1} R: rho M0 for m / v, (1/kappa) M0 for p, (Cinv (x) M0) for s (eq. mass). */
static void cell_inv_mass(const orc_t *o, int c, const double *R, double *out)
{
    int N = o->N;
    /* inverse mass: rho M0 for m / v, (1/kappa) M0 for p, (Cinv (x) M0) for s */
    const double *L0 = o->L0 + (size_t)c * N * N;
    if (o->med[c] == FLUID) {
        double kap = o->rho[c] * o->pa[c] * o->pa[c];
        for (int a = 0; a < N; ++a) { out[a] = kap * R[a]; out[N + a] = R[N + a] / o->rho[c]; out[2 * N + a] = R[2 * N + a] / o->rho[c]; }
        for (int bl = 0; bl < 3; ++bl) chol_solve(N, L0, out + bl * N);
    } else {
        const double *Ci = o->Cinv_iv + (size_t)c * 9;
        for (int a = 0; a < N; ++a) {
            out[a] = R[a] / o->rho[c];
            out[N + a] = R[N + a] / o->rho[c];
            for (int al = 0; al < 3; ++al) {
                double v = 0;
                for (int be = 0; be < 3; ++be) v += Ci[al * 3 + be] * R[(2 + be) * N + a];
                out[(2 + al) * N + a] = v;
            }
        }
        for (int bl = 0; bl < 5; ++bl) chol_solve(N, L0, out + bl * N);
    }
}

/* Cell residual R = F_T - K_T U_T - K_TF U_F and dU = M^{-1} R (eq. ex_solve, second line). */
static void cell_update(orc_t *o, const double *U, const double *UF, double t, double *dU)
{
    int N = o->N;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        static const double zero[64] = {0};
        const double *u = U + o->off[c];
        int s = o->cptr[c], m = o->cptr[c + 1] - s, nd = o->off[c + 1] - o->off[c];
        const double *uf[16];
        for (int t2 = 0; t2 < m; ++t2) uf[t2] = face_slice(o, UF, o->cf[s + t2], o->med[c], zero);
        double R[5 * 64];
        cell_residual(o, c, u, uf, R);
        /* loads F_T (eq. rhs, load-vector reading): point sources and separable dense terms */
        for (int q = 0; q < o->nsrc; ++q) {
            if (o->src_cell[q] != c) continue;
            const double *pp = o->src_par + 5 * q, *ph = o->src_phi + (size_t)q * N;
            double w = pp[4] * ricker(t, pp[2], pp[3]);
            if (o->med[c] == FLUID) for (int a = 0; a < N; ++a) R[a] += w * pp[0] * ph[a];
            else for (int cc = 0; cc < 2; ++cc) for (int a = 0; a < N; ++a) R[cc * N + a] += w * pp[cc] * ph[a];
        }
        for (int q = 0; q < o->nterm; ++q) {
            double w = sin(o->domega[q] * t + o->dphase[q]);
            const double *g = o->dload + (size_t)q * o->off[o->nc] + o->off[c];
            for (int i = 0; i < nd; ++i) R[i] += w * g[i];
        }
        cell_inv_mass(o, c, R, dU + o->off[c]);
    }
}

/* dU/dt = M^{-1}(F_T(t) - K_eff U_T): face condensation then cell update */
void orc_rhs(orc_t *o, const double *U, double t, double *dU)
{
    orc_face_values(o, U, o->UF);
    cell_update(o, U, o->UF, t, dU);
}

/* ERK(s) Butcher tableaux, eq. ERK */
static void tableau(int s, double A[4][4], double *b, double *c)
{
    memset(A, 0, sizeof(double) * 16);
    if (s == 2) { A[1][0] = 0.5; b[0] = 0; b[1] = 1; c[0] = 0; c[1] = 0.5; }
    else if (s == 3) { A[1][0] = 0.5; A[2][0] = -1; A[2][1] = 2; b[0] = 1.0 / 6; b[1] = 2.0 / 3; b[2] = 1.0 / 6; c[0] = 0; c[1] = 0.5; c[2] = 1; }
    else { A[1][0] = 0.5; A[2][1] = 0.5; A[3][2] = 1; b[0] = 1.0 / 6; b[1] = 1.0 / 3; b[2] = 1.0 / 3; b[3] = 1.0 / 6; c[0] = 0; c[1] = 0.5; c[2] = 0.5; c[3] = 1; }
}

/* n_steps of ERK(s) from time t0 with step dt, U updated in place.
 * If E is non-NULL, E[n] receives the energy after step n (n = 0 .. n_steps-1). */
double orc_energy(const orc_t *o, const double *U);
int orc_erk(orc_t *o, int s, double *U, double t0, double dt, int nsteps, double *Eout)
{
    if (s < 2 || s > 4) return -1;
    double A[4][4], b[4], c[4];
    tableau(s, A, b, c);
    size_t nd = o->off[o->nc];
    double *K = malloc(sizeof(double) * nd * s), *Y = malloc(sizeof(double) * nd);
    for (int n = 0; n < nsteps; ++n) {
        double t = t0 + n * dt;
        for (int i = 0; i < s; ++i) {
            for (size_t q = 0; q < nd; ++q) {
                double v = U[q];
                for (int j = 0; j < i; ++j) v += dt * A[i][j] * K[j * nd + q];
                Y[q] = v;
            }
            orc_rhs(o, Y, t + c[i] * dt, K + i * nd);
        }
        for (size_t q = 0; q < nd; ++q) {
            double v = 0;
            for (int i = 0; i < s; ++i) v += b[i] * K[i * nd + q];
            U[q] += dt * v;
        }
        if (Eout) Eout[n] = orc_energy(o, U);
    }
    free(K); free(Y);
    return 0;
}

/* Discrete energy of Sec. 5.1: half the mass-weighted squared norms of the cell unknowns. */
double orc_energy(const orc_t *o, const double *U)
{
    int N = o->N;
    double E = 0;
#pragma omp parallel for reduction(+ : E) schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        const double *u = U + o->off[c], *M0 = o->M0 + (size_t)c * N * N;
        double e = 0;
        if (o->med[c] == FLUID) {
            double kap = o->rho[c] * o->pa[c] * o->pa[c];
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b)
                    e += M0[a * N + b] * (u[a] * u[b] / kap + o->rho[c] * (u[N + a] * u[N + b] + u[2 * N + a] * u[2 * N + b]));
        } else {
            const double *Ci = o->Cinv + (size_t)c * 9;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    double v = o->rho[c] * (u[a] * u[b] + u[N + a] * u[N + b]);
                    for (int al = 0; al < 3; ++al)
                        for (int be = 0; be < 3; ++be) v += Ci[al * 3 + be] * u[(2 + al) * N + a] * u[(2 + be) * N + b];
                    e += M0[a * N + b] * v;
                }
        }
        E += 0.5 * e;
    }
    return E;
}

/* Mass-weighted inner product U^T M V (the energy's bilinear form, times 2). */
double orc_mass_dot(const orc_t *o, const double *U, const double *V)
{
    int N = o->N;
    double E = 0;
    for (int c = 0; c < o->nc; ++c) {
        const double *u = U + o->off[c], *v = V + o->off[c], *M0 = o->M0 + (size_t)c * N * N;
        if (o->med[c] == FLUID) {
            double kap = o->rho[c] * o->pa[c] * o->pa[c];
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b)
                    E += M0[a * N + b] * (u[a] * v[b] / kap + o->rho[c] * (u[N + a] * v[N + b] + u[2 * N + a] * v[2 * N + b]));
        } else {
            const double *Ci = o->Cinv + (size_t)c * 9;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    double w = o->rho[c] * (u[a] * v[b] + u[N + a] * v[N + b]);
                    for (int al = 0; al < 3; ++al)
                        for (int be = 0; be < 3; ++be) w += Ci[al * 3 + be] * u[(2 + al) * N + a] * v[(2 + be) * N + b];
                    E += M0[a * N + b] * w;
                }
        }
    }
    return E;
}

/* Stabilisation energy sum_T eta tau_T || S_dT(u_T, u_dT) ||^2 at (U, U_F(U)) (eq. stab). */
double orc_stab_energy(orc_t *o, const double *U)
{
    int N = o->N, nf = o->nf;
    static const double zero[64] = {0};
    orc_face_values(o, U, o->UF);
    double S = 0;
    for (int c = 0; c < o->nc; ++c) {
        const double *u = U + o->off[c];
        int s = o->cptr[c], m = o->cptr[c + 1] - s, ncomp = o->med[c] == FLUID ? 1 : 2;
        for (int t = 0; t < m; ++t) {
            int e = s + t, f = o->cf[e];
            const double *E = o->E + (size_t)e * N * N, *G = o->G + (size_t)e * N * nf, *MF = o->MF + (size_t)f * nf * nf;
            const double *uf = face_slice(o, o->UF, f, o->med[c], zero);
            for (int cc = 0; cc < ncomp; ++cc) {
                const double *ut = u + cc * N, *ufc = uf + cc * nf;
                double v = 0;
                for (int a = 0; a < N; ++a) for (int b = 0; b < N; ++b) v += ut[a] * E[a * N + b] * ut[b];
                for (int a = 0; a < N; ++a) for (int i = 0; i < nf; ++i) v -= 2 * ut[a] * G[a * nf + i] * ufc[i];
                for (int i = 0; i < nf; ++i) for (int l = 0; l < nf; ++l) v += ufc[i] * MF[i * nf + l] * ufc[l];
                S += o->tau[c] * v;
            }
        }
    }
    return S;
}

/* point values of the cell polynomials of U at (x, y): ncomp = 3 (fluid) or 5 (solid) */
int orc_point_values(const orc_t *o, const double *U, double x, double y, double *vals)
{
    int c = orc_locate(o, x, y);
    if (c < 0) return -1;
    double phi[64];
    basis_eval(o, c, x, y, phi, NULL, NULL);
    int nb = o->med[c] == FLUID ? 3 : 5;
    for (int bl = 0; bl < nb; ++bl) {
        double v = 0;
        for (int a = 0; a < o->N; ++a) v += phi[a] * U[o->off[c] + bl * o->N + a];
        vals[bl] = v;
    }
    return c;
}

/* ================================================================ discrete adjoint support
 *
 * The adjoint of the explicit Runge-Kutta path needs the transpose of the condensed operator
 * L = -M^{-1} K_eff, K_eff = K_T - K_TF K_F^{-1} K_FT (eq. compact_AR, eq. ex_solve).  The oracle
 * builds the blocks of K explicitly, cell by cell and face by face, by applying the residual
 * routines above to unit vectors (they are linear), and then applies transposes with plain
 * loops.  Parameter derivatives follow from the blocks that depend on the materials: the mass
 * matrices (eq. mass) and the stabilisation weight tau_T (eq. stab); the reconstructions and the
 * coupling block do not depend on them.
 */

/* face unknowns of a cell's slice on one face: fluid nf (p_F), solid 2 nf (v_F) */
static int cell_face_width(const orc_t *o, int c) { return (o->med[c] == FLUID ? 1 : 2) * o->nf; }

/* offset of a cell's slice inside the face unknown block of face f */
static int face_slice_offset(const orc_t *o, int f, int c)
{
    return (o->ftag[f] == T_GAMMA && o->med[c] == SOLID) ? o->nf : 0;
}

static int face_width(const orc_t *o, int f) { return o->foff[f + 1] - o->foff[f]; }

void orc_build_blocks(orc_t *o)
{
    if (o->KT) return;
    int nc = o->nc, nfc = o->nfc;
    o->kt_off = malloc(sizeof(size_t) * (nc + 1));
    o->ktf_off = malloc(sizeof(size_t) * (nc + 1));
    o->kf_off = malloc(sizeof(size_t) * (nfc + 1));
    o->kft_off = malloc(sizeof(size_t) * (nfc + 1));
    o->kt_off[0] = o->ktf_off[0] = 0;
    for (int c = 0; c < nc; ++c) {
        size_t nd = o->off[c + 1] - o->off[c], m = o->cptr[c + 1] - o->cptr[c];
        o->kt_off[c + 1] = o->kt_off[c] + nd * nd;
        o->ktf_off[c + 1] = o->ktf_off[c] + nd * m * cell_face_width(o, c);
    }
    o->kf_off[0] = o->kft_off[0] = 0;
    for (int f = 0; f < nfc; ++f) {
        size_t n = face_width(o, f), nd = 0;
        if (n) for (int side = 0; side < 2; ++side) nd += o->off[o->fc[2 * f + side] + 1] - o->off[o->fc[2 * f + side]];
        o->kf_off[f + 1] = o->kf_off[f] + n * n;
        o->kft_off[f + 1] = o->kft_off[f] + n * nd;
    }
    o->KT = calloc(o->kt_off[nc] + 1, sizeof(double));
    o->KTF = calloc(o->ktf_off[nc] + 1, sizeof(double));
    o->KF = calloc(o->kf_off[nfc] + 1, sizeof(double));
    o->KFT = calloc(o->kft_off[nfc] + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; ++c) {
        static const double zero[64] = {0};
        int nd = o->off[c + 1] - o->off[c], m = o->cptr[c + 1] - o->cptr[c], w = cell_face_width(o, c);
        double u[5 * 64], R[5 * 64], e[64];
        const double *uf[16];
        /* K_T[:, j] = -R(u = e_j, u_F = 0) */
        for (int t = 0; t < m; ++t) uf[t] = zero;
        double *KT = o->KT + o->kt_off[c];
        for (int j = 0; j < nd; ++j) {
            memset(u, 0, sizeof(double) * nd);
            u[j] = 1.0;
            cell_residual(o, c, u, uf, R);
            for (int a = 0; a < nd; ++a) KT[a * nd + j] = -R[a];
        }
        /* K_TF[:, (t, i)] = -R(u = 0, u_F on face t = e_i); boundary faces have no unknowns */
        double *KTF = o->KTF + o->ktf_off[c];
        memset(u, 0, sizeof(double) * nd);
        int ncol = m * w;
        for (int t = 0; t < m; ++t) {
            int f = o->cf[o->cptr[c] + t];
            if (!face_width(o, f)) continue;
            for (int i = 0; i < w; ++i) {
                memset(e, 0, sizeof(double) * w);
                e[i] = 1.0;
                uf[t] = e;
                cell_residual(o, c, u, uf, R);
                uf[t] = zero;
                for (int a = 0; a < nd; ++a) KTF[a * ncol + t * w + i] = -R[a];
            }
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int f = 0; f < nfc; ++f) {
        int n = face_width(o, f);
        if (!n) continue;
        int c0 = o->fc[2 * f], c1 = o->fc[2 * f + 1];
        int nd0 = o->off[c0 + 1] - o->off[c0], nd1 = o->off[c1 + 1] - o->off[c1], nd = nd0 + nd1;
        double u0[5 * 64], u1[5 * 64], A[576], r[24];
        const double *us[2] = {u0, u1};
        double *KFT = o->KFT + o->kft_off[f];
        for (int j = 0; j < nd; ++j) {
            memset(u0, 0, sizeof(double) * nd0);
            memset(u1, 0, sizeof(double) * nd1);
            if (j < nd0) u0[j] = 1.0;
            else u1[j - nd0] = 1.0;
            face_system(o, f, us, A, r);
            for (int i = 0; i < n; ++i) KFT[i * nd + j] = -r[i];  /* r = -K_FT u */
        }
        memcpy(o->KF + o->kf_off[f], A, sizeof(double) * n * n);
    }
}

/* K_eff z from the explicit blocks: K_T z + K_TF U_F, U_F = -K_F^{-1} K_FT z. */
void orc_keff(orc_t *o, const double *z, double *out)
{
    orc_build_blocks(o);
    double *UF = calloc(o->foff[o->nfc] + 1, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int f = 0; f < o->nfc; ++f) {
        int n = face_width(o, f);
        if (!n) continue;
        int c0 = o->fc[2 * f], c1 = o->fc[2 * f + 1];
        int nd0 = o->off[c0 + 1] - o->off[c0], nd = nd0 + o->off[c1 + 1] - o->off[c1];
        const double *KFT = o->KFT + o->kft_off[f];
        double A[576], r[24];
        for (int i = 0; i < n; ++i) {
            double v = 0;
            for (int j = 0; j < nd; ++j) v -= KFT[i * nd + j] * (j < nd0 ? z[o->off[c0] + j] : z[o->off[c1] + j - nd0]);
            r[i] = v;
        }
        memcpy(A, o->KF + o->kf_off[f], sizeof(double) * n * n);
        lu_solve(n, A, r);
        memcpy(UF + o->foff[f], r, sizeof(double) * n);
    }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        int nd = o->off[c + 1] - o->off[c], m = o->cptr[c + 1] - o->cptr[c], w = cell_face_width(o, c);
        const double *KT = o->KT + o->kt_off[c], *KTF = o->KTF + o->ktf_off[c], *zc = z + o->off[c];
        for (int a = 0; a < nd; ++a) {
            double v = 0;
            for (int j = 0; j < nd; ++j) v += KT[a * nd + j] * zc[j];
            for (int t = 0; t < m; ++t) {
                int f = o->cf[o->cptr[c] + t];
                if (!face_width(o, f)) continue;
                const double *uf = UF + o->foff[f] + face_slice_offset(o, f, c);
                for (int i = 0; i < w; ++i) v += KTF[a * m * w + t * w + i] * uf[i];
            }
            out[o->off[c] + a] = v;
        }
    }
    free(UF);
}

/* K_eff^T z = K_T^T z + K_FT^T W_F with the adjoint face values W_F = -K_F^{-T} K_TF^T z
 * (written to WF in the face unknown layout if WF is not NULL). */
void orc_keff_T(orc_t *o, const double *z, double *out, double *WF)
{
    orc_build_blocks(o);
    double *W = calloc(o->foff[o->nfc] + 1, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int f = 0; f < o->nfc; ++f) {
        int n = face_width(o, f);
        if (!n) continue;
        double a[24], A[576], At[576];
        memset(a, 0, sizeof(a));
        for (int side = 0; side < 2; ++side) {
            int c = o->fc[2 * f + side];
            int t = o->fj[2 * f + side], m = o->cptr[c + 1] - o->cptr[c], w = cell_face_width(o, c);
            int nd = o->off[c + 1] - o->off[c], so = face_slice_offset(o, f, c);
            const double *KTF = o->KTF + o->ktf_off[c], *zc = z + o->off[c];
            for (int i = 0; i < w; ++i) {
                double v = 0;
                for (int r = 0; r < nd; ++r) v += KTF[r * m * w + t * w + i] * zc[r];
                a[so + i] += v;
            }
        }
        memcpy(A, o->KF + o->kf_off[f], sizeof(double) * n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) At[i * n + j] = A[j * n + i];
        lu_solve(n, At, a);
        for (int i = 0; i < n; ++i) W[o->foff[f] + i] = -a[i];
    }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        int nd = o->off[c + 1] - o->off[c], m = o->cptr[c + 1] - o->cptr[c];
        const double *KT = o->KT + o->kt_off[c], *zc = z + o->off[c];
        double *oc = out + o->off[c];
        for (int j = 0; j < nd; ++j) {
            double v = 0;
            for (int a = 0; a < nd; ++a) v += KT[a * nd + j] * zc[a];
            oc[j] = v;
        }
        for (int t = 0; t < m; ++t) {
            int f = o->cf[o->cptr[c] + t], n = face_width(o, f);
            if (!n) continue;
            int c0 = o->fc[2 * f], nd0 = o->off[c0 + 1] - o->off[c0];
            int cnd = nd0 + o->off[o->fc[2 * f + 1] + 1] - o->off[o->fc[2 * f + 1]];
            int col0 = (c == c0) ? 0 : nd0;
            const double *KFT = o->KFT + o->kft_off[f], *Wf = W + o->foff[f];
            for (int j = 0; j < nd; ++j) {
                double v = 0;
                for (int i = 0; i < n; ++i) v += KFT[i * cnd + col0 + j] * Wf[i];
                oc[j] += v;
            }
        }
    }
    if (WF) memcpy(WF, W, sizeof(double) * o->foff[o->nfc]);
    free(W);
}

/* M^{-1} x for every cell (eq. mass). */
void orc_inv_mass(orc_t *o, const double *x, double *out)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) cell_inv_mass(o, c, x + o->off[c], out + o->off[c]);
}

/* L^T x = -K_eff^T M^{-1} x (the transpose of the condensed operator). */
void orc_rhs_T(orc_t *o, const double *x, double *out)
{
    int nd = o->off[o->nc];
    double *z = malloc(sizeof(double) * (nd + 1));
    orc_inv_mass(o, x, z);
    orc_keff_T(o, z, out, NULL);
    for (int i = 0; i < nd; ++i) out[i] = -out[i];
    free(z);
}

/* Parameter derivatives of one stage, accumulated per cell into grad[c][3]:
 *   grad -= w^T (dM/dtheta) k + (d tau_T / dtheta) sum_{F in dT} (Y_T - Y_F, w_T - W_F)_F
 * with w = M^{-1} mu, Y_F = forward face values of Y, W_F = adjoint face values of w
 * (mu^T (dL/dtheta) Y with L = -M^{-1} K_eff, the Schur-complement derivative written as a
 * bilinear form on the full cell-and-face system).  Parameters: fluid (rho, c, -), solid
 * (rho, lambda, mu); kappa = rho c^2, tau^f = eta^f / (rho c), tau^s = eta^s rho c^s. */
void orc_grad_terms(orc_t *o, const double *Y, const double *k, const double *mu, double *grad)
{
    int N = o->N, nf = o->nf, nd = o->off[o->nc];
    double *w = malloc(sizeof(double) * (nd + 1)), *tmp = malloc(sizeof(double) * (nd + 1));
    double *YF = calloc(o->foff[o->nfc] + 1, sizeof(double)), *WF = calloc(o->foff[o->nfc] + 1, sizeof(double));
    orc_inv_mass(o, mu, w);
    orc_face_values(o, Y, YF);
    orc_keff_T(o, w, tmp, WF);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        static const double zero[64] = {0};
        const double *M0 = o->M0 + (size_t)c * N * N;
        const double *yc = Y + o->off[c], *kc = k + o->off[c], *wc = w + o->off[c];
        double rho = o->rho[c], g[3] = {0, 0, 0};
        /* block b of w paired through M0 with block b' of k */
        #define MDOT(bw, bk) ({ double s_ = 0; for (int a_ = 0; a_ < N; ++a_) for (int b_ = 0; b_ < N; ++b_) \
                                s_ += wc[(bw) * N + a_] * M0[a_ * N + b_] * kc[(bk) * N + b_]; s_; })
        int ncomp;
        if (o->med[c] == FLUID) {
            double cf = o->pa[c], kap = rho * cf * cf;
            double wp = MDOT(0, 0), wm = MDOT(1, 1) + MDOT(2, 2);
            g[0] -= -wp / (rho * kap) + wm;       /* d(1/kappa)/drho = -1/(rho kappa), d rho/d rho = 1 */
            g[1] -= -2.0 * wp / (cf * kap);       /* d(1/kappa)/dc = -2/(c kappa) */
            ncomp = 1;
        } else {
            double lam = o->pa[c], muL = o->pb[c], lpm = lam + muL;
            double wv = MDOT(0, 0) + MDOT(1, 1);
            double dl[9] = {-1.0 / (4 * lpm * lpm), -1.0 / (4 * lpm * lpm), 0, -1.0 / (4 * lpm * lpm),
                            -1.0 / (4 * lpm * lpm), 0, 0, 0, 0};
            double dA = -(lam * lam + 2 * lam * muL + 2 * muL * muL) / (4 * muL * muL * lpm * lpm);
            double dB = lam * (lam + 2 * muL) / (4 * muL * muL * lpm * lpm);
            double dm[9] = {dA, dB, 0, dB, dA, 0, 0, 0, -1.0 / (2 * muL * muL)};
            double sl = 0, sm = 0;
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) {
                    double v = MDOT(2 + al, 2 + be);
                    sl += dl[al * 3 + be] * v;
                    sm += dm[al * 3 + be] * v;
                }
            g[0] -= wv;
            g[1] -= sl;
            g[2] -= sm;
            ncomp = 2;
        }
        #undef MDOT
        /* stabilisation: sum over faces of (Y_T - Y_F, w_T - W_F)_F, primal components */
        double stab = 0;
        int s = o->cptr[c], m = o->cptr[c + 1] - s;
        for (int t = 0; t < m; ++t) {
            int e = s + t, f = o->cf[e];
            const double *E = o->E + (size_t)e * N * N, *G = o->G + (size_t)e * N * nf, *MF = o->MF + (size_t)f * nf * nf;
            const double *yf = face_slice(o, YF, f, o->med[c], zero), *wf = face_slice(o, WF, f, o->med[c], zero);
            for (int cc = 0; cc < ncomp; ++cc) {
                const double *yt = yc + cc * N, *wt = wc + cc * N, *yfc = yf + cc * nf, *wfc = wf + cc * nf;
                double v = 0;
                for (int a = 0; a < N; ++a)
                    for (int b = 0; b < N; ++b) v += yt[a] * E[a * N + b] * wt[b];
                for (int a = 0; a < N; ++a)
                    for (int i = 0; i < nf; ++i) v -= yt[a] * G[a * nf + i] * wfc[i] + wt[a] * G[a * nf + i] * yfc[i];
                for (int i = 0; i < nf; ++i)
                    for (int l = 0; l < nf; ++l) v += yfc[i] * MF[i * nf + l] * wfc[l];
                stab += v;
            }
        }
        double tau = o->tau[c];
        if (o->med[c] == FLUID) {
            g[0] -= (-tau / rho) * stab;
            g[1] -= (-tau / o->pa[c]) * stab;
        } else {
            double l2m = o->pa[c] + 2 * o->pb[c];
            if (o->stab_speed == 0) {
                g[0] -= tau / (2 * rho) * stab;
                g[1] -= tau / (2 * l2m) * stab;
                g[2] -= tau / l2m * stab;
            } else {
                g[0] -= tau / (2 * rho) * stab;
                g[2] -= tau / (2 * o->pb[c]) * stab;
            }
        }
        for (int q = 0; q < 3; ++q) grad[3 * c + q] += g[q];
    }
    free(w); free(tmp); free(YF); free(WF);
}
