// Initial states given by a field in closed form, L2-projected onto the orthonormal cell bases on
// the host (float64): the Ricker-shaped initial field of eq. ricker_ic (Sec. 5.2).
#pragma once

#include <cmath>
#include <vector>

namespace hho {

// Gauss-Legendre rule of n points on [0, 1] (Newton iteration on the Legendre polynomial).
inline void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 1; m < n; ++m) {
                const double p2 = ((2.0 * m + 1.0) * z * p1 - m * p0) / (m + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2 / ((1 - z^2) P_n'(z)^2) on [-1, 1], halved
    }
}

// Quadrature over a polygon: the fan of triangles (centre, v_i, v_{i+1}), each mapped from the
// unit square by the collapsed (Duffy) map with n x n Gauss-Legendre points; f(x, y, weight).
template <typename F>
void polygon_quadrature(const double *xy, const int *vtx, int nv, double cx, double cy, int n, F &&f) {
    std::vector<double> g, gw;
    gauss_legendre01(n, g, gw);
    for (int e = 0; e < nv; ++e) {
        const double ax = xy[2 * vtx[e]], ay = xy[2 * vtx[e] + 1];
        const double bx = xy[2 * vtx[(e + 1) % nv]], by = xy[2 * vtx[(e + 1) % nv] + 1];
        // x = c + s [(a - c) + t (b - a)],  |dx / d(s, t)| = s |det(a - c, b - a)|
        const double ux = ax - cx, uy = ay - cy, vx = bx - ax, vy = by - ay;
        const double det = std::fabs(ux * vy - uy * vx);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double s = g[i], t = g[j];
                f(cx + s * (ux + t * vx), cy + s * (uy + t * vy), gw[i] * gw[j] * s * det);
            }
    }
}

// The field of eq. ricker_ic: g = theta exp(-pi^2 r^2 / lambda^2), r the distance to (xc, yc).
//   field 1: the velocity m_0 = g (x - xc, y - yc) as printed (the fluid's m and the solid's v);
//   field 0: the pressure pulse g (the fluid's p) of the granite-water case, which takes the
//            field "from the right-hand side" of the equation as a scalar pulse (its amplitude).
struct RickerIC {
    double xc, yc, theta, lambda;
    int field;
    double g(double x, double y) const {
        const double r2 = (x - xc) * (x - xc) + (y - yc) * (y - yc);
        return theta * std::exp(-M_PI * M_PI * r2 / (lambda * lambda));
    }
};

// Coefficients of the L2 projection of eq. ricker_ic on one cell with an orthonormal basis:
// out[comp * nb + a] = (f_comp, phi_a)_T for the components of the cell's layout that the field
// sets (fluid [p | m_x | m_y], solid [v_x | v_y | s...]; `vel` = offset of the velocity block and
// nb_p / nb_v the number of basis functions of the pressure / velocity fields).  eval(x, y, phi)
// evaluates the cell's basis (at least max(nb_p, nb_v) functions).
template <typename E>
void project_ricker_cell(const RickerIC &ic, const double *xy, const int *vtx, int nv, double cx, double cy,
                         bool fluid, int nb_p, int nb_v, int nbasis, E &&eval, double *out) {
    std::vector<double> phi(nbasis);
    const int nq = 12;
    polygon_quadrature(xy, vtx, nv, cx, cy, nq, [&](double x, double y, double w) {
        const double g = ic.g(x, y) * w;
        eval(x, y, phi.data());
        if (ic.field == 0) {
            if (fluid)
                for (int a = 0; a < nb_p; ++a) out[a] += g * phi[a];
        } else {
            const int vel = fluid ? nb_p : 0;  // fluid: m after p; solid: v first
            for (int a = 0; a < nb_v; ++a) {
                out[vel + a] += g * (x - ic.xc) * phi[a];
                out[vel + nb_v + a] += g * (y - ic.yc) * phi[a];
            }
        }
    });
}

}  // namespace hho
