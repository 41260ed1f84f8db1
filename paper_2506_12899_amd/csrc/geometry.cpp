// Level sets and closest-point projection (paper, Sec. 4.1 and Sec. 4.2).
//
// Omega = {phi < 0}.  For each surrogate quadrature point x~ the nearest point
// x of Gamma = {phi = 0} is found once at setup; the shift is d = x - x~.
//  * union of balls: exact.  The nearest point of the union's boundary is one
//    of: the radial projection onto a sphere, the nearest point of a pairwise
//    intersection circle (2D: one of the two intersection points), or (3D) a
//    point common to three spheres; candidates strictly inside another ball
//    (by more than 1e-12) are discarded, the nearest survivor wins and ties go
//    to the first in that enumeration order.
//  * 2D star r(t) = r0 + a sin(k t): the squared distance is sampled at 4096
//    equispaced t; the best sample (smallest t on ties) seeds a bracketed
//    Newton iteration on the derivative.
//  * callback level set and ellipsoid (phi = |diag(1/a) R^T (x - c)|^2 - 1):
//    Newton on the stationarity conditions of the Lagrangian
//    |x - x~|^2 + mu phi(x) (Sec. 4.2), started from the first-order
//    projection x~ - phi grad phi / |grad phi|^2.
#include <cmath>
#include <limits>

#include "common.hpp"

namespace sbm {

static const double kInsideTol = 1e-12;

static double norm(const double *v, int d) {
    double s = 0;
    for (int i = 0; i < d; ++i) s += v[i] * v[i];
    return std::sqrt(s);
}

double Geometry::phi(const double *x) const {
    if (kind == SBM_GEOM_BALLS) {
        double best = std::numeric_limits<double>::infinity();
        int m = (int)radii.size();
        for (int j = 0; j < m; ++j) {
            double v[3];
            for (int c = 0; c < dim; ++c) v[c] = x[c] - centers[j * dim + c];
            double s = norm(v, dim) - radii[j];
            if (s < best) best = s;
        }
        return best;
    }
    if (kind == SBM_GEOM_STAR2D) {
        double t = std::atan2(x[1], x[0]);
        return std::sqrt(x[0] * x[0] + x[1] * x[1]) - (r0 + a * std::sin(k * t));
    }
    return lphi(x);
}

// ellipsoid: phi(x) = |diag(1/a) R^T (x - c)|^2 - 1
static void ell_local(const Geometry &g, const double *x, double *y) {
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += g.rot[c * 3 + i] * (x[c] - g.centers[c]);
        y[i] = s;
    }
}

double Geometry::lphi(const double *x) const {
    if (kind != SBM_GEOM_ELLIPSOID) return cb_phi(x, user);
    double y[3], s = 0.0;
    ell_local(*this, x, y);
    for (int i = 0; i < 3; ++i) s += (y[i] / radii[i]) * (y[i] / radii[i]);
    return s - 1.0;
}

void Geometry::lgrad(const double *x, double *gr) const {
    if (kind != SBM_GEOM_ELLIPSOID) {
        cb_grad(x, gr, user);
        return;
    }
    double y[3];
    ell_local(*this, x, y);
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += rot[c * 3 + i] * 2.0 * y[i] / (radii[i] * radii[i]);
        gr[c] = s;
    }
}

void Geometry::lhess(const double *x, double *H) const {
    if (kind != SBM_GEOM_ELLIPSOID) {
        cb_hess(x, H, user);
        return;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += rot[a * 3 + i] * rot[b * 3 + i] * 2.0 / (radii[i] * radii[i]);
            H[a * 3 + b] = s;
        }
}

namespace {

struct BallsCP {
    const Geometry &g;
    int d, m;
    explicit BallsCP(const Geometry &geo) : g(geo), d(geo.dim), m((int)geo.radii.size()) {}
    const double *c(int j) const { return &g.centers[j * d]; }
    double r(int j) const { return g.radii[j]; }

    bool outside_others(const double *y, int s0, int s1, int s2) const {
        for (int j = 0; j < m; ++j) {
            if (j == s0 || j == s1 || j == s2) continue;
            double v[3];
            for (int q = 0; q < d; ++q) v[q] = y[q] - c(j)[q];
            if (norm(v, d) < r(j) - kInsideTol) return false;
        }
        return true;
    }

    void consider(const double *x, const double *y, double &best, double *out) const {
        double v[3];
        for (int q = 0; q < d; ++q) v[q] = y[q] - x[q];
        double dist = norm(v, d);
        if (dist < best) {  // strict: ties keep the earlier candidate
            best = dist;
            for (int q = 0; q < d; ++q) out[q] = y[q];
        }
    }

    bool closest(const double *x, double *out) const {
        double best = std::numeric_limits<double>::infinity();
        // radial projections
        for (int j = 0; j < m; ++j) {
            double v[3];
            for (int q = 0; q < d; ++q) v[q] = x[q] - c(j)[q];
            double nv = norm(v, d);
            if (nv == 0.0) {
                for (int q = 0; q < d; ++q) v[q] = 0.0;
                v[0] = 1.0;
                nv = 1.0;
            }
            double y[3];
            for (int q = 0; q < d; ++q) y[q] = c(j)[q] + r(j) * v[q] / nv;
            if (outside_others(y, j, -1, -1)) consider(x, y, best, out);
        }
        // pairwise intersections
        for (int j = 0; j < m; ++j)
            for (int k = j + 1; k < m; ++k) {
                double e[3];
                for (int q = 0; q < d; ++q) e[q] = c(k)[q] - c(j)[q];
                double L = norm(e, d);
                if (!(std::fabs(r(j) - r(k)) < L && L < r(j) + r(k))) continue;
                for (int q = 0; q < d; ++q) e[q] /= L;
                double aa = (L * L + r(j) * r(j) - r(k) * r(k)) / (2.0 * L);
                double rho = std::sqrt(std::fmax(r(j) * r(j) - aa * aa, 0.0));
                double mc[3];
                for (int q = 0; q < d; ++q) mc[q] = c(j)[q] + aa * e[q];
                if (d == 2) {
                    double perp[2] = {-e[1], e[0]};
                    for (int sgn = 0; sgn < 2; ++sgn) {
                        double y[2];
                        double s = sgn == 0 ? 1.0 : -1.0;
                        for (int q = 0; q < 2; ++q) y[q] = mc[q] + s * rho * perp[q];
                        if (outside_others(y, j, k, -1)) consider(x, y, best, out);
                    }
                } else {
                    double w[3], xe = 0.0;
                    for (int q = 0; q < 3; ++q) xe += (x[q] - mc[q]) * e[q];
                    for (int q = 0; q < 3; ++q) w[q] = (x[q] - mc[q]) - xe * e[q];
                    double nw = norm(w, 3);
                    if (nw == 0.0) {
                        int ax = 0;
                        for (int q = 1; q < 3; ++q)
                            if (std::fabs(e[q]) < std::fabs(e[ax])) ax = q;
                        double t[3] = {0, 0, 0};
                        t[ax] = 1.0;
                        double te = e[ax];
                        for (int q = 0; q < 3; ++q) w[q] = t[q] - te * e[q];
                        nw = norm(w, 3);
                    }
                    double y[3];
                    for (int q = 0; q < 3; ++q) y[q] = mc[q] + rho * w[q] / nw;
                    if (outside_others(y, j, k, -1)) consider(x, y, best, out);
                }
            }
        // triple points (3D)
        if (d == 3)
            for (int j = 0; j < m; ++j)
                for (int k = j + 1; k < m; ++k)
                    for (int l = k + 1; l < m; ++l) {
                        double y[2][3];
                        int cnt = triple(j, k, l, y);
                        for (int t = 0; t < cnt; ++t)
                            if (outside_others(y[t], j, k, l)) consider(x, y[t], best, out);
                    }
        return std::isfinite(best);
    }

    static void cross(const double *u, const double *v, double *w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    }
    static double dot3(const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

    int triple(int j, int k, int l, double y[2][3]) const {
        const double *c1 = c(j), *c2 = c(k), *c3 = c(l);
        double r1 = r(j), r2 = r(k), r3 = r(l);
        double a2[3], a3[3];
        for (int q = 0; q < 3; ++q) {
            a2[q] = 2.0 * (c2[q] - c1[q]);
            a3[q] = 2.0 * (c3[q] - c1[q]);
        }
        double b2 = r1 * r1 - r2 * r2 + dot3(c2, c2) - dot3(c1, c1);
        double b3 = r1 * r1 - r3 * r3 + dot3(c3, c3) - dot3(c1, c1);
        double u[3];
        cross(a2, a3, u);
        double nu = dot3(u, u);
        if (nu < 1e-30) return 0;
        double t1[3], t2[3], y0[3];
        cross(a3, u, t1);
        cross(u, a2, t2);
        for (int q = 0; q < 3; ++q) y0[q] = (b2 * t1[q] + b3 * t2[q]) / nu;
        double s = std::sqrt(nu), uu[3];
        for (int q = 0; q < 3; ++q) uu[q] = u[q] / s;
        double w[3];
        for (int q = 0; q < 3; ++q) w[q] = y0[q] - c1[q];
        double bq = dot3(w, uu), cq = dot3(w, w) - r1 * r1;
        double disc = bq * bq - cq;
        if (disc < 0.0) return 0;
        double sd = std::sqrt(disc);
        for (int q = 0; q < 3; ++q) {
            y[0][q] = y0[q] + (-bq - sd) * uu[q];
            y[1][q] = y0[q] + (-bq + sd) * uu[q];
        }
        return 2;
    }
};

// squared distance to the star curve and its first two theta-derivatives
void star_F(const Geometry &g, const double *x, double th, double &F, double &F1, double &F2) {
    double r = g.r0 + g.a * std::sin(g.k * th);
    double r1 = g.a * g.k * std::cos(g.k * th);
    double r2 = -g.a * g.k * g.k * std::sin(g.k * th);
    double c = std::cos(th), s = std::sin(th);
    double xe = x[0] * c + x[1] * s;
    double xe1 = -x[0] * s + x[1] * c;
    F = x[0] * x[0] + x[1] * x[1] - 2.0 * r * xe + r * r;
    F1 = -2.0 * r1 * xe - 2.0 * r * xe1 + 2.0 * r * r1;
    F2 = -2.0 * r2 * xe - 4.0 * r1 * xe1 + 2.0 * r * xe + 2.0 * r1 * r1 + 2.0 * r * r2;
}

bool star_closest(const Geometry &g, const double *x, double *y) {
    const int ns = 4096;
    int best = 0;
    double bestF = std::numeric_limits<double>::infinity();
    for (int m = 0; m < ns; ++m) {
        double th = 2.0 * M_PI * m / ns, F, F1, F2;
        star_F(g, x, th, F, F1, F2);
        if (F < bestF) {
            bestF = F;
            best = m;
        }
    }
    double dth = 2.0 * M_PI / ns;
    double t = 2.0 * M_PI * best / ns;
    double lo = t - dth, hi = t + dth;
    for (int it = 0; it < 100; ++it) {
        double F, F1, F2;
        star_F(g, x, t, F, F1, F2);
        if (std::fabs(F1) < 1e-15) break;
        if (F1 > 0.0) hi = t; else lo = t;
        double tn = F2 > 0.0 ? t - F1 / F2 : 0.5 * (lo + hi);
        if (!(lo < tn && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == t || hi - lo < 1e-16) {
            t = tn;
            break;
        }
        t = tn;
    }
    double r = g.r0 + g.a * std::sin(g.k * t);
    y[0] = r * std::cos(t);
    y[1] = r * std::sin(t);
    return std::isfinite(y[0]) && std::isfinite(y[1]);
}

bool newton_closest(const Geometry &g, const double *xt, double *y) {
    const int d = g.dim;
    double x[3], gr[3], H[9];
    double f = g.lphi(xt);
    g.lgrad(xt, gr);
    double gg = 0;
    for (int c = 0; c < d; ++c) gg += gr[c] * gr[c];
    if (!(gg > 0)) return false;
    for (int c = 0; c < d; ++c) x[c] = xt[c] - f * gr[c] / gg;
    g.lgrad(x, gr);
    gg = 0;
    double dg = 0;
    for (int c = 0; c < d; ++c) {
        gg += gr[c] * gr[c];
        dg += (x[c] - xt[c]) * gr[c];
    }
    double mu = -2.0 * dg / gg;
    for (int it = 0; it < 100; ++it) {
        f = g.lphi(x);
        g.lgrad(x, gr);
        g.lhess(x, H);
        double res[4], rn = 0;
        for (int c = 0; c < d; ++c) {
            res[c] = 2.0 * (x[c] - xt[c]) + mu * gr[c];
            rn += res[c] * res[c];
        }
        res[d] = f;
        if (std::fabs(f) < 1e-14 && std::sqrt(rn) < 1e-13) break;
        // J = [[2I + mu H, g], [g^T, 0]]; solve J s = -res by Gaussian elimination
        int m = d + 1;
        double J[4][5];
        for (int i = 0; i < d; ++i) {
            for (int j = 0; j < d; ++j) J[i][j] = (i == j ? 2.0 : 0.0) + mu * H[i * d + j];
            J[i][d] = gr[i];
            J[i][m] = -res[i];
        }
        for (int j = 0; j < d; ++j) J[d][j] = gr[j];
        J[d][d] = 0.0;
        J[d][m] = -res[d];
        for (int col = 0; col < m; ++col) {
            int piv = col;
            for (int i = col + 1; i < m; ++i)
                if (std::fabs(J[i][col]) > std::fabs(J[piv][col])) piv = i;
            if (J[piv][col] == 0.0) return false;
            if (piv != col)
                for (int j = 0; j <= m; ++j) std::swap(J[piv][j], J[col][j]);
            for (int i = col + 1; i < m; ++i) {
                double fct = J[i][col] / J[col][col];
                for (int j = col; j <= m; ++j) J[i][j] -= fct * J[col][j];
            }
        }
        double s[4];
        for (int i = m - 1; i >= 0; --i) {
            double acc = J[i][m];
            for (int j = i + 1; j < m; ++j) acc -= J[i][j] * s[j];
            s[i] = acc / J[i][i];
        }
        for (int c = 0; c < d; ++c) x[c] += s[c];
        mu += s[d];
    }
    for (int c = 0; c < d; ++c) y[c] = x[c];
    return std::fabs(g.lphi(x)) < 1e-10;
}

}  // namespace

bool Geometry::closest(const double *x, double *y) const {
    if (kind == SBM_GEOM_BALLS) return BallsCP(*this).closest(x, y);
    if (kind == SBM_GEOM_STAR2D) return star_closest(*this, x, y);
    return newton_closest(*this, x, y);
}

}  // namespace sbm
