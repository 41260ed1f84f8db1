// 1D reference element on [0, 1]: GLL nodes, Gauss rule, Lagrange basis.
//
// Nodal Lagrange basis on tensor-product cells (paper, Sec. 2.2).  The node
// set is the Gauss-Lobatto one (closed forms for p <= 3) and the quadrature is
// the (p+1)-point Gauss-Legendre rule, computed here by Newton's method on the
// Legendre polynomial.
#include <cmath>

#include "common.hpp"

namespace sbm {

void gauss_rule(int nq, double *x, double *w) {
    // roots of P_nq on [-1, 1] by Newton from the Chebyshev guesses, then mapped to [0, 1]
    for (int i = 0; i < nq; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= nq; ++k) {
                double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (nq == 1) { p1 = t; p0 = 1.0; }
            dp = nq * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        // recompute derivative at the converged root for the weight
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= nq; ++k) {
            double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        if (nq == 1) { p1 = t; p0 = 1.0; }
        dp = nq * (t * p1 - p0) / (t * t - 1.0);
        double wt = 2.0 / ((1.0 - t * t) * dp * dp);
        // ascending order on [0, 1]
        x[nq - 1 - i] = 0.5 * (t + 1.0);
        w[nq - 1 - i] = 0.5 * wt;
    }
}

void lagrange(const double *nodes, int n1, double x, double *v, double *dv) {
    for (int a = 0; a < n1; ++a) {
        double den = 1.0, val = 1.0, der = 0.0;
        for (int b = 0; b < n1; ++b) {
            if (b == a) continue;
            den *= nodes[a] - nodes[b];
            // product rule: der = der * (x - x_b) + val ; val *= (x - x_b)
            der = der * (x - nodes[b]) + val;
            val *= x - nodes[b];
        }
        v[a] = val / den;
        if (dv) dv[a] = der / den;
    }
}

Ref1D make_ref(int p) {
    Ref1D r;
    r.p = p;
    r.n1 = p + 1;
    if (p == 1) {
        r.x[0] = 0.0; r.x[1] = 1.0;
    } else if (p == 2) {
        r.x[0] = 0.0; r.x[1] = 0.5; r.x[2] = 1.0;
    } else {
        const double s = 1.0 / std::sqrt(5.0);
        r.x[0] = 0.0; r.x[1] = 0.5 * (1.0 - s); r.x[2] = 0.5 * (1.0 + s); r.x[3] = 1.0;
    }
    gauss_rule(r.n1, r.gq, r.wq);
    for (int q = 0; q < r.n1; ++q) lagrange(r.x, r.n1, r.gq[q], r.S[q], r.Sd[q]);
    for (int a = 0; a < r.n1; ++a)
        for (int b = 0; b < r.n1; ++b) {
            double m = 0.0, k = 0.0;
            for (int q = 0; q < r.n1; ++q) {
                m += r.wq[q] * r.S[q][a] * r.S[q][b];
                k += r.wq[q] * r.Sd[q][a] * r.Sd[q][b];
            }
            r.M[a][b] = m;
            r.K[a][b] = k;
        }
    lagrange(r.x, r.n1, 0.0, r.e[0], r.g[0]);
    lagrange(r.x, r.n1, 1.0, r.e[1], r.g[1]);
    return r;
}

}  // namespace sbm
