// Host setup: levels, active sets, surrogate faces, shifts, cell blocks,
// block inverses, transfer maps and the coarsest-level matrix.
//
// Paper references:
//  * hierarchy: p-levels p, p-1, ..., 1 on the finest mesh, then geometric
//    coarsening with p = 1 (Sec. 3, opening); every level has its own active
//    set and re-discretised operator (Sec. 4.3);
//  * active cells and surrogate boundary (Sec. 2.1); here a cell is active iff
//    phi(cell centre) < 0, a cheap surrogate of the volume-fraction rule that
//    Sec. 2.1 explicitly allows;
//  * cell blocks A_i = R_i A R_i^T (Sec. 3.1, local operator) inverted once
//    by LU with partial pivoting and reused at every smoothing step;
//  * shifts computed once per surrogate quadrature point per level (Sec. 4.2).
//
// The cell operator is written in reference units on a Cartesian cell of
// size h: A_K = h^(d-2) [ sum_k M x .. x T_k x .. x M + sum_surrogate faces S_f ]
// where M is the exact 1D mass matrix, T_k the 1D stiffness matrix plus the
// 1D face terms of the two faces normal to e_k (SIPG self terms on interior
// faces, unshifted Nitsche terms on surrogate faces), and S_f the part of a
// surrogate face's Nitsche terms that carries the shift.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "common.hpp"
#include "setup.hpp"

namespace sbm {

template <typename F>
static void parallel_for(long long n, F f) {
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (n < 64 || nt == 1) {
        for (long long i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<long long> next(0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (;;) {
                long long i = next.fetch_add(16);
                if (i >= n) break;
                long long e = std::min(n, i + 16);
                for (long long j = i; j < e; ++j) f(j);
            }
        });
    for (auto &t : th) t.join();
}

// 1D self operator for a direction with face types (t0 at xi = 0, t1 at xi = 1)
static void self_1d(const HostLevel &L, double alpha, int t0, int t1, double T[MAXN1][MAXN1]) {
    const Ref1D &r = L.ref;
    int n1 = r.n1;
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) {
            double v = r.K[a][b];
            for (int s = 0; s < 2; ++s) {
                double sg = s == 1 ? 1.0 : -1.0;
                int type = s == 0 ? t0 : t1;
                const double *e = r.e[s], *g = r.g[s];
                if (type == 0)
                    v += -0.5 * sg * (e[a] * g[b] + g[a] * e[b]) + L.sigF * e[a] * e[b];
                else
                    v += -sg * e[a] * g[b] - alpha * sg * g[a] * e[b] + L.sigG * e[a] * e[b];
            }
            T[a][b] = v;
        }
}

// unpack DoF index into per-direction node indices (x fastest)
static inline void unpack(int i, int n1, int d, int *idx) {
    for (int c = 0; c < d; ++c) {
        idx[c] = i % n1;
        i /= n1;
    }
}

// Kronecker-sum part of a cell block (volume + unshifted face terms)
static void kron_part(const HostLevel &L, const double Tk[3][MAXN1][MAXN1], double *D) {
    int nc = L.nc, n1 = L.n1, d = L.d;
    for (int i = 0; i < nc; ++i) {
        int ii[3];
        unpack(i, n1, d, ii);
        for (int j = 0; j < nc; ++j) {
            int jj[3];
            unpack(j, n1, d, jj);
            double v = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = Tk[k][ii[k]][jj[k]];
                for (int c = 0; c < d; ++c)
                    if (c != k) t *= L.ref.M[ii[c]][jj[c]];
                v += t;
            }
            D[i * nc + j] = v;
        }
    }
}

// shifted part of one surrogate face: D[i][j] += sum_q w_q A_q[i] E_q[j]
static void shift_part(const HostLevel &L, double alpha, int ext, int k, int s, const double *dhat,
                       double *D) {
    const Ref1D &r = L.ref;
    int d = L.d, n1 = L.n1, nc = L.nc, nf = L.nf;
    double sg = s == 1 ? 1.0 : -1.0;
    int tang[2], nt = 0;
    for (int c = 0; c < d; ++c)
        if (c != k) tang[nt++] = c;
    std::vector<double> A(nc), E(nc);
    for (int q = 0; q < nf; ++q) {
        int qq[2] = {q % n1, q / n1};
        double wq = 1.0, xi[3];
        xi[k] = (double)s;
        for (int t = 0; t < nt; ++t) {
            wq *= r.wq[qq[t]];
            xi[tang[t]] = r.gq[qq[t]];
        }
        const double *dq = dhat + (size_t)q * d;
        // shifted point basis values (ext = 1)
        double lv[3][MAXN1];
        if (ext == 1)
            for (int c = 0; c < d; ++c) lagrange(r.x, n1, xi[c] + dq[c], lv[c], nullptr);
        for (int i = 0; i < nc; ++i) {
            int ii[3];
            unpack(i, n1, d, ii);
            double tp = 1.0;  // product of tangential basis values at q
            for (int t = 0; t < nt; ++t) tp *= r.S[qq[t]][ii[tang[t]]];
            A[i] = (-alpha * sg * r.g[s][ii[k]] + L.sigG * r.e[s][ii[k]]) * tp;
            double e;
            if (ext == 0) {
                e = dq[k] * r.g[s][ii[k]] * tp;
                for (int t = 0; t < nt; ++t) {
                    int c = tang[t];
                    double v = r.e[s][ii[k]] * r.Sd[qq[t]][ii[c]];
                    for (int t2 = 0; t2 < nt; ++t2)
                        if (t2 != t) v *= r.S[qq[t2]][ii[tang[t2]]];
                    e += dq[c] * v;
                }
            } else {
                double pv = 1.0;
                for (int c = 0; c < d; ++c) pv *= lv[c][ii[c]];
                e = pv - r.e[s][ii[k]] * tp;
            }
            E[i] = e;
        }
        for (int i = 0; i < nc; ++i) {
            double ai = wq * A[i];
            if (ai == 0.0) continue;
            double *row = D + (size_t)i * nc;
            for (int j = 0; j < nc; ++j) row[j] += ai * E[j];
        }
    }
}

// In-place inverse by LU with partial pivoting.  Returns false if a pivot is
// below tol * max|D| (then D is left undefined).
bool invert(double *D, int n, double rel_tol, double reg) {
    double amax = 0.0;
    for (int i = 0; i < n * n; ++i) amax = std::max(amax, std::fabs(D[i]));
    if (reg > 0.0)
        for (int i = 0; i < n; ++i) D[i * n + i] += reg * amax;
    std::vector<double> LU(D, D + (size_t)n * n);
    std::vector<int> piv(n);
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(LU[(size_t)i * n + c]) > std::fabs(LU[(size_t)pr * n + c])) pr = i;
        if (!(std::fabs(LU[(size_t)pr * n + c]) > rel_tol * amax)) return false;
        piv[c] = pr;
        if (pr != c)
            for (int j = 0; j < n; ++j) std::swap(LU[(size_t)pr * n + j], LU[(size_t)c * n + j]);
        double inv = 1.0 / LU[(size_t)c * n + c];
        for (int i = c + 1; i < n; ++i) {
            double f = LU[(size_t)i * n + c] * inv;
            LU[(size_t)i * n + c] = f;
            if (f != 0.0)
                for (int j = c + 1; j < n; ++j) LU[(size_t)i * n + j] -= f * LU[(size_t)c * n + j];
        }
    }
    // solve for each column of the identity (rows permuted)
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
        for (int c = 0; c < n; ++c) std::swap(col[c], col[piv[c]]);
        for (int i = 0; i < n; ++i) {
            double acc = col[i];
            for (int k = 0; k < i; ++k) acc -= LU[(size_t)i * n + k] * col[k];
            col[i] = acc;
        }
        for (int i = n - 1; i >= 0; --i) {
            double acc = col[i];
            for (int k = i + 1; k < n; ++k) acc -= LU[(size_t)i * n + k] * col[k];
            col[i] = acc / LU[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) D[(size_t)i * n + j] = col[i];
    }
    return true;
}

void cell_block(const HostLevel &L, double alpha, int ext, int K, double *D) {
    int d = L.d;
    double Tk[3][MAXN1][MAXN1];
    for (int k = 0; k < d; ++k)
        self_1d(L, alpha, L.nbr[K * 2 * d + 2 * k] < 0, L.nbr[K * 2 * d + 2 * k + 1] < 0, Tk[k]);
    kron_part(L, Tk, D);
    for (int f = 0; f < 2 * d; ++f) {
        int nb = L.nbr[K * 2 * d + f];
        if (nb >= 0) continue;
        int rec = -nb - 1;
        std::vector<double> dhat((size_t)L.nf * d);
        for (size_t t = 0; t < dhat.size(); ++t) dhat[t] = L.shifts[(size_t)rec * L.nf * d + t] / L.h;
        shift_part(L, alpha, ext, f / 2, f % 2, dhat.data(), D);
    }
    double sc = std::pow(L.h, d - 2);
    for (int t = 0; t < L.nc * L.nc; ++t) D[t] *= sc;
}

void coupling_block(const HostLevel &L, int k, int s, double *C) {
    // test in K, trial in the neighbour across face (k, s)
    const Ref1D &r = L.ref;
    double Cp[MAXN1][MAXN1], C1[MAXN1][MAXN1];
    for (int a = 0; a < L.n1; ++a)
        for (int b = 0; b < L.n1; ++b)
            Cp[a][b] = -0.5 * r.e[1][a] * r.g[0][b] + 0.5 * r.g[1][a] * r.e[0][b] - L.sigF * r.e[1][a] * r.e[0][b];
    for (int a = 0; a < L.n1; ++a)
        for (int b = 0; b < L.n1; ++b) C1[a][b] = s == 1 ? Cp[a][b] : Cp[b][a];
    int nc = L.nc, n1 = L.n1, d = L.d;
    double sc = std::pow(L.h, d - 2);
    for (int i = 0; i < nc; ++i) {
        int ii[3];
        unpack(i, n1, d, ii);
        for (int j = 0; j < nc; ++j) {
            int jj[3];
            unpack(j, n1, d, jj);
            double t = C1[ii[k]][jj[k]];
            for (int c = 0; c < d; ++c)
                if (c != k) t *= r.M[ii[c]][jj[c]];
            C[i * nc + j] = sc * t;
        }
    }
}

// Volume-fraction rule (Sec. 2.1; Sec. 4.1 computes the fraction by cut-cell
// quadrature): the fraction is the share of the m^d cell-midpoint samples
// (cell split into m^d equal sub-cells) with phi < 0, and the cell is active
// iff it exceeds lambda (lambda = 1: every sample inside).  A cell whose
// centre and 2^d corners all lie on one side of Gamma is taken as wholly
// inside or outside without sampling.
static bool volume_fraction_active(const Geometry &g, const HostLevel &L, const int *mi, double lambda, int m) {
    const int d = L.d;
    double x[3];
    for (int c = 0; c < d; ++c) x[c] = L.lo + L.h * (mi[c] + 0.5);
    const bool in0 = g.phi(x) < 0.0;
    bool mixed = false;
    for (int v = 0; v < (1 << d) && !mixed; ++v) {
        for (int c = 0; c < d; ++c) x[c] = L.lo + L.h * (mi[c] + ((v >> c) & 1));
        mixed = (g.phi(x) < 0.0) != in0;
    }
    if (!mixed) return in0;
    long long total = 1, inside = 0;
    for (int c = 0; c < d; ++c) total *= m;
    for (long long s = 0; s < total; ++s) {
        long long t = s;
        for (int c = 0; c < d; ++c) {
            x[c] = L.lo + L.h * (mi[c] + ((t % m) + 0.5) / m);
            t /= m;
        }
        inside += g.phi(x) < 0.0;
    }
    if (lambda >= 1.0) return inside == total;
    return (double)inside > lambda * (double)total;
}

// Keep the k-core of the active cells' face-adjacency graph: drop every cell
// with fewer than k active face neighbours, and again for the neighbours that
// fall below k, until none is left to drop (the result does not depend on the
// order of removal).
static void prune_active(std::vector<char> &active, int n, int d, int k) {
    const long long ncell = (long long)active.size();
    long long stride[3] = {1, n, (long long)n * n};
    auto count = [&](long long lin) {
        int c = 0;
        long long t = lin;
        for (int a = 0; a < d; ++a) {
            const int m = (int)(t % n);
            t /= n;
            if (m > 0 && active[lin - stride[a]]) ++c;
            if (m < n - 1 && active[lin + stride[a]]) ++c;
        }
        return c;
    };
    std::vector<long long> queue;
    for (long long lin = 0; lin < ncell; ++lin)
        if (active[lin] && count(lin) < k) queue.push_back(lin);
    while (!queue.empty()) {
        const long long lin = queue.back();
        queue.pop_back();
        if (!active[lin]) continue;
        active[lin] = 0;
        long long t = lin;
        for (int a = 0; a < d; ++a) {
            const int m = (int)(t % n);
            t /= n;
            const long long nb[2] = {m > 0 ? lin - stride[a] : -1, m < n - 1 ? lin + stride[a] : -1};
            for (long long q : nb)
                if (q >= 0 && active[q] && count(q) < k) queue.push_back(q);
        }
    }
}

// Singular value decomposition of an n x n matrix by one-sided Jacobi
// rotations (Hestenes): on return the columns of W are sigma_j u_j and V holds
// the right singular vectors (D = W V^T), both column-major.
static void jacobi_svd(const double *D, int n, std::vector<double> &W, std::vector<double> &V) {
    W.assign((size_t)n * n, 0.0);
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) W[(size_t)j * n + i] = D[(size_t)i * n + j];
    for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int a = 0; a < n - 1; ++a)
            for (int b = a + 1; b < n; ++b) {
                double *wa = &W[(size_t)a * n], *wb = &W[(size_t)b * n];
                double al = 0, be = 0, ga = 0;
                for (int i = 0; i < n; ++i) {
                    al += wa[i] * wa[i];
                    be += wb[i] * wb[i];
                    ga += wa[i] * wb[i];
                }
                if (!(std::fabs(ga) > 1e-15 * std::sqrt(al * be))) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double tn = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + tn * tn), sn = cs * tn;
                for (int i = 0; i < n; ++i) {
                    const double p0 = wa[i], q0 = wb[i];
                    wa[i] = cs * p0 - sn * q0;
                    wb[i] = sn * p0 + cs * q0;
                }
                double *va = &V[(size_t)a * n], *vb = &V[(size_t)b * n];
                for (int i = 0; i < n; ++i) {
                    const double p0 = va[i], q0 = vb[i];
                    va[i] = cs * p0 - sn * q0;
                    vb[i] = sn * p0 + cs * q0;
                }
            }
        if (!rotated) break;
    }
}

static double smallest_singular_value(const double *D, int n) {
    std::vector<double> W, V;
    jacobi_svd(D, n, W, V);
    double smin = INFINITY;
    for (int j = 0; j < n; ++j) {
        double s2 = 0;
        for (int i = 0; i < n; ++i) s2 += W[(size_t)j * n + i] * W[(size_t)j * n + i];
        smin = std::min(smin, std::sqrt(s2));
    }
    return smin;
}

// Stabilised inverse of a cell block: B = sum_j v_j u_j^T / max(sigma_j, floor)
// (the exact inverse when every sigma_j >= floor).  Returns true if a singular
// value was raised.  B: n x n row-major.
static bool clipped_inverse(const double *D, int n, double floor_, double *B) {
    std::vector<double> W, V;
    jacobi_svd(D, n, W, V);
    bool clipped = false;
    for (int t = 0; t < n * n; ++t) B[t] = 0.0;
    for (int j = 0; j < n; ++j) {
        const double *w = &W[(size_t)j * n];
        double s2 = 0;
        for (int i = 0; i < n; ++i) s2 += w[i] * w[i];
        const double sg = std::sqrt(s2);
        if (!(sg > 0.0)) continue;
        if (sg < floor_) clipped = true;
        const double f = 1.0 / (sg * std::max(sg, floor_));   // u_j = w / sigma
        const double *v = &V[(size_t)j * n];
        for (int r = 0; r < n; ++r) {
            const double vr = v[r] * f;
            for (int c = 0; c < n; ++c) B[(size_t)r * n + c] += vr * w[c];
        }
    }
    return clipped;
}

int build_level(const Geometry &g, const sbm_options &o, int n, int p, bool finest_mesh, HostLevel &L,
                std::string &err) {
    const int d = g.dim;
    L.d = d;
    L.n = n;
    L.p = p;
    L.n1 = p + 1;
    L.nc = d == 2 ? L.n1 * L.n1 : L.n1 * L.n1 * L.n1;
    L.nf = d == 2 ? L.n1 : L.n1 * L.n1;
    L.lo = o.lo;
    L.h = (o.hi - o.lo) / n;
    L.ref = make_ref(p);
    const int pp = o.penalty_p > 0 ? o.penalty_p : p;
    L.sigF = o.c_F * (pp + 1) * (pp + 1);
    L.sigG = o.c_G * (pp + 1) * (pp + 1);
    long long ncell = 1;
    for (int c = 0; c < d; ++c) ncell *= n;
    // classification (centre rule) and red-black lexicographic order
    std::vector<char> active(ncell);
    parallel_for(ncell, [&](long long lin) {
        long long t = lin;
        int mi[3] = {0, 0, 0};
        double x[3];
        for (int c = 0; c < d; ++c) {
            mi[c] = (int)(t % n);
            x[c] = L.lo + L.h * (mi[c] + 0.5);
            t /= n;
        }
        if (o.lambda_frac > 0.0)
            active[lin] = volume_fraction_active(g, L, mi, o.lambda_frac, o.frac_m);
        else
            active[lin] = g.phi(x) < 0.0;
    });
    // the k-core rule shapes the finest mesh (all its p-levels); the
    // h-coarsened p = 1 levels keep the plain rule
    if (o.min_neighbours > 0 && finest_mesh) prune_active(active, n, d, o.min_neighbours);
    L.cell_of.assign(ncell, -1);
    L.cells.clear();
    for (int col = 0; col < 2; ++col)
        for (long long lin = 0; lin < ncell; ++lin) {
            if (!active[lin]) continue;
            long long t = lin;
            int mi[3], sum = 0;
            for (int c = 0; c < d; ++c) {
                mi[c] = (int)(t % n);
                sum += mi[c];
                t /= n;
            }
            if (sum % 2 != col) continue;
            L.cell_of[lin] = (int)(L.cells.size() / d);
            for (int c = 0; c < d; ++c) L.cells.push_back(mi[c]);
        }
    L.n_act = (int)(L.cells.size() / d);
    L.n_col0 = 0;
    for (int K = 0; K < L.n_act; ++K) {
        int sum = 0;
        for (int c = 0; c < d; ++c) sum += L.cells[K * d + c];
        if (sum % 2 == 0) L.n_col0++;
    }
    // neighbours and surrogate faces ordered by (cell, k, s)
    L.nbr.assign((size_t)L.n_act * 2 * d, -1);
    L.surr_cell.clear();
    L.surr_k.clear();
    L.surr_s.clear();
    for (int K = 0; K < L.n_act; ++K)
        for (int k = 0; k < d; ++k)
            for (int s = 0; s < 2; ++s) {
                int mi[3];
                for (int c = 0; c < d; ++c) mi[c] = L.cells[K * d + c];
                mi[k] += 2 * s - 1;
                int nb = -1;
                if (mi[k] >= 0 && mi[k] < n) {
                    long long lin = 0, st = 1;
                    for (int c = 0; c < d; ++c) {
                        lin += mi[c] * st;
                        st *= n;
                    }
                    nb = L.cell_of[lin];
                }
                if (nb < 0) {
                    nb = -(int)L.surr_cell.size() - 1;
                    L.surr_cell.push_back(K);
                    L.surr_k.push_back(k);
                    L.surr_s.push_back(s);
                }
                L.nbr[(size_t)K * 2 * d + 2 * k + s] = nb;
            }
    L.n_surr = (int)L.surr_cell.size();
    // closest points at the surrogate Gauss points
    L.shifts.assign((size_t)L.n_surr * L.nf * d, 0.0);
    std::atomic<int> bad(0);
    parallel_for(L.n_surr, [&](long long f) {
        int K = L.surr_cell[f], k = L.surr_k[f], s = L.surr_s[f];
        int tang[2], nt = 0;
        for (int c = 0; c < d; ++c)
            if (c != k) tang[nt++] = c;
        for (int q = 0; q < L.nf; ++q) {
            int qq[2] = {q % L.n1, q / L.n1};
            double x[3], y[3];
            x[k] = L.lo + L.h * (L.cells[K * d + k] + s);
            for (int t = 0; t < nt; ++t) x[tang[t]] = L.lo + L.h * (L.cells[K * d + tang[t]] + L.ref.gq[qq[t]]);
            if (!g.closest(x, y)) {
                bad++;
                continue;
            }
            for (int c = 0; c < d; ++c) L.shifts[((size_t)f * L.nf + q) * d + c] = y[c] - x[c];
        }
    });
    if (bad) {
        err = "closest-point search failed";
        return SBM_EGEOM;
    }
    // boundary cells
    L.bnd_of.assign(L.n_act, -1);
    L.bnd_cells.clear();
    for (int K = 0; K < L.n_act; ++K) {
        bool b = false;
        for (int f = 0; f < 2 * d; ++f) b |= L.nbr[(size_t)K * 2 * d + f] < 0;
        if (b) {
            L.bnd_of[K] = (int)L.bnd_cells.size();
            L.bnd_cells.push_back(K);
        }
    }
    L.n_bnd = (int)L.bnd_cells.size();
    return build_blocks(L, o, err);
}

int build_blocks(HostLevel &L, const sbm_options &o, std::string &err) {
    const int d = L.d;
    // blocks and inverses
    const int nc = L.nc;
    const double reg = o.allow_singular ? 1e-10 : 0.0;
    L.Dint.assign((size_t)nc * nc, 0.0);
    {
        double Tk[3][MAXN1][MAXN1];
        for (int k = 0; k < d; ++k) self_1d(L, o.alpha, 0, 0, Tk[k]);
        kron_part(L, Tk, L.Dint.data());
        double sc = std::pow(L.h, d - 2);
        for (auto &v : L.Dint) v *= sc;
    }
    L.Bint = L.Dint;
    if (!invert(L.Bint.data(), nc, 1e-12, reg)) {
        err = "singular interior block";
        return SBM_ESINGULAR;
    }
    L.Dbnd.assign((size_t)L.n_bnd * nc * nc, 0.0);
    L.Bbnd.assign((size_t)L.n_bnd * nc * nc, 0.0);
    std::atomic<int> sing(0);
    parallel_for(L.n_bnd, [&](long long b) {
        double *D = &L.Dbnd[(size_t)b * nc * nc];
        cell_block(L, o.alpha, o.ext, L.bnd_cells[b], D);
        double *B = &L.Bbnd[(size_t)b * nc * nc];
        std::memcpy(B, D, sizeof(double) * nc * nc);
        if (!invert(B, nc, 1e-12, reg)) sing++;
    });
    if (sing) {
        err = "singular boundary-cell block (set allow_singular to shift it)";
        return SBM_ESINGULAR;
    }
    L.n_clipped = 0;
    L.clipped.assign(L.n_bnd, 0);
    if (o.stab > 0.0) {
        // floor = stab * (smallest singular value of the interior block); a
        // block needs the SVD only if 1 / |B_K|_F < floor (sigma_min >= 1/|B|_F)
        const double floor_ = o.stab * smallest_singular_value(L.Dint.data(), nc);
        std::atomic<int> nclip(0);
        parallel_for(L.n_bnd, [&](long long b) {
            double *B = &L.Bbnd[(size_t)b * nc * nc];
            double f2 = 0;
            for (int t = 0; t < nc * nc; ++t) f2 += B[t] * B[t];
            if (1.0 / std::sqrt(f2) >= floor_) return;
            if (clipped_inverse(&L.Dbnd[(size_t)b * nc * nc], nc, floor_, B)) {
                L.clipped[b] = 1;
                nclip++;
            }
        });
        L.n_clipped = nclip;
    }
    return SBM_OK;
}

void build_transfer(const HostLevel &Lc, HostLevel &Lf) {
    const int d = Lf.d;
    Lf.ratio = Lf.n / Lc.n;
    const int nch = Lf.ratio == 2 ? (1 << d) : 1;
    Lf.parent.assign(Lf.n_act, -1);
    Lf.childpos.assign(Lf.n_act, 0);
    Lf.children.assign((size_t)Lc.n_act * nch, -1);
    for (int K = 0; K < Lf.n_act; ++K) {
        long long lin = 0, st = 1;
        int bits = 0;
        for (int c = 0; c < d; ++c) {
            int m = Lf.cells[K * d + c];
            lin += (m / Lf.ratio) * st;
            st *= Lc.n;
            if (Lf.ratio == 2) bits |= (m % 2) << c;
        }
        int pc = Lc.cell_of[lin];
        Lf.parent[K] = pc;
        Lf.childpos[K] = bits;
        if (pc >= 0) Lf.children[(size_t)pc * nch + bits] = K;
    }
}

void embedding_1d(const HostLevel &Lc, const HostLevel &Lf, double P1[2][MAXN1][MAXN1]) {
    int ratio = Lf.n / Lc.n;
    for (int o = 0; o < 2; ++o)
        for (int a = 0; a < Lf.n1; ++a) {
            double xc = ratio == 2 ? 0.5 * (o + Lf.ref.x[a]) : Lf.ref.x[a];
            double v[MAXN1];
            lagrange(Lc.ref.x, Lc.n1, xc, v, nullptr);
            for (int b = 0; b < MAXN1; ++b) P1[o][a][b] = b < Lc.n1 ? v[b] : 0.0;
        }
}

int coarse_matrix(const HostLevel &L, double alpha, int ext, std::vector<double> &A) {
    const int nc = L.nc, d = L.d;
    const long long nd = (long long)L.n_act * nc;
    A.assign((size_t)(nd * nd), 0.0);
    std::vector<double> D((size_t)nc * nc), C((size_t)nc * nc);
    for (int K = 0; K < L.n_act; ++K) {
        if (L.bnd_of[K] >= 0)
            std::memcpy(D.data(), &L.Dbnd[(size_t)L.bnd_of[K] * nc * nc], sizeof(double) * nc * nc);
        else
            D = L.Dint;
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) A[(size_t)(K * nc + i) * nd + K * nc + j] = D[i * nc + j];
        for (int f = 0; f < 2 * d; ++f) {
            int nb = L.nbr[(size_t)K * 2 * d + f];
            if (nb < 0) continue;
            coupling_block(L, f / 2, f % 2, C.data());
            for (int i = 0; i < nc; ++i)
                for (int j = 0; j < nc; ++j) A[(size_t)(K * nc + i) * nd + nb * nc + j] = C[i * nc + j];
        }
    }
    (void)alpha;
    (void)ext;
    return SBM_OK;
}

void make_kref(const HostLevel &L, const sbm_options &o, double omega, KRef<double> &k) {
    std::memset(&k, 0, sizeof(k));
    const Ref1D &r = L.ref;
    for (int a = 0; a < MAXN1; ++a)
        for (int b = 0; b < MAXN1; ++b) {
            k.M[a][b] = r.M[a][b];
            k.S[a][b] = r.S[a][b];
            k.Sd[a][b] = r.Sd[a][b];
        }
    for (int v = 0; v < 4; ++v) {
        double T[MAXN1][MAXN1] = {};
        self_1d(L, o.alpha, v & 1, (v >> 1) & 1, T);
        for (int a = 0; a < MAXN1; ++a)
            for (int b = 0; b < MAXN1; ++b) k.Tv[v][a][b] = T[a][b];
    }
    for (int a = 0; a < MAXN1; ++a) {
        k.w[a] = r.wq[a];
        k.gq[a] = r.gq[a];
        k.g[0][a] = r.g[0][a];
        k.g[1][a] = r.g[1][a];
        k.x[a] = r.x[a];
    }
    for (int a = 0; a <= L.p; ++a) {
        double den = 1.0;
        for (int b = 0; b <= L.p; ++b)
            if (b != a) den *= r.x[a] - r.x[b];
        k.bw[a] = 1.0 / den;
    }
    k.sigF = L.sigF;
    k.sigG = L.sigG;
    k.alpha = o.alpha;
    k.scale = std::pow(L.h, L.d - 2);
    k.omega = omega;
    k.ext = o.ext;
}

}  // namespace sbm
