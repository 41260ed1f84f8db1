// Internal data structures shared by the host setup, the kernels and the solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sbm.h"

namespace sbm {

constexpr int MAXN1 = 4;  // p <= 3

// ---------------------------------------------------------------------------
// 1D reference element on [0, 1] (host, double): Gauss-Lobatto nodes, the
// (p+1)-point Gauss rule, Lagrange values/derivatives at the Gauss points and
// the exact 1D mass and stiffness matrices.
struct Ref1D {
    int p = 1, n1 = 2;
    double x[MAXN1] = {};             // GLL nodes
    double gq[MAXN1] = {}, wq[MAXN1] = {};
    double S[MAXN1][MAXN1] = {};      // S[q][a]  = l_a(gq[q])
    double Sd[MAXN1][MAXN1] = {};     // Sd[q][a] = l_a'(gq[q])
    double M[MAXN1][MAXN1] = {};      // sum_q w_q l_a l_b
    double K[MAXN1][MAXN1] = {};      // sum_q w_q l_a' l_b'
    double e[2][MAXN1] = {};          // l_a(0), l_a(1)
    double g[2][MAXN1] = {};          // l_a'(0), l_a'(1)
};
Ref1D make_ref(int p);
void lagrange(const double *nodes, int n1, double x, double *v, double *dv);
void gauss_rule(int nq, double *x, double *w);

// ---------------------------------------------------------------------------
// Reference data handed to the kernels by value (kernel-argument segment).
// Everything is in reference units; the physical operator is scale * (...)
// with scale = h^(d-2).
template <typename T>
struct KRef {
    T M[MAXN1][MAXN1];
    T Tv[4][MAXN1][MAXN1];  // 1D self operator per face-type pair (low + 2*high), type 1 = surrogate
    T S[MAXN1][MAXN1];
    T Sd[MAXN1][MAXN1];
    T w[MAXN1];
    T gq[MAXN1];
    T g[2][MAXN1];
    T x[MAXN1];
    T bw[MAXN1];            // barycentric weights 1 / prod_{b != a} (x_a - x_b) of the nodes x
    T sigF, sigG, alpha, scale, omega;
    int ext;
};

// ---------------------------------------------------------------------------
struct Geometry {
    int dim = 2, kind = SBM_GEOM_BALLS;
    std::vector<double> centers, radii;
    double r0 = 0, a = 0;
    int k = 0;
    double (*cb_phi)(const double *, void *) = nullptr;
    void (*cb_grad)(const double *, double *, void *) = nullptr;
    void (*cb_hess)(const double *, double *, void *) = nullptr;
    void *user = nullptr;

    std::vector<double> rot;     // ellipsoid: 3x3 row-major, columns = principal axes

    double phi(const double *x) const;
    // nearest point of Gamma to x; returns false if the search failed
    bool closest(const double *x, double *y) const;
    // smooth level sets (callback, ellipsoid): value, gradient, Hessian
    double lphi(const double *x) const;
    void lgrad(const double *x, double *g) const;
    void lhess(const double *x, double *H) const;
};

// ---------------------------------------------------------------------------
// Host-side description of one multigrid level.
struct HostLevel {
    int d = 2, n = 0, p = 1, n1 = 2, nc = 4, nf = 2;
    double lo = -1, h = 0;
    int n_act = 0, n_col0 = 0;
    std::vector<int> cells;      // n_act * d, DoF order
    std::vector<int> cell_of;    // n^d -> active index or -1
    std::vector<int> nbr;        // n_act * 2d: >= 0 neighbour, < 0: -(surrogate face + 1)
    int n_surr = 0;
    std::vector<int> surr_cell, surr_k, surr_s;
    std::vector<double> shifts;  // n_surr * nf * d, physical d = x - x~
    int n_bnd = 0;
    std::vector<int> bnd_of;     // n_act -> boundary block index or -1
    std::vector<int> bnd_cells;  // n_bnd
    std::vector<double> Dint, Bint;  // nc*nc row-major, B = D^{-1}
    std::vector<double> Dbnd, Bbnd;  // n_bnd * nc*nc
    int n_clipped = 0;            // boundary blocks whose inverse the stabilisation changed
    std::vector<char> clipped;    // n_bnd: 1 for those blocks
    // relation to the next coarser level (absent on level 0)
    int ratio = 1;                // 2 = h-transfer, 1 = p-transfer
    std::vector<int> parent;      // n_act -> coarse active index or -1
    std::vector<int> childpos;    // n_act -> child offset bits (bit c = offset in direction c)
    std::vector<int> children;    // n_act_coarse * 2^d (or 1) fine active indices or -1
    Ref1D ref;
    double sigF = 0, sigG = 0;    // reference units: c (p+1)^2
};

// ---------------------------------------------------------------------------
// Device copy of a level in precision T.
template <typename T>
struct DevLevel {
    int d = 2, p = 1, nc = 4, nf = 2, n_act = 0, n_col0 = 0, n_bnd = 0, n_surr = 0;
    int *nbr = nullptr;       // n_act * 2d
    int *bnd_of = nullptr;    // n_act
    int *bnd_cells = nullptr; // n_bnd
    int *batch_start = nullptr;  // colour-interleaved batch table (see CellArgs)
    int nbatch = 0;
    T *shift = nullptr;       // n_surr * nf * d, reference units d / h
    T *Bint_t = nullptr;      // transposed shared inverse, [j][i]
    T *Bbnd_t = nullptr;      // n_bnd * nc*nc transposed inverses
    int *parent = nullptr;    // transfer maps (see HostLevel)
    int *childpos = nullptr;
    int *children = nullptr;
    int *rr_perm = nullptr;   // child cells of the coarse cells in spatial order of the coarse cells
    int *rr_grp = nullptr;    // the coarse cell of each group of children in rr_perm
    int *rr_gbnd = nullptr;   // bnd_of of that coarse cell (coarse level's block index, -1: interior)
    T P1[2][MAXN1][MAXN1];    // 1D embedding coarse->fine per child offset, [o][a_fine][b_coarse]
    int pc = 1;               // coarse degree for the transfer
    KRef<T> kref;
    // learned correction on this level (finest only), may be null
    T *lw = nullptr, *lU = nullptr, *lV = nullptr;  // n_bnd, n_bnd*nc*4, n_bnd*nc*4
    // cells whose inverse the stabilisation changed (their block update does
    // not zero the block residual): hold[n_bnd] flags their blocks; rep1 lists
    // the colour-1 ones, clip0 the colour-0 ones with clip0_cbnd their block
    // index on the next coarser level (p-transfers keep the cells)
    int *hold = nullptr;
    int *rep1 = nullptr, n_rep1 = 0;
    int *clip0 = nullptr, *clip0_cbnd = nullptr, n_clip0 = 0;
    // pencil path (3D levels it supports): interior cells in mesh order
    // (whole-level operations) and by colour (n_int0 of colour 0 first), the
    // boundary cells by colour (n_bl0 of colour 0 first) for the other kernel
    bool pencil = false;
    int *pen_all = nullptr, *pen_col = nullptr, *bnd_list = nullptr;
    int *bl_cbnd = nullptr;   // p-transfer below: the next coarser level's block index of bnd_list's cells
    int n_int0 = 0, n_int1 = 0, n_bl0 = 0, n_bl1 = 0;
    // level work vectors (coarser levels and the FP32 cycle)
    T *z = nullptr, *b = nullptr, *r = nullptr;
    // Chebyshev-accelerated block-Jacobi smoother: search direction and the
    // estimate of the largest eigenvalue of B A on this level
    T *dcheb = nullptr;
    double cheb_lmax = 0.0;
};

struct CoarseDev {
    int n = 0;
    double *Ainv64 = nullptr;   // dense inverse, used by the FP64 and the FP32 cycle
};

// Device scalars of one FGMRES solve (the pinned staging buffer has the same
// size): three sum areas of SBM_MAX_RESTART + 1 (Gram-Schmidt pass 1, pass 2,
// explicit norm), the least-squares coefficients and beta^2.
constexpr int SOLVE_SCALARS = 4 * (SBM_MAX_RESTART + 1) + 1;
// Host Arnoldi storage: Hessenberg matrix, Givens cosines and sines, reduced
// right-hand side, coefficients.
constexpr size_t ARNOLDI_DOUBLES =
    (size_t)(SBM_MAX_RESTART + 1) * SBM_MAX_RESTART + 4 * (size_t)SBM_MAX_RESTART + 1;

}  // namespace sbm

// The opaque problem handle.
struct sbm_problem {
    sbm_options opt;
    sbm::Geometry geom;
    int dim = 2, n = 0, p = 1;
    std::vector<sbm::HostLevel> levels;       // 0 = coarsest
    std::vector<sbm::DevLevel<double>> dev64;
    std::vector<sbm::DevLevel<float>> dev32;
    sbm::CoarseDev coarse;
    std::vector<double> A0;                   // dense coarsest matrix (host)
    hipStream_t stream = nullptr;
    // FGMRES workspace (FP64)
    int ws_restart = 0;
    double *V = nullptr, *Z = nullptr, *w = nullptr, *red = nullptr, *hdev = nullptr;
    double *r32in = nullptr;   // unused placeholder for alignment
    float *f32_in = nullptr, *f32_out = nullptr;   // FP32 cycle in/out on the finest level
    double *pinned = nullptr;  // host staging for reductions (SOLVE_SCALARS)
    std::vector<double> arnoldi;  // ARNOLDI_DOUBLES, sized at setup
    std::vector<void *> allocations;
    std::string last_error;
    bool host_only = false;    // set up with device < 0: host data only (tests)
    // learned boundary-cell correction of the finest level
    bool learned_on = false;
    int learned_nout = 0;
    float *lrn_X = nullptr, *lrn_O = nullptr;
    short *lrn_wbuf = nullptr;
    // finest-level work vectors of the training-data entry points (allocated on first use)
    double *pair_r = nullptr, *pair_t = nullptr;
};
