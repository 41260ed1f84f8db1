// Kernel launchers (kernels.hip).
#pragma once

#include "common.hpp"

namespace sbm {

enum { OP_APPLY = 0, OP_RESID = 1, OP_SMOOTH = 2, OP_RESTRICT = 3 };

template <typename T>
struct CellArgs {
    const int *nbr;       // n_act * 2d
    const T *shift;       // n_surr * nf * d (reference units)
    const int *bnd_of;    // n_act
    const T *Bint_t;      // nc * nc, transposed
    const T *Bbnd_t;      // n_bnd * nc * nc, transposed
    const T *lw, *lU, *lV;  // learned correction (may be null)
    // Optional batch table for whole-level operations: batch b covers the cells
    // [batch_start[b], min(batch_start[b] + CPB, end of its colour)); colour 0
    // ends at split.  The table interleaves the two colours by position so that
    // the contiguous range of batches an XCD receives is one spatial region.
    const int *batch_start;
    int nbatch, split;
    // Optional cell list: the launch treats the cells perm[0 .. ncells)
    // instead of a contiguous range or the batch table
    const int *perm;
    // zero-start update (smooth_zero): nonzero = interior colour-0 cells are
    // left to the pencil kernel (neither computed nor written)
    int skip_interior;
};

// waves per block of the cell kernels for cells of nc DoFs (measured: two
// waves; four and one were slower on the 2D Q2, 3D Q2 and 3D Q3 solves)
constexpr int cell_waves(int) { return 2; }

// cells per block of the cell kernels (cell_waves waves, 64 / (p+1)^d cells per wave)
inline int cells_per_block(int d, int p) {
    int nc = d == 2 ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
    return cell_waves(nc) * (64 / nc);
}

template <typename T>
struct TransferArgs {
    T P1[2][MAXN1][MAXN1];
};

// Where a colour update also sends the cells' new values (the last update of
// each colour in the last smoothing step of a level, after which they are
// final): added through the embedding into the next finer level, h (2^d
// children per cell, Q1) or p (the same cell one degree up), or copied to FP64.
enum { EMIT_NONE = 0, EMIT_H = 1, EMIT_P = 2, EMIT_F64 = 3 };

template <typename T>
struct EmitArgs {
    int kind;
    const int *children;      // EMIT_H: n_act * 2^d fine cells (-1: inactive); EMIT_P: n_act fine cells
    T *zf;                    // EMIT_H / EMIT_P: fine-level vector, zf += P z
    double *z64;              // EMIT_F64: receives z in FP64
    T P1[2][MAXN1][MAXN1];    // 1D embedding [child offset][fine node][coarse node]
    // optional, per boundary block of the updated level: nonzero = this launch
    // does not send the cell's values on (a later launch updates it again)
    const int *hold;
};

// First colour-0 update of the coarser level from z = 0, formed by the
// residual-restriction kernel from the right-hand side it has just computed:
// z_K = omega B_K bc_K for coarse cells K < split, z_K = 0 for the others.
template <typename T>
struct ZeroStartArgs {
    T *z;                     // coarse-level z (all cells written)
    const int *bnd_of;        // coarse level: boundary-block index of each cell (-1: interior)
    const int *grp_bnd;       // h-transfers: bnd_of of the coarse cell of each child group
    const T *Bint_t, *Bbnd_t; // coarse level: transposed cell inverses
    int split;                // coarse cells of colour 0
    T omega;
};

// Interior cells of a level by the pencil kernel (pencil.hip): OP_APPLY,
// OP_RESID or OP_SMOOTH on the cells cells[0 .. ncells), all of which must
// have every face neighbour; e: null or EMIT_F64.  Levels it handles:
bool pencil_supported(int d, int p);
template <typename T>
int launch_pencil(int d, int p, int op, int ncells, const int *cells, const T *x, T *y, const T *b,
                  const CellArgs<T> &a, const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e);
// the boundary cells (bcells, one thread per DoF) and the interior cells
// (pcells, pencil form) of a 3D Q2/Q3 level in one launch: OP_APPLY, OP_RESID
// or OP_SMOOTH (e: null, or EMIT_F64 in FP32 only); FP32 and FP64
template <typename T>
int launch_fused(int d, int p, int op, int nbnd, const int *bcells, int npen, const int *pcells, const T *x, T *y,
                 const T *b, const CellArgs<T> &a, const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e);
// residual restricted to the same cells one degree down, bc = E^T (b - A x),
// and zc = 0 there (when given), on the listed interior cells
template <typename T>
int launch_pencil_rr(int d, int p, int ncells, const int *cells, const T *x, const T *b, T *bc, T *zc,
                     const CellArgs<T> &a, const KRef<T> &R, const TransferArgs<T> &tr, hipStream_t st);
// one block-Jacobi step d_K = alpha d_K + beta B_int r_K, z_K += d_K on the
// listed interior cells (d not read when alpha = 0)
template <typename T>
int launch_pencil_bj(int d, int p, int ncells, const int *cells, const T *r, T *dv, T *z, const T *Bint_t, T alpha,
                     T beta, hipStream_t st);
// p-prolongation zf += E zc on every cell of a 3D Q2/Q3 level (parent: the
// same cell one degree down)
template <typename T>
int launch_pencil_prolong(int d, int p, int ncells, const int *parent, const T *zc, T *zf, const TransferArgs<T> &tr,
                          hipStream_t st);
// the zero-start colour-0 update z_K = omega B_int b_K on the listed interior cells
template <typename T, typename TB>
int launch_pencil_zero(int d, int p, int ncells, const int *cells, const TB *b, T *z, const T *Bint_t, T omega,
                       hipStream_t st);

template <typename T>
int launch_cellop(int d, int p, int op, int cell0, int ncells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                  const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e = nullptr);
// bc = R (b - A x) for the next coarser level: residual and restriction in one
// launch (perm: child cells grouped by coarse cell, grp: the coarse cell of
// each group; both ordered spatially)
// (zs: also the coarser level's zero-start colour-0 update; c1_only, p-transfers:
// the colour-0 residual is known to vanish, so only colour-1 cells are computed
// and the colour-0 part of bc and zs->z is set to zero)
template <typename T>
int launch_resid_restrict(int d, int p, int n_coarse, int nch, int n1c, const int *perm, const int *grp, const T *x,
                          const T *b, T *bc, const CellArgs<T> &a, const KRef<T> &R, const TransferArgs<T> &tr,
                          hipStream_t st, const ZeroStartArgs<T> *zs = nullptr, bool c1_only = false);
// first colour-0 update from z = 0; b may be FP64 for an FP32 cycle, bcopy
// (optional) receives b in the cycle precision
template <typename T, typename TB>
int launch_smooth_zero(int d, int p, int n_act, int split, const TB *b, T *bcopy, T *z, const CellArgs<T> &a, T omega,
                       hipStream_t st);
template <typename T>
int launch_prolong(int d, int n_fine, int n1f, int n1c, const int *parent, const int *childpos, const T *zc, T *zf,
                   const TransferArgs<T> &tr, hipStream_t st);
template <typename T>
int launch_restrict(int d, int n_coarse, int n1f, int n1c, int nch, const int *children, const T *rf, T *bc,
                    const TransferArgs<T> &tr, hipStream_t st);
template <typename TA, typename TX>
int launch_dense_gemv(int n, const TA *A, const TX *x, TX *y, hipStream_t st);
// y = A x on a Q1 coarsest level (n = n_cells * 2^d) and e's prolongation of y
// into the next level (EMIT_H or EMIT_P) in one launch
template <typename TX>
int launch_coarse_solve_prolong(int d, int n, const double *A, const TX *x, TX *y, const EmitArgs<TX> &e,
                                hipStream_t st);
template <typename T>
int launch_fill(long long n, T *x, T v, hipStream_t st);
// x[0..n) = 0 and, if y is given, y[0..n) = 0 (one launch; x, y 16-byte aligned)
template <typename T>
int launch_zero2(long long n, T *x, T *y, hipStream_t st);
// Additive (block-Jacobi) update of every active cell of a level:
// d_K = alpha d_K + beta B_K r_K (alpha = 0: d is not read), then z_K += d_K
// when z is given.  B_K: the cell's (transposed) inverse.
template <typename T>
int launch_block_jacobi(int n_act, int nc, const int *bnd_of, const T *Bint_t, const T *Bbnd_t, const T *r, T *d,
                        T *z, T alpha, T beta, hipStream_t st, const int *list = nullptr);
int launch_cast_d2f(long long n, const double *x, float *y, hipStream_t st);
int launch_cast_f2d(long long n, const float *x, double *y, hipStream_t st);
// Gram-Schmidt kernels.  Partial-sum buffers hold gs_partials_max() doubles;
// the two passes of one Arnoldi step use two different buffers.
constexpr int gs_partials_max() { return 256 * 32; }
// part <- per-block partials of V_i . w (i < m) and w . w
int launch_gs_dots(long long n, int m, const double *V, const double *w, double *part, hipStream_t st);
// h = sums of hpart (also stored in hout[0..m]); w -= V h; part <- partials of V_i . w and w . w
int launch_gs_axpy_dots(long long n, int m, const double *V, const double *hpart, double *hout, double *w,
                        double *part, hipStream_t st);
// out[0..nv) = sums of the partials left by a kernel above for vectors of length n
int launch_gs_reduce(long long n, int nv, const double *part, double *out, hipStream_t st);
// v = (w - V h) * inv
int launch_gs_axpy_scale(long long n, int m, const double *V, const double *h, double inv, const double *w, double *v,
                         hipStream_t st);
int launch_multiaxpy(long long n, int m, double sign, const double *h, const double *V, double *w, hipStream_t st);
int launch_scale(long long n, const double *nrm2, const double *w, double *v, hipStream_t st);

}  // namespace sbm
