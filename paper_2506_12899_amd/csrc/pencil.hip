// Pencil form of the cell operator on the interior cells of 3D levels
// (operator of Sec. 2.2, cell-wise block update of Sec. 3.1).
//
// An interior cell has all 2d face neighbours, hence no surrogate face: its 1D
// self operator is the interior one T in every direction, and its block
// inverse is the level's shared one.  On such a cell, in reference units and
// scaled by h^(d-2),
//   (A u)_K = sum_k (prod_{d != k} M_d) (T_k u_K + E_k f_k)
// where f_k holds the SIPG face data of the two neighbours across the faces
// normal to e_k, at each face node: va = -sg dn / 2 - sigma_F t and vb = t / 2
// from the neighbour's trace t and normal derivative dn (sg = -1 on the low
// face, +1 on the high one), and E_k places them along e_k: va on the end node
// of that face, sg vb times the derivative of the basis there.  So every face
// term is a source of the contraction stage of its normal direction.
//
// Thread mapping: (P+1)^2 lanes per cell, each holding one line of P+1 nodes
// (a pencil): along x in the first stage (A = M_x u, B = T_x u + E_x f_x),
// along y in the second (Q = M_y A, R = T_y A + M_y B + E_y M_x f_y), along z
// in the third (y = M_z R + T_z Q + E_z M_y M_x f_z).  The direction changes
// and the tangential contractions of the y and z face data go through LDS;
// every other coefficient index is a compile-time constant, so the 1D
// operators come from the kernel arguments (scalar registers).  A cell's lanes
// share a wave, so its LDS exchanges need no block barrier.  Against the
// one-thread-per-DoF kernel this removes the per-DoF index arithmetic and most
// LDS reads, which bound that kernel's instruction issue on 64-DoF cells.
#include "pencil_body.hpp"

namespace sbm {

template <int P, typename T, int OP, bool F64OUT>
__global__ __launch_bounds__(64 * PSh<P>::WAVES) void pencil_kernel(int ncells, const int *__restrict__ cells,
                                                                     const T *xin, T *out, const T *__restrict__ b,
                                                                     const int *__restrict__ nbr,
                                                                     const T *__restrict__ Bint_t, KRef<T> R,
                                                                     double *__restrict__ z64, T *__restrict__ bc,
                                                                     T *__restrict__ zc, TransferArgs<T> tr) {
    __shared__ PencilShared<P, T, OP> SH;
    pencil_block<P, T, OP, F64OUT>(xcd_remap(blockIdx.x, gridDim.x), SH, ncells, cells, xin, out, b, nbr, Bint_t, R,
                                   z64, bc, zc, tr);
}

// Block products with the shared inverse on the listed interior cells.
// BJ = false: the first colour-0 update from z = 0, whose residual is b
// itself: z_K = omega B_int b_K (b read in its own precision TB).
// BJ = true: one block-Jacobi step of the Chebyshev smoother (Sec. 3.1
// additive variant) from the residual r = b: d_K = alpha d_K + omega B_int r_K
// (d not read when alpha = 0), z_K += d_K.
template <int P, typename T, typename TB, bool BJ>
__global__ __launch_bounds__(64 * PSh<P>::WAVES) void pencil_zero_kernel(int ncells, const int *__restrict__ cells,
                                                                          const TB *__restrict__ b,
                                                                          T *__restrict__ z,
                                                                          const T *__restrict__ Bint_t, T omega,
                                                                          T *__restrict__ dv, T alpha) {
    using S = PSh<P>;
    constexpr int N1 = S::N1, NP = S::NP, NC = S::NC, CPW = S::CPW;
    constexpr bool FULL = CPW * NP == 64;
    constexpr bool MF = P == 3;    // as in the colour update
    constexpr bool SBL = sizeof(T) == 4 && !MF;
    __shared__ T sr[MF ? 1 : S::CPB * PLayout<P>::VS];
    __shared__ T sB[SBL ? NC * NC : 1];
    __shared__ int scell[MF ? S::CPB : 1];
    constexpr int RS = S::CPB + 1;   // as in the colour update
    __shared__ T sRm[MF ? NC * RS : 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = lane / NP;
    const bool inslot = FULL || slot < CPW;
    const int q = inslot ? lane - slot * NP : 0;
    const int lc = wave * CPW + (inslot ? slot : 0);
    const int pos = xcd_remap(blockIdx.x, gridDim.x) * S::CPB + lc;
    const bool live = inslot && pos < ncells;
    InverseStager<P, T, SBL> bst;
    bst.load(Bint_t);
    constexpr int KS = MF ? NC / 4 : 1;
    T bsl[KS];
    if constexpr (MF) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bsl[ks] = Bint_t[(size_t)(4 * ks + lane / 16) * NC + 16 * wave + lane % 16];
    }
    const int cell = live ? cells[pos] : 0;
    T bv[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) bv[c] = (T)b[(size_t)cell * NC + q + NP * c];
    bst.store(sB);
    if constexpr (MF) {
#pragma unroll
        for (int c = 0; c < N1; ++c) sRm[(q + NP * c) * RS + lc] = bv[c];
        if (q == 0) scell[lc] = live ? cell : -1;
        __syncthreads();
        typedef typename Tile16<T>::v4 f4;
        f4 acc = {T(0), T(0), T(0), T(0)};
        const int col = lane % 16;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = Tile16<T>::step(bsl[ks], sRm[(4 * ks + lane / 16) * RS + col], acc);
        const int ccell = scell[col];
        if (ccell >= 0) {
            const size_t o = (size_t)ccell * NC + 16 * wave;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const size_t g = o + Tile16<T>::row(lane / 16, r);
                if constexpr (BJ) {
                    const T dn = alpha == T(0) ? omega * acc[r] : alpha * dv[g] + omega * acc[r];
                    dv[g] = dn;
                    z[g] += dn;
                } else {
                    z[g] = T(0) + omega * acc[r];
                }
            }
        }
        return;
    }
    if (inslot) {
#pragma unroll
        for (int c = 0; c < N1; ++c) sr[PLayout<P>::at(lc, q + NP * c)] = bv[c];
    }
    wave_sync();
    if constexpr (SBL) __syncthreads();
    T corr[N1];
    interior_correction<P, T, SBL>(sB, Bint_t, sr + PLayout<P>::at(lc, 0), q, corr);
    if (live) {
#pragma unroll
        for (int c = 0; c < N1; ++c) {
            const size_t g = (size_t)cell * NC + q + NP * c;
            if constexpr (BJ) {
                const T dn = alpha == T(0) ? omega * corr[c] : alpha * dv[g] + omega * corr[c];
                dv[g] = dn;
                z[g] += dn;
            } else {
                z[g] = T(0) + omega * corr[c];
            }
        }
    }
}

// p-prolongation on every cell of a 3D level of degree P from the same cell
// one degree down (Sec. 3.2: the embedding E = tr.P1[0] along each
// direction): zf_K += (E x E x E) zc_parent(K), by sum factorisation along x
// (lanes of coarse (y, z) lines), y (fine x, coarse z), z (fine x, y: the
// lane's pencil of the fine cell).
template <int P, typename T>
__global__ __launch_bounds__(64 * PSh<P>::WAVES) void pencil_prolong_kernel(int ncells, const int *__restrict__ parent,
                                                                             const T *__restrict__ zc,
                                                                             T *__restrict__ zf, TransferArgs<T> tr) {
    using S = PSh<P>;
    constexpr int N1 = S::N1, NP = S::NP, NC = S::NC, CPW = S::CPW, N1C = P, NCC = P * P * P;
    constexpr bool FULL = CPW * NP == 64;
    __shared__ T s1[S::CPB][N1 * N1C * N1C];   // after x: [fine x][coarse y][coarse z]
    __shared__ T s2[S::CPB][N1 * N1 * N1C];    // after y: [fine x][fine y][coarse z]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = lane / NP;
    const bool inslot = FULL || slot < CPW;
    const int q = inslot ? lane - slot * NP : 0;
    const int qa = q % N1, qb = q / N1;
    const int lc = wave * CPW + (inslot ? slot : 0);
    const int cell = xcd_remap(blockIdx.x, gridDim.x) * S::CPB + lc;
    const bool live = inslot && cell < ncells;
    const int K = live ? cell : 0;
    const int pc = parent[K];
    const T *zp = zc + (size_t)(pc < 0 ? 0 : pc) * NCC;
    // this lane's fine values (its z pencil) are read early, with the coarse line
    T old[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) old[c] = zf[(size_t)K * NC + q + NP * c];
    if (inslot && q < N1C * N1C) {
        T c[N1C];
#pragma unroll
        for (int a = 0; a < N1C; ++a) c[a] = zp[a + N1C * q];
#pragma unroll
        for (int f = 0; f < N1; ++f) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1C; ++a) acc += tr.P1[0][f][a] * c[a];
            s1[lc][f + N1 * q] = acc;
        }
    }
    wave_sync();
    if (inslot && q < N1 * N1C) {
        const int fx = q % N1, cz = q / N1;
        T c[N1C];
#pragma unroll
        for (int a = 0; a < N1C; ++a) c[a] = s1[lc][fx + N1 * (a + N1C * cz)];
#pragma unroll
        for (int f = 0; f < N1; ++f) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1C; ++a) acc += tr.P1[0][f][a] * c[a];
            s2[lc][fx + N1 * (f + N1 * cz)] = acc;
        }
    }
    wave_sync();
    T c[N1C];
#pragma unroll
    for (int a = 0; a < N1C; ++a) c[a] = s2[lc][qa + N1 * (qb + N1 * a)];
    if (live && pc >= 0) {
#pragma unroll
        for (int f = 0; f < N1; ++f) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1C; ++a) acc += tr.P1[0][f][a] * c[a];
            zf[(size_t)K * NC + q + NP * f] = old[f] + acc;
        }
    }
}

template <typename T>
int launch_pencil_prolong(int d, int p, int ncells, const int *parent, const T *zc, T *zf, const TransferArgs<T> &tr,
                          hipStream_t st) {
    if (ncells <= 0) return 0;
    if (!pencil_supported(d, p) || parent == nullptr) return -1;
    if (p == 3) {
        using S = PSh<3>;
        hipLaunchKernelGGL((pencil_prolong_kernel<3, T>), dim3((ncells + S::CPB - 1) / S::CPB), dim3(64 * S::WAVES), 0,
                           st, ncells, parent, zc, zf, tr);
    } else {
        using S = PSh<2>;
        hipLaunchKernelGGL((pencil_prolong_kernel<2, T>), dim3((ncells + S::CPB - 1) / S::CPB), dim3(64 * S::WAVES), 0,
                           st, ncells, parent, zc, zf, tr);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_pencil_prolong<double>(int, int, int, const int *, const double *, double *,
                                           const TransferArgs<double> &, hipStream_t);
template int launch_pencil_prolong<float>(int, int, int, const int *, const float *, float *,
                                          const TransferArgs<float> &, hipStream_t);

template <int P, typename T>
static int launch_p(int op, int ncells, const int *cells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                    const KRef<T> &R, hipStream_t st, double *z64) {
    using S = PSh<P>;
    const dim3 g((ncells + S::CPB - 1) / S::CPB), bl(64 * S::WAVES);
    if (op == OP_APPLY)
        hipLaunchKernelGGL((pencil_kernel<P, T, OP_APPLY, false>), g, bl, 0, st, ncells, cells, x, y, b, a.nbr,
                           a.Bint_t, R, nullptr, nullptr, nullptr, TransferArgs<T>{});
    else if (op == OP_RESID)
        hipLaunchKernelGGL((pencil_kernel<P, T, OP_RESID, false>), g, bl, 0, st, ncells, cells, x, y, b, a.nbr,
                           a.Bint_t, R, nullptr, nullptr, nullptr, TransferArgs<T>{});
    else if (op == OP_SMOOTH && z64 == nullptr)
        hipLaunchKernelGGL((pencil_kernel<P, T, OP_SMOOTH, false>), g, bl, 0, st, ncells, cells, x, y, b, a.nbr,
                           a.Bint_t, R, nullptr, nullptr, nullptr, TransferArgs<T>{});
    else if (op == OP_SMOOTH) {
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL((pencil_kernel<P, T, OP_SMOOTH, true>), g, bl, 0, st, ncells, cells, x, y, b, a.nbr,
                               a.Bint_t, R, z64, nullptr, nullptr, TransferArgs<T>{});
        else
            return -1;
    } else {
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool pencil_supported(int d, int p) { return d == 3 && (p == 2 || p == 3); }

template <typename T>
int launch_pencil(int d, int p, int op, int ncells, const int *cells, const T *x, T *y, const T *b,
                  const CellArgs<T> &a, const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e) {
    if (ncells <= 0) return 0;
    if (!pencil_supported(d, p) || cells == nullptr) return -1;
    double *z64 = nullptr;
    if (e != nullptr) {
        if (e->kind != EMIT_F64 || op != OP_SMOOTH || e->z64 == nullptr) return -1;
        z64 = e->z64;
    }
    return p == 3 ? launch_p<3, T>(op, ncells, cells, x, y, b, a, R, st, z64)
                  : launch_p<2, T>(op, ncells, cells, x, y, b, a, R, st, z64);
}
template int launch_pencil<double>(int, int, int, int, const int *, const double *, double *, const double *,
                                   const CellArgs<double> &, const KRef<double> &, hipStream_t,
                                   const EmitArgs<double> *);
template int launch_pencil<float>(int, int, int, int, const int *, const float *, float *, const float *,
                                  const CellArgs<float> &, const KRef<float> &, hipStream_t, const EmitArgs<float> *);

template <typename T, typename TB>
int launch_pencil_zero(int d, int p, int ncells, const int *cells, const TB *b, T *z, const T *Bint_t, T omega,
                       hipStream_t st) {
    if (ncells <= 0) return 0;
    if (!pencil_supported(d, p) || cells == nullptr) return -1;
    if (p == 3) {
        using S = PSh<3>;
        hipLaunchKernelGGL((pencil_zero_kernel<3, T, TB, false>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, b, z, Bint_t, omega, (T *)nullptr, T(0));
    } else {
        using S = PSh<2>;
        hipLaunchKernelGGL((pencil_zero_kernel<2, T, TB, false>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, b, z, Bint_t, omega, (T *)nullptr, T(0));
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_pencil_bj(int d, int p, int ncells, const int *cells, const T *r, T *dv, T *z, const T *Bint_t, T alpha,
                     T beta, hipStream_t st) {
    if (ncells <= 0) return 0;
    if (!pencil_supported(d, p) || cells == nullptr || dv == nullptr || z == nullptr) return -1;
    if (p == 3) {
        using S = PSh<3>;
        hipLaunchKernelGGL((pencil_zero_kernel<3, T, T, true>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, r, z, Bint_t, beta, dv, alpha);
    } else {
        using S = PSh<2>;
        hipLaunchKernelGGL((pencil_zero_kernel<2, T, T, true>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, r, z, Bint_t, beta, dv, alpha);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_pencil_bj<double>(int, int, int, const int *, const double *, double *, double *, const double *,
                                      double, double, hipStream_t);
template int launch_pencil_bj<float>(int, int, int, const int *, const float *, float *, float *, const float *, float,
                                     float, hipStream_t);
template int launch_pencil_zero<double, double>(int, int, int, const int *, const double *, double *, const double *,
                                                double, hipStream_t);
template int launch_pencil_zero<float, float>(int, int, int, const int *, const float *, float *, const float *, float,
                                              hipStream_t);
template int launch_pencil_zero<float, double>(int, int, int, const int *, const double *, float *, const float *,
                                               float, hipStream_t);

template <typename T>
int launch_pencil_rr(int d, int p, int ncells, const int *cells, const T *x, const T *b, T *bc, T *zc,
                     const CellArgs<T> &a, const KRef<T> &R, const TransferArgs<T> &tr, hipStream_t st) {
    if (ncells <= 0) return 0;
    if (!pencil_supported(d, p) || cells == nullptr || bc == nullptr) return -1;
    if (p == 3) {
        using S = PSh<3>;
        hipLaunchKernelGGL((pencil_kernel<3, T, OP_RESTRICT, false>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, x, (T *)nullptr, b, a.nbr, a.Bint_t, R,
                           (double *)nullptr, bc, zc, tr);
    } else {
        using S = PSh<2>;
        hipLaunchKernelGGL((pencil_kernel<2, T, OP_RESTRICT, false>), dim3((ncells + S::CPB - 1) / S::CPB),
                           dim3(64 * S::WAVES), 0, st, ncells, cells, x, (T *)nullptr, b, a.nbr, a.Bint_t, R,
                           (double *)nullptr, bc, zc, tr);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_pencil_rr<double>(int, int, int, const int *, const double *, const double *, double *, double *,
                                      const CellArgs<double> &, const KRef<double> &, const TransferArgs<double> &,
                                      hipStream_t);
template int launch_pencil_rr<float>(int, int, int, const int *, const float *, const float *, float *, float *,
                                     const CellArgs<float> &, const KRef<float> &, const TransferArgs<float> &,
                                     hipStream_t);

}  // namespace sbm
