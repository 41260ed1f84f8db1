// Device code of the pencil kernel (interior cells of 3D Q2/Q3 levels),
// shared by its own kernels (pencil.hip) and the launch that also takes a
// level's boundary cells (kernels.hip).
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "device_util.hpp"

namespace sbm {

template <int P>
struct PSh {
    static constexpr int N1 = P + 1, NP = N1 * N1, NC = NP * N1;
    static constexpr int CPW = 64 / NP;      // cells per wave
    static constexpr int WAVES = 4;          // waves per block
    static constexpr int CPB = CPW * WAVES;  // cells per block
};

// Position of DoF i of cell slot lc in a stage array: for Q3 each line of 4
// nodes along x is followed by one unused element and a cell takes 80 (the
// line stride 5 and the cell stride, 16 banks apart, spread the x-, y- and
// z-pencil accesses of a wave over the 32 LDS banks: a bank model of the four
// access patterns gives 1.4x the conflict-free pass count against 3.2x
// unpadded); the 27-DoF cells of Q2 are spread by their odd size already.
template <int P>
struct PLayout {
    static constexpr int NC = PSh<P>::NC, NP = PSh<P>::NP;
    static constexpr int VS = P == 3 ? 80 : NC;
    // face arrays [side][va, vb][face node] of a cell: 64 values for Q3, stride
    // 80 for the same reason
    static constexpr int FS = P == 3 ? 80 : 4 * NP;
    __device__ __forceinline__ static int at(int lc, int i) { return lc * VS + (P == 3 ? i + (i >> 2) : i); }
    __device__ __forceinline__ static int face(int lc, int s, int w, int j) { return lc * FS + (2 * s + w) * NP + j; }
};

template <int P, typename T>
struct PencilLds {
    static constexpr int CPB = PSh<P>::CPB, VS = PLayout<P>::VS, FS = PLayout<P>::FS;
    T v0[CPB * VS];   // A, then Q, then (smoother) the residual
    T v1[CPB * VS];   // B, then R
    T fa[CPB * FS];   // face data
    T fg[CPB * FS];   // z-face data after the x contraction
};

// face data of one neighbour line (its nodes along the face normal, from the
// far end to the shared face or back): va, vb as above; s = side of the cell
template <int P, typename T>
__device__ __forceinline__ void face_data(const KRef<T> &R, int s, const T *line, T &va, T &vb) {
    constexpr int N1 = P + 1;
    const T *gN = R.g[s == 1 ? 0 : 1];   // the neighbour's derivative at the shared face
    const T t = line[s == 1 ? 0 : P];
    T dn = 0;
#pragma unroll
    for (int m = 0; m < N1; ++m) dn += gN[m] * line[m];
    const T sg = s == 1 ? T(1) : T(-1);
    va = T(-0.5) * sg * dn - R.sigF * t;
    vb = T(0.5) * t;
}

// pencil += E_s (va, vb): va on the end node of side s, sg vb g_s along the line
template <int P, typename T>
__device__ __forceinline__ void inject(const KRef<T> &R, int s, T va, T vb, T *v) {
    constexpr int N1 = P + 1;
    const T sg = s == 1 ? T(1) : T(-1);
    v[s == 1 ? P : 0] += va;
#pragma unroll
    for (int c = 0; c < N1; ++c) v[c] += sg * R.g[s][c] * vb;
}

// entry a of a row-major N1 x N1 table at a lane-dependent row, by selects
// (an indexed kernel-argument read would go through scratch memory)
template <int N1, typename T>
__device__ __forceinline__ T row_entry(const T (&M)[MAXN1][MAXN1], int row, int a) {
    T v = M[0][a];
#pragma unroll
    for (int r = 1; r < N1; ++r) v = row == r ? M[r][a] : v;
    return v;
}

// One K step of a 16 x 16 tile product on the matrix cores, D += A B with A
// 16 x 4, B 4 x 16 (wave64 operand layout: A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k; the result D[i][j] sits in lane j + 16 g, register r,
// with i = row(g, r): 4 g + r in FP32, g + 4 r in FP64; both checked by an
// in-bounds probe)
template <typename T>
struct Tile16;
template <>
struct Tile16<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ static v4 step(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
};
template <>
struct Tile16<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ static v4 step(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int g, int r) { return g + 4 * r; }
};

// The shared interior inverse B_int (given transposed, [j][i]) staged into
// LDS by the whole block, laid out [j][q][c] so that a lane's N1 outputs
// i = q + NP c sit next to each other; load() issues the loads, store()
// writes them (the caller's first loads go out in between).  SBL = false:
// nothing (the columns are read from memory).
template <int P, typename T, bool SBL>
struct InverseStager {
    static constexpr int N1 = P + 1, NP = N1 * N1, NC = NP * N1, NT = 64 * PSh<P>::WAVES;
    static constexpr int PER = SBL ? (NC * NC + NT - 1) / NT : 1;
    T v[PER];
    __device__ __forceinline__ void load(const T *__restrict__ Bint_t) {
        if constexpr (SBL) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int t = (int)threadIdx.x + k * NT;   // destination index [j][qq][c]
                const int j = t / NC, rem = t % NC, qq = rem / N1, c = rem % N1;
                v[k] = t < NC * NC ? Bint_t[(size_t)j * NC + qq + NP * c] : T(0);
            }
        }
    }
    __device__ __forceinline__ void store(T *sB) const {
        if constexpr (SBL) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int t = (int)threadIdx.x + k * NT;
                if (t < NC * NC) sB[t] = v[k];
            }
        }
    }
};

// corr[c] = (B_int r)_(q + NP c), c = 0..P: r is the cell's residual in LDS
// (stage-array layout, PLayout);
// B_int from the staged copy (SBL) or its transposed columns in memory, read
// in groups of JB loads in flight
template <int P, typename T, bool SBL>
__device__ __forceinline__ void interior_correction(const T *sB, const T *__restrict__ Bint_t, const T *r, int q,
                                                    T (&corr)[P + 1]) {
    constexpr int N1 = P + 1, NP = N1 * N1, NC = NP * N1;
#pragma unroll
    for (int c = 0; c < N1; ++c) corr[c] = 0;
    if constexpr (SBL) {
#pragma unroll 8
        for (int j = 0; j < NC; ++j) {
            const T rj = r[PLayout<P>::at(0, j)];
#pragma unroll
            for (int c = 0; c < N1; ++c) corr[c] += sB[(j * NP + q) * N1 + c] * rj;
        }
    } else {
        constexpr int JB = NC % 8 == 0 ? 8 : (NC % 9 == 0 ? 9 : 1);
#pragma unroll 1
        for (int j0 = 0; j0 < NC; j0 += JB) {
            T col[JB][N1];
#pragma unroll
            for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                for (int c = 0; c < N1; ++c) col[jj][c] = Bint_t[(size_t)(j0 + jj) * NC + q + NP * c];
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                const T rj = r[PLayout<P>::at(0, j0 + jj)];
#pragma unroll
                for (int c = 0; c < N1; ++c) corr[c] += col[jj][c] * rj;
            }
        }
    }
}

// OP_APPLY: out = A x; OP_RESID: out = b - A x; OP_SMOOTH: x (= out) += omega
// B_int (b - A x) on the listed cells (F64OUT: the new values also go to z64);
// OP_RESTRICT: bc = E^T (b - A x) on the same cell of the next coarser level,
// degree P - 1 (Sec. 3.2 p-restriction, E = tr.P1[0] along each direction),
// and zc = 0 there when zc is given (the coarser level's zero start on cells
// of colour 1).  cells[0 .. ncells): interior cells of the level.
// LDS of one block of the pencil kernel.  The smoother's shared inverse in
// LDS (sB), laid out [j][q][c] (the lane's N1 outputs q + NP c next to each
// other): Q2 FP32 only.  Q3 (MF): the block's 16 corrections B_int r_K as one
// 64 x 64 by 64 x 16 product on the matrix cores (16x16x4 tiles, FP32 or
// FP64; wave w forms rows 16 w .. 16 w + 15 of all 16 cells, its slab of
// B_int held in registers), the residuals as the product's B operand in sRm,
// [DoF][cell slot] with rows of CPB + 1 (the writes of a cell's 16 lanes and
// the operand reads of a half-wave fall on distinct banks).
template <int P, typename T, int OP>
struct PencilShared {
    static constexpr int NC = PSh<P>::NC, CPB = PSh<P>::CPB, RS = CPB + 1;
    static constexpr bool MF = OP == OP_SMOOTH && P == 3;
    static constexpr bool SBL = OP == OP_SMOOTH && sizeof(T) == 4 && !MF;
    PencilLds<P, T> L;
    T sB[SBL ? NC * NC : 1];
    int scell[MF ? CPB : 1];
    T sRm[MF ? NC * RS : 1];
};

// One block (batch bb of the cell list) of the pencil kernel.
template <int P, typename T, int OP, bool F64OUT>
__device__ __forceinline__ void pencil_block(int bb, PencilShared<P, T, OP> &SH, int ncells,
                                             const int *__restrict__ cells, const T *xin, T *out,
                                             const T *__restrict__ b, const int *__restrict__ nbr,
                                             const T *__restrict__ Bint_t, const KRef<T> &R,
                                             double *__restrict__ z64, T *__restrict__ bc, T *__restrict__ zc,
                                             const TransferArgs<T> &tr) {
    using S = PSh<P>;
    using SHT = PencilShared<P, T, OP>;
    constexpr int N1 = S::N1, NP = S::NP, NC = S::NC, CPW = S::CPW;
    constexpr bool FULL = CPW * NP == 64;
    constexpr bool MF = SHT::MF, SBL = SHT::SBL;
    constexpr int RS = SHT::RS;
    auto &L = SH.L;
    T *sB = SH.sB;
    int *scell = SH.scell;
    T *sRm = SH.sRm;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = lane / NP;
    const bool inslot = FULL || slot < CPW;
    const int q = inslot ? lane - slot * NP : 0;
    const int qa = q % N1, qb = q / N1;
    const int lc = wave * CPW + (inslot ? slot : 0);
    const int pos = bb * S::CPB + lc;
    const bool live = inslot && pos < ncells;

    // ---- loads: the staged inverse, the cell's own data and its neighbour indices
    InverseStager<P, T, SBL> bst;
    bst.load(Bint_t);
    // MF: this lane's entries of the wave's slab, A[i][k] = B_int[16 w + lane % 16][4 s + lane / 16]
    // for the K steps s (operand layout of the 16x16x4 product: A[i][k] from lane i + 16 k)
    constexpr int KS = MF ? NC / 4 : 1;
    T bsl[KS];
    if constexpr (MF) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bsl[ks] = Bint_t[(size_t)(4 * ks + lane / 16) * NC + 16 * wave + lane % 16];
    }
    const int cell = live ? cells[pos] : 0;
    const T *xc = xin + (size_t)cell * NC;
    T u[N1], bv[N1], xz[N1];
#pragma unroll
    for (int m = 0; m < N1; ++m) u[m] = xc[m + N1 * q];
    if constexpr (OP != OP_APPLY) {
#pragma unroll
        for (int c = 0; c < N1; ++c) bv[c] = b[(size_t)cell * NC + q + NP * c];
    }
    if constexpr (OP == OP_SMOOTH && !MF) {
#pragma unroll
        for (int c = 0; c < N1; ++c) xz[c] = xc[q + NP * c];
    }
    if constexpr (MF) {
        if (q == 0) scell[lc] = live ? cell : -1;
    }
    int nb[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int v = live ? nbr[(size_t)cell * 6 + f] : cell;
        nb[f] = v >= 0 ? v : cell;   // (listed cells have all six; clamped all the same)
    }
    T Ma[N1], Mb[N1];
#pragma unroll
    for (int m = 0; m < N1; ++m) {
        Ma[m] = row_entry<N1>(R.M, qa, m);
        Mb[m] = row_entry<N1>(R.M, qb, m);
    }
    // neighbour lines through this lane's face nodes: x faces at (y, z) = (qa,
    // qb), y faces at (x, z) = (qa, qb), z faces at (x, y) = (qa, qb)
    T xl[2][N1], yl[2][N1], zl[2][N1];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T *nx = xin + (size_t)nb[s] * NC;
        const T *ny = xin + (size_t)nb[2 + s] * NC;
        const T *nz = xin + (size_t)nb[4 + s] * NC;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            xl[s][m] = nx[m + N1 * q];
            yl[s][m] = ny[qa + N1 * m + NP * qb];
            zl[s][m] = nz[qa + N1 * qb + NP * m];
        }
    }
    bst.store(sB);

    // ---- stage x: A = M u, B = T u + E_x f_x along x at (y, z) = (qa, qb)
    T A[N1], B[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) {
        T a = 0, bb = 0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            a += R.M[c][m] * u[m];
            bb += R.Tv[0][c][m] * u[m];
        }
        A[c] = a;
        B[c] = bb;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        T va, vb;
        face_data<P>(R, s, xl[s], va, vb);
        inject<P>(R, s, va, vb, B);
    }
    if (inslot) {
#pragma unroll
        for (int c = 0; c < N1; ++c) {
            L.v0[PLayout<P>::at(lc, c + N1 * q)] = A[c];
            L.v1[PLayout<P>::at(lc, c + N1 * q)] = B[c];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T va, vb;
            face_data<P>(R, s, yl[s], va, vb);
            L.fa[PLayout<P>::face(lc, s, 0, q)] = va;
            L.fa[PLayout<P>::face(lc, s, 1, q)] = vb;
        }
    }
    wave_sync();

    // ---- stage y: along y at (x, z) = (qa, qb)
    T Qv[N1], Rv[N1];
    {
        T a[N1], bb[N1];
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            a[m] = L.v0[PLayout<P>::at(lc, qa + N1 * m + NP * qb)];
            bb[m] = L.v1[PLayout<P>::at(lc, qa + N1 * m + NP * qb)];
        }
#pragma unroll
        for (int c = 0; c < N1; ++c) {
            T t1 = 0, t2 = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
                t1 += R.M[c][m] * a[m];
                t2 += R.Tv[0][c][m] * a[m] + R.M[c][m] * bb[m];
            }
            Qv[c] = t1;
            Rv[c] = t2;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            // y-face data contracted along x at face node (x, z) = (qa, qb)
            T fa = 0, fb = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
                fa += Ma[m] * L.fa[PLayout<P>::face(lc, s, 0, m + N1 * qb)];
                fb += Ma[m] * L.fa[PLayout<P>::face(lc, s, 1, m + N1 * qb)];
            }
            inject<P>(R, s, fa, fb, Rv);
        }
    }
    wave_sync();
    if (inslot) {
#pragma unroll
        for (int c = 0; c < N1; ++c) {
            L.v0[PLayout<P>::at(lc, qa + N1 * c + NP * qb)] = Qv[c];
            L.v1[PLayout<P>::at(lc, qa + N1 * c + NP * qb)] = Rv[c];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T va, vb;
            face_data<P>(R, s, zl[s], va, vb);
            L.fa[PLayout<P>::face(lc, s, 0, q)] = va;
            L.fa[PLayout<P>::face(lc, s, 1, q)] = vb;
        }
    }
    wave_sync();
    // z-face data contracted along x, at face node (x, y) = (qa, qb)
    {
        T g[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                T acc = 0;
#pragma unroll
                for (int m = 0; m < N1; ++m) acc += Ma[m] * L.fa[PLayout<P>::face(lc, s, w, m + N1 * qb)];
                g[s][w] = acc;
            }
        if (inslot) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int w = 0; w < 2; ++w) L.fg[PLayout<P>::face(lc, s, w, q)] = g[s][w];
        }
    }
    wave_sync();

    // ---- stage z: along z at (x, y) = (qa, qb); DoF q + NP c
    T y[N1];
    {
        T qv[N1], rv[N1];
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            qv[m] = L.v0[PLayout<P>::at(lc, q + NP * m)];
            rv[m] = L.v1[PLayout<P>::at(lc, q + NP * m)];
        }
#pragma unroll
        for (int c = 0; c < N1; ++c) {
            T t = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) t += R.M[c][m] * rv[m] + R.Tv[0][c][m] * qv[m];
            y[c] = t;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            // and along y
            T fa = 0, fb = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
                fa += Mb[m] * L.fg[PLayout<P>::face(lc, s, 0, qa + N1 * m)];
                fb += Mb[m] * L.fg[PLayout<P>::face(lc, s, 1, qa + N1 * m)];
            }
            inject<P>(R, s, fa, fb, y);
        }
#pragma unroll
        for (int c = 0; c < N1; ++c) y[c] *= R.scale;
    }

    // ---- output
    T *oc = out + (size_t)cell * NC;
    if constexpr (OP == OP_APPLY) {
        if (live) {
#pragma unroll
            for (int c = 0; c < N1; ++c) oc[q + NP * c] = y[c];
        }
    } else if constexpr (OP == OP_RESID) {
        if (live) {
#pragma unroll
            for (int c = 0; c < N1; ++c) oc[q + NP * c] = bv[c] - y[c];
        }
    } else if constexpr (OP == OP_RESTRICT) {
        // the residual contracted with E along z, then y, then x; the coarse
        // cell has N1C = P nodes per direction
        constexpr int N1C = P, NCC = N1C * N1C * N1C;
        T rz[N1C];
#pragma unroll
        for (int b2 = 0; b2 < N1C; ++b2) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc += tr.P1[0][a][b2] * (bv[a] - y[a]);
            rz[b2] = acc;
        }
        wave_sync();   // the z stage has read v0 and v1
        if (inslot) {
#pragma unroll
            for (int b2 = 0; b2 < N1C; ++b2) L.v0[PLayout<P>::at(lc, q + NP * b2)] = rz[b2];   // [x][y][z coarse]
        }
        wave_sync();
        // along y: lane q < N1 N1C takes fine x = q % N1, coarse z = q / N1
        const bool ylane = q < N1 * N1C;
        const int xa = q % N1, zb = ylane ? q / N1 : 0;
        T ry[N1C];
#pragma unroll
        for (int b1 = 0; b1 < N1C; ++b1) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc += tr.P1[0][a][b1] * L.v0[PLayout<P>::at(lc, xa + N1 * a + NP * zb)];
            ry[b1] = acc;
        }
        if (inslot && ylane) {
#pragma unroll
            for (int b1 = 0; b1 < N1C; ++b1) L.v1[PLayout<P>::at(lc, xa + N1 * b1 + N1 * N1C * zb)] = ry[b1];   // [x][y c][z c]
        }
        wave_sync();
        // along x: lane q < N1C^2 takes coarse (y, z) = (q % N1C, q / N1C)
        const bool xlane = q < N1C * N1C;
        const int yb = q % N1C, zb2 = xlane ? q / N1C : 0;
        T rx[N1C];
#pragma unroll
        for (int b0 = 0; b0 < N1C; ++b0) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc += tr.P1[0][a][b0] * L.v1[PLayout<P>::at(lc, a + N1 * yb + N1 * N1C * zb2)];
            rx[b0] = acc;
        }
        if (live && xlane) {
            const size_t o = (size_t)cell * NCC + N1C * (yb + N1C * zb2);
#pragma unroll
            for (int b0 = 0; b0 < N1C; ++b0) bc[o + b0] = rx[b0];
            if (zc != nullptr) {
#pragma unroll
                for (int b0 = 0; b0 < N1C; ++b0) zc[o + b0] = T(0);
            }
        }
    } else {
        if constexpr (MF) {
            // all 16 residuals of the block, then Z = B_int R: B operand R[k][j]
            // (cell slot j = lane % 16, DoF k = 4 s + lane / 16) from lane j + 16 k;
            // result D[i][j] in lane j + 16 (i / 4), register i % 4
#pragma unroll
            for (int c = 0; c < N1; ++c) sRm[(q + NP * c) * RS + lc] = bv[c] - y[c];
            __syncthreads();
            typedef typename Tile16<T>::v4 f4;
            f4 acc = {T(0), T(0), T(0), T(0)};
            const int col = lane % 16;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) acc = Tile16<T>::step(bsl[ks], sRm[(4 * ks + lane / 16) * RS + col], acc);
            const int ccell = scell[col];
            if (ccell >= 0) {
                const size_t o = (size_t)ccell * NC + 16 * wave;
                const int g = lane / 16;
                if constexpr (sizeof(T) == 4) {
                    // rows 4 g .. 4 g + 3: one vector access
                    f4 old = *reinterpret_cast<const f4 *>(xin + o + 4 * g);
                    f4 nw;
#pragma unroll
                    for (int r = 0; r < 4; ++r) nw[r] = old[r] + R.omega * acc[r];
                    *reinterpret_cast<f4 *>(out + o + 4 * g) = nw;
                    if constexpr (F64OUT) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) z64[o + 4 * g + r] = (double)nw[r];
                    }
                } else {
                    T old[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) old[r] = xin[o + Tile16<T>::row(g, r)];
#pragma unroll
                    for (int r = 0; r < 4; ++r) out[o + Tile16<T>::row(g, r)] = old[r] + R.omega * acc[r];
                }
            }
            return;
        }
        wave_sync();   // the z stage has read v0
        if (inslot) {
#pragma unroll
            for (int c = 0; c < N1; ++c) L.v0[PLayout<P>::at(lc, q + NP * c)] = bv[c] - y[c];
        }
        wave_sync();
        if constexpr (SBL) __syncthreads();   // the staged inverse
        T corr[N1];
        interior_correction<P, T, SBL>(sB, Bint_t, L.v0 + PLayout<P>::at(lc, 0), q, corr);
        if (live) {
#pragma unroll
            for (int c = 0; c < N1; ++c) {
                const T xn = xz[c] + R.omega * corr[c];
                oc[q + NP * c] = xn;
                if constexpr (F64OUT) z64[(size_t)cell * NC + q + NP * c] = (double)xn;
            }
        }
    }
}

}  // namespace sbm
