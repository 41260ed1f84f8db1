// HIP kernels for gfx950 (CDNA4, wave64): DG-SBM cell operator (apply,
// residual, red-black cell-block smoother), h/p transfers, coarse solve,
// FGMRES vector kernels and precision casts.
//
// Operator (paper Sec. 2.2, full DG-SBM bilinear form; Sec. 2.1 extension):
// on a Cartesian cell of size h, in reference units and scaled by h^(d-2),
//   (A u)_K = sum_k (M x .. x T_k x .. x M) u_K              volume + unshifted face self terms
//           + sum_{interior faces} (M x M)_tangential C_f u_N  SIPG coupling to the neighbour
//           + sum_{surrogate faces} S_f u_K                    shift part of the Nitsche terms
// with T_k chosen by the face types of the two faces normal to e_k.  The
// volume/self part is applied by sum factorisation (one 1D contraction per
// direction and operand), the couplings through the neighbour's trace and
// normal derivative on the shared face, the shift part at the face Gauss points.
//
// Thread mapping: one thread per DoF, 64 / (p+1)^d cells per wave (a cell
// never straddles a wave, so the cell's threads exchange LDS data without
// block barriers), 2 waves per block, one batch of cells per block; cell data staged in
// LDS.  The
// block index is remapped so that each of the 8 XCDs works on a contiguous
// range of cells (neighbour traces then hit that XCD's L2).
#include <type_traits>

#include "kernels.hpp"
#include "device_util.hpp"
#include "pencil_body.hpp"

namespace sbm {

template <int D, int P>
struct Sh {
    static constexpr int N1 = P + 1;
    static constexpr int NC = D == 2 ? N1 * N1 : N1 * N1 * N1;
    static constexpr int NF = D == 2 ? N1 : N1 * N1;
    static constexpr int CPW = 64 / NC;
    static constexpr int WAVES = cell_waves(NC);
    static constexpr int CPB = CPW * WAVES;
    static constexpr int NFACE = 2 * D;
};

// DoF index of node (m along direction k, tangential index j) of a cell
template <int D, int P>
__device__ __forceinline__ int compose(int k, int m, int j) {
    constexpr int N1 = P + 1;
    if (D == 2) {
        return k == 0 ? m + N1 * j : j + N1 * m;
    } else {
        int j1 = j % N1, j2 = j / N1;
        if (k == 0) return m + N1 * (j1 + N1 * j2);
        if (k == 1) return j1 + N1 * (m + N1 * j2);
        return j1 + N1 * (j2 + N1 * m);
    }
}

// node coordinate along k and tangential index of DoF i
template <int D, int P>
__device__ __forceinline__ void decompose(int i, int k, int &m, int &j) {
    constexpr int N1 = P + 1;
    int c0 = i % N1, c1 = (i / N1) % N1, c2 = D == 3 ? i / (N1 * N1) : 0;
    if (D == 2) {
        m = k == 0 ? c0 : c1;
        j = k == 0 ? c1 : c0;
    } else {
        if (k == 0) { m = c0; j = c1 + N1 * c2; }
        else if (k == 1) { m = c1; j = c0 + N1 * c2; }
        else { m = c2; j = c0 + N1 * c1; }
    }
}

// Lagrange basis of the nodes at x in barycentric form: v_a = bw_a prod_{b != a} (x - x_b)
template <typename T, int N1>
__device__ __forceinline__ void lagrange_dev(const T *nodes, const T *bw, T x, T *v) {
#pragma unroll
    for (int a = 0; a < N1; ++a) {
        T num = bw[a];
#pragma unroll
        for (int b = 0; b < N1; ++b)
            if (b != a) num *= x - nodes[b];
        v[a] = num;
    }
}

// --------------------------------------------------------------------------
// Cell operator.
//  OP_APPLY : out = A x
//  OP_RESID : out = b - A x
//  OP_SMOOTH: x (= out, in place) += omega * B_K (b - A x)_K on cells [cell0, cell0+ncells)

// LDS of one block of NW waves (CPW cells per wave)
template <int D, int P, typename T, int NW>
struct CellLds {
    static constexpr int NC = Sh<D, P>::NC, NF = Sh<D, P>::NF, NFACE = 2 * D, CPB = NW * Sh<D, P>::CPW;
    T su[CPB][NC];
    T sa[CPB][NC];
    T sb[CPB][NC];
    T fa[CPB][NFACE][NF];
    T fb[CPB][NFACE][NF];
    T ga[CPB][NFACE][NF];
    T gb[CPB][NFACE][NF];
    int snb[CPB][NFACE];
};

struct NoHook {
    __device__ void operator()() const {}
};

// Block-wide copy of a small table (W 32-bit words, NT threads) into LDS in
// two halves: load() issues all of this thread's loads, store() writes them,
// so that the kernel's other first loads go out in between.  (A plain copy
// loop waits for each load before its LDS write: one memory round trip per
// iteration, ahead of everything else.)
template <int W, int NT>
struct Stager {
    static constexpr int PER = (W + NT - 1) / NT;
    unsigned v[PER];
    __device__ __forceinline__ void load(const void *src) {
        const unsigned *s = reinterpret_cast<const unsigned *>(src);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int t = (int)threadIdx.x + k * NT;
            v[k] = t < W ? s[t] : 0u;
        }
    }
    __device__ __forceinline__ void store(void *dst) const {
        unsigned *d = reinterpret_cast<unsigned *>(dst);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int t = (int)threadIdx.x + k * NT;
            if (t < W) d[t] = v[k];
        }
    }
};

// EMIT (OP_SMOOTH only): see EmitArgs; e is an EmitArgs<T> unless EMIT_NONE,
// sP the LDS copy of the fine-by-coarse 1D embedding [2][N1E][N1].  hook()
// runs once the cell data have arrived, before the neighbour loads: a caller
// issues loads there whose addresses depend on loads it issued before the batch.
// One batch of cells [bstart, bend), at most NW * CPW of them: wave w takes the
// cells bstart + w * CPW + (0 .. CPW-1), one thread per DoF.  R and sB (the
// transposed interior-cell inverse, OP_SMOOTH) are block-shared LDS copies,
// written by stage() and read after a block barrier, so that their staging
// overlaps the batch's cell-data loads.
//
// Every global load is issued as early as its address is known, so that a
// batch costs three dependent memory round trips (cell data; neighbour traces,
// shift vectors and the boundary-cell inverse; the store) rather than one per
// stage: small levels are bound by this latency.
// stage(): the block's LDS staging writes (sR, sB, ...), called once the cell
// data loads are issued and before the barrier that guards those tables.
template <int D, int P, typename T, int OP, int NW, int EMIT = EMIT_NONE, typename EA = int, typename Hook = NoHook,
          typename Stage = NoHook>
__device__ __forceinline__ void cell_batch(CellLds<D, P, T, NW> &L, const T *sB, int bstart, int bend,
                                           const T *xin, T *out, const T *__restrict__ b, const CellArgs<T> &a,
                                           const KRef<T> &R, const int *__restrict__ perm = nullptr,
                                           const EA &e = EA(), const T *sP = nullptr, Hook hook = Hook(),
                                           Stage stage = Stage()) {
    using S = Sh<D, P>;
    static_assert(EMIT == EMIT_NONE || OP == OP_SMOOTH, "only the smoother sends values on");
    static_assert(EMIT != EMIT_H || P == 1, "h-transfers are between Q1 levels");
    constexpr int N1 = S::N1, NC = S::NC, NF = S::NF, NFACE = S::NFACE;
    auto &su = L.su;
    auto &sa = L.sa;
    auto &sb = L.sb;
    auto &fa = L.fa;
    auto &fb = L.fb;
    auto &ga = L.ga;
    auto &gb = L.gb;
    auto &snb = L.snb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool slot = lane < S::CPW * NC;
    const int lc = slot ? wave * S::CPW + lane / NC : 0;
    const int i = slot ? lane % NC : 0;
    // with perm, batch slot e takes the cell perm[e] (-1: no cell)
    const int slotpos = bstart + lc;
    const int cell = perm != nullptr ? (slot && slotpos < bend ? perm[slotpos] : -1) : slotpos;
    const bool live = slot && slotpos < bend && cell >= 0;
    wave_sync();  // the previous batch is done with this wave's LDS slices

    // all of the cell's loads first, then the LDS writes that need them
    T bval = 0, xv = 0;
    int bi = -1, nbv = 0;
    if (live) {
        xv = xin[(size_t)cell * NC + i];
        if (i < NFACE) nbv = a.nbr[(size_t)cell * NFACE + i];
        if (OP != OP_APPLY) bval = b[(size_t)cell * NC + i];
        if (OP == OP_SMOOTH) bi = a.bnd_of[cell];
    }
    // emission: the fine cell this thread writes (h: child i of the cell; p:
    // the same cell, outputs i, i + NC, ...) and its old values
    constexpr bool EPRO = EMIT == EMIT_H || EMIT == EMIT_P;
    constexpr int N1E = EMIT == EMIT_P ? N1 + 1 : N1;
    constexpr int NCE = D == 2 ? N1E * N1E : N1E * N1E * N1E;
    constexpr int NOUT = EMIT == EMIT_H ? NCE : (NCE + NC - 1) / NC;
    int efc = -1;
    T ezf[EPRO ? NOUT : 1];
    if constexpr (EPRO) {
        if (live) efc = EMIT == EMIT_H ? e.children[(size_t)cell * NC + i] : e.children[cell];
    }
    stage();
    if (live) {
        su[lc][i] = xv;
        if (i < NFACE) snb[lc][i] = nbv;
    }
    wave_sync();
    __syncthreads();   // R, sB and the embedding staged
    hook();
    if constexpr (EPRO) {
        if (efc >= 0) {
#pragma unroll
            for (int k = 0; k < NOUT; ++k) {
                const int ao = EMIT == EMIT_H ? k : i + k * NC;
                ezf[k] = e.zf[(size_t)efc * NCE + (ao < NCE ? ao : NCE - 1)];   // (clamped, not guarded)
            }
        }
    }

    // Face items (face f, tangential index j) handled by this thread: the
    // neighbour's nodes on the line through the face point (interior
    // faces) or the shift vector at the face Gauss point (surrogate
    // faces).  Loaded here, consumed after the volume stage.
    constexpr int ITEMS = (NFACE * NF + NC - 1) / NC;
    // Register budget (measured on the 3D Q2 and Q3 solves): the boundary-cell
    // inverse column stays in registers up to 16 entries; the shift-stage loops
    // unroll fully up to 16 DoFs per cell, and for 27 in FP32 (1.5 % on the 3D
    // Q2 solve; FP64 loses 9 % that way and unrolls by 9); 64-DoF cells unroll
    // by 8 (better than 1 by 8 % and than 16 by 9 % on the 3D Q3 solve): the
    // latency of dependent LDS reads traded against occupancy.
    constexpr bool PRE_B = NC <= 16;
    constexpr int SHIFT_UNROLL = NC <= 16 ? NC : (NC <= 27 ? (sizeof(T) == 4 ? 27 : 9) : 8);
    constexpr int CORR_UNROLL = NC <= 27 ? NC : 8;
    T raw[ITEMS][N1];
    T dqr[ITEMS][D];
    T bcol[PRE_B ? NC : 1];
    if (live) {
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            int it = i + q * NC;
            if (it < NFACE * NF) {
                int f = it / NF, j = it % NF, k = f >> 1;
                int nb = snb[lc][f];
                // the line is loaded on every face (a surrogate face reads the
                // cell's own, unused): with the two loads on exclusive branches
                // the allocator shared their registers and made the shift
                // loads wait for all the line loads
                const T *un = xin + (size_t)(nb >= 0 ? nb : cell) * NC;
#pragma unroll
                for (int m = 0; m < N1; ++m) raw[q][m] = un[compose<D, P>(k, m, j)];
                if (nb < 0) {
                    const T *dq = a.shift + ((size_t)(-nb - 1) * NF + j) * D;
#pragma unroll
                    for (int c = 0; c < D; ++c) dqr[q][c] = dq[c];
                }
            }
        }
        if (OP == OP_SMOOTH && PRE_B && bi >= 0) {
            const T *Bt = a.Bbnd_t + (size_t)bi * NC * NC;
#pragma unroll
            for (int j = 0; j < (PRE_B ? NC : 1); ++j) bcol[j] = Bt[(size_t)j * NC + i];
        }
    }
    // a held cell keeps its values to itself in this launch
    bool held = false;
    if constexpr (EMIT != EMIT_NONE) {
        if (live && bi >= 0 && e.hold != nullptr) held = e.hold[bi] != 0;
    }

    // ---------------- volume + unshifted self terms (sum factorisation)
    T y = 0;
    int c0 = i % N1, c1 = (i / N1) % N1, c2 = D == 3 ? i / (N1 * N1) : 0;
    int vx = 0, vy = 0, vz = 0;
    if (live) {
        vx = (snb[lc][0] < 0) + 2 * (snb[lc][1] < 0);
        vy = (snb[lc][2] < 0) + 2 * (snb[lc][3] < 0);
        if (D == 3) vz = (snb[lc][4] < 0) + 2 * (snb[lc][5] < 0);
        T am = 0, bt = 0;
        int base = i - c0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            T u = su[lc][base + m];
            am += R.M[c0][m] * u;
            bt += R.Tv[vx][c0][m] * u;
        }
        sa[lc][i] = am;
        sb[lc][i] = bt;
    }
    wave_sync();
    if (D == 2) {
        if (live) {
#pragma unroll
            for (int m = 0; m < N1; ++m) y += R.M[c1][m] * sb[lc][c0 + N1 * m] + R.Tv[vy][c1][m] * sa[lc][c0 + N1 * m];
        }
    } else {
        T aM = 0, aT = 0, bM = 0;
        if (live) {
            int base = i - N1 * c1;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
                T av = sa[lc][base + N1 * m], bv = sb[lc][base + N1 * m];
                aM += R.M[c1][m] * av;
                aT += R.Tv[vy][c1][m] * av;
                bM += R.M[c1][m] * bv;
            }
        }
        wave_sync();
        if (live) {
            sa[lc][i] = aM;
            sb[lc][i] = aT + bM;
        }
        wave_sync();
        if (live) {
            int base = i - N1 * N1 * c2;
#pragma unroll
            for (int m = 0; m < N1; ++m)
                y += R.M[c2][m] * sb[lc][base + N1 * N1 * m] + R.Tv[vz][c2][m] * sa[lc][base + N1 * N1 * m];
        }
    }

    // ---------------- interior-face couplings: neighbour trace and normal derivative
    if (live) {
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int it = i + q * NC;
            if (it < NFACE * NF) {
                int f = it / NF, j = it % NF, s = f & 1;
                int nb = snb[lc][f];
                T va = 0, vb = 0;
                if (nb >= 0) {
                    const T *gN = R.g[s == 1 ? 0 : 1];
                    // the trace node picked by 0/1 weights (exact), not by a
                    // select: the compiler turns a select of two elements into
                    // a dynamic index, and raw then lives in scratch memory
                    T t = 0, dn = 0;
#pragma unroll
                    for (int m = 0; m < N1; ++m) {
                        t += T(m == (s == 1 ? 0 : P)) * raw[q][m];
                        dn += gN[m] * raw[q][m];
                    }
                    T sg = s == 1 ? T(1) : T(-1);
                    va = T(-0.5) * sg * dn - R.sigF * t;
                    vb = T(0.5) * t;
                }
                fa[lc][f][j] = va;
                fb[lc][f][j] = vb;
            }
        }
    }
    wave_sync();
    // tangential mass along the first tangential direction
    if (live) {
        for (int it = i; it < NFACE * NF; it += NC) {
            int f = it / NF, j = it % NF;
            int j1 = j % N1, rest = j - j1;
            T va = 0, vb = 0;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
                va += R.M[j1][m] * fa[lc][f][rest + m];
                vb += R.M[j1][m] * fb[lc][f][rest + m];
            }
            ga[lc][f][j] = va;
            gb[lc][f][j] = vb;
        }
    }
    wave_sync();
    if (D == 3) {
        if (live) {
            for (int it = i; it < NFACE * NF; it += NC) {
                int f = it / NF, j = it % NF;
                int j1 = j % N1, j2 = j / N1;
                T va = 0, vb = 0;
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    va += R.M[j2][m] * ga[lc][f][j1 + N1 * m];
                    vb += R.M[j2][m] * gb[lc][f][j1 + N1 * m];
                }
                fa[lc][f][j] = va;
                fb[lc][f][j] = vb;
            }
        }
        wave_sync();
    }
    if (live) {
#pragma unroll
        for (int f = 0; f < NFACE; ++f) {
            if (snb[lc][f] < 0) continue;
            int k = f >> 1, s = f & 1, m, j;
            decompose<D, P>(i, k, m, j);
            T ev = (m == (s ? P : 0)) ? T(1) : T(0);
            T sg = s == 1 ? T(1) : T(-1);
            T F1 = D == 3 ? fa[lc][f][j] : ga[lc][f][j];
            T F2 = D == 3 ? fb[lc][f][j] : gb[lc][f][j];
            y += ev * F1 + sg * R.g[s][m] * F2;
        }
    }
    wave_sync();

    // ---------------- shift part of the Nitsche terms on surrogate faces
    bool bnd = false;
    if (live) {
#pragma unroll
        for (int f = 0; f < NFACE; ++f) bnd |= snb[lc][f] < 0;
    }
    if (live && bnd) {
#pragma unroll
        for (int qi = 0; qi < ITEMS; ++qi) {
            const int it = i + qi * NC;
            if (it >= NFACE * NF) break;
            int f = it / NF, q = it % NF, k = f >> 1, s = f & 1;
            int nb = snb[lc][f];
            T zeta = 0;
            if (nb < 0) {
                const T *dq = dqr[qi];
                int q1 = q % N1, q2 = D == 3 ? q / N1 : 0;
                T wq = R.w[q1] * (D == 3 ? R.w[q2] : T(1));
                const int layer = s ? P : 0;
                T E = 0;
                // boundary cells only: the loops are unrolled (independent LDS
                // reads in flight together) except for the largest cells, where
                // they stay rolled to bound the register pressure
                if (R.ext == 0) {
                    // gradient of u at the face Gauss point
                    T dk = 0, dt1 = 0, dt2 = 0;
#pragma unroll(SHIFT_UNROLL)
                    for (int j = 0; j < NF; ++j) {
                        int j1 = j % N1, j2 = D == 3 ? j / N1 : 0;
                        T s1 = R.S[q1][j1], s2 = D == 3 ? R.S[q2][j2] : T(1);
                        T d1 = R.Sd[q1][j1], d2 = D == 3 ? R.Sd[q2][j2] : T(0);
                        T nd = 0;
#pragma unroll
                        for (int m = 0; m < N1; ++m) nd += R.g[s][m] * su[lc][compose<D, P>(k, m, j)];
                        T ul = su[lc][compose<D, P>(k, layer, j)];
                        dk += s1 * s2 * nd;
                        dt1 += d1 * s2 * ul;
                        if (D == 3) dt2 += s1 * d2 * ul;
                    }
                    int t1 = k == 0 ? 1 : 0;
                    int t2 = k == 2 ? 1 : 2;
                    // components picked with selects: dq lives in registers
                    const T dk_k = k == 0 ? dq[0] : (k == 1 ? dq[1] : dq[D - 1]);
                    const T dk_t1 = t1 == 0 ? dq[0] : dq[1];
                    E = dk_k * dk + dk_t1 * dt1;
                    if (D == 3) E += (t2 == 1 ? dq[1] : dq[D - 1]) * dt2;
                } else {
                    // cell polynomial at the shifted point minus its value at the face point
                    T lv[3][N1];
                    const int t1 = k == 0 ? 1 : 0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        T xc = c == k ? T(s) : (c == t1 ? R.gq[q1] : R.gq[q2]);
                        lagrange_dev<T, N1>(R.x, R.bw, xc + dq[c], lv[c]);
                    }
                    // sum factorised: x first (contiguous nodes), then y, then z
                    T acc = 0;
#pragma unroll
                    for (int a2 = 0; a2 < (D == 3 ? N1 : 1); ++a2) {
                        T s2 = 0;
#pragma unroll
                        for (int a1 = 0; a1 < N1; ++a1) {
                            T s1 = 0;
#pragma unroll
                            for (int a0 = 0; a0 < N1; ++a0) s1 += lv[0][a0] * su[lc][a0 + N1 * (a1 + N1 * a2)];
                            s2 += lv[1][a1] * s1;
                        }
                        acc += (D == 3 ? lv[2][a2] : T(1)) * s2;
                    }
                    T face = 0;
#pragma unroll
                    for (int j2 = 0; j2 < (D == 3 ? N1 : 1); ++j2) {
                        T f1 = 0;
#pragma unroll
                        for (int j1 = 0; j1 < N1; ++j1)
                            f1 += R.S[q1][j1] * su[lc][compose<D, P>(k, layer, j1 + N1 * j2)];
                        face += (D == 3 ? R.S[q2][j2] : T(1)) * f1;
                    }
                    E = acc - face;
                }
                zeta = wq * E;
            }
            fa[lc][f][q] = zeta;
        }
    }
    wave_sync();
    if (live && bnd) {
#pragma unroll
        for (int f = 0; f < NFACE; ++f) {
            if (snb[lc][f] >= 0) continue;
            int k = f >> 1, s = f & 1, m, j;
            decompose<D, P>(i, k, m, j);
            T sg = s == 1 ? T(1) : T(-1);
            T ev = (m == (s ? P : 0)) ? T(1) : T(0);
            T coef = -R.alpha * sg * R.g[s][m] + R.sigG * ev;
            int j1 = j % N1, j2 = D == 3 ? j / N1 : 0;
            T acc = 0;
#pragma unroll(SHIFT_UNROLL)
            for (int q = 0; q < NF; ++q) {
                int q1 = q % N1, q2 = D == 3 ? q / N1 : 0;
                T sv = R.S[q1][j1] * (D == 3 ? R.S[q2][j2] : T(1));
                acc += fa[lc][f][q] * sv;
            }
            y += coef * acc;
        }
    }

    // ---------------- output
    y *= R.scale;
    if (OP == OP_APPLY) {
        if (live) out[(size_t)cell * NC + i] = y;
    } else if (OP == OP_RESID) {
        if (live) out[(size_t)cell * NC + i] = bval - y;
    } else if (OP == OP_RESTRICT) {
        // the residual stays in LDS for the restriction that follows
        wave_sync();
        if (slot) sa[lc][i] = live ? bval - y : T(0);
        wave_sync();
    } else {
        wave_sync();
        if (live) sa[lc][i] = bval - y;
        wave_sync();
        T xnew = 0;
        if (live) {
            T corr = 0;
            if (bi < 0 && NC <= 27) {
#pragma unroll(CORR_UNROLL)
                for (int j = 0; j < NC; ++j) corr += sB[j * NC + i] * sa[lc][j];
            } else if (PRE_B) {
#pragma unroll
                for (int j = 0; j < (PRE_B ? NC : 1); ++j) corr += bcol[j] * sa[lc][j];
            } else {
                // large blocks: the column in groups of G loads in flight (the
                // last group is cut at NC); FP32 takes 32 (two round trips for
                // a 64-DoF cell instead of four), FP64 16 (register budget)
                constexpr int G = sizeof(T) == 4 ? 32 : 16;
                const T *Bt = (NC > 27 && bi < 0) ? a.Bint_t : a.Bbnd_t + (size_t)bi * NC * NC;
#pragma unroll 1
                for (int j0 = 0; j0 < NC; j0 += G) {
                    T col[G];
#pragma unroll
                    for (int j = 0; j < G; ++j) col[j] = Bt[(size_t)min(j0 + j, NC - 1) * NC + i];   // (clamped)
#pragma unroll
                    for (int j = 0; j < G; ++j)
                        if (j0 + j < NC) corr += col[j] * sa[lc][j0 + j];
                }
            }
            if (a.lw != nullptr && bi >= 0) {
                const T *U = a.lU + (size_t)bi * NC * 4;
                const T *V = a.lV + (size_t)bi * NC * 4;
                T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
#pragma unroll(CORR_UNROLL)
                for (int j = 0; j < NC; ++j) {
                    T r = sa[lc][j];
                    v0 += V[j * 4 + 0] * r;
                    v1 += V[j * 4 + 1] * r;
                    v2 += V[j * 4 + 2] * r;
                    v3 += V[j * 4 + 3] * r;
                }
                corr += U[i * 4 + 0] * v0 + U[i * 4 + 1] * v1 + U[i * 4 + 2] * v2 + U[i * 4 + 3] * v3;
                corr *= a.lw[bi];
            }
            xnew = su[lc][i] + R.omega * corr;
            out[(size_t)cell * NC + i] = xnew;
            if constexpr (EMIT == EMIT_F64) {
                if (!held) e.z64[(size_t)cell * NC + i] = (double)xnew;
            }
        }
        if constexpr (EPRO) {
            // the cell's new values to all its lanes, then zf += E z (Sec. 3.2
            // embedding, same products and order as the prolongation kernel)
            wave_sync();
            if (live) sb[lc][i] = xnew;
            wave_sync();
            if (efc >= 0 && !held) {
                const int o = EMIT == EMIT_H ? i : 0;
#pragma unroll
                for (int k = 0; k < NOUT; ++k) {
                    const int ao = EMIT == EMIT_H ? k : i + k * NC;
                    if (ao < NCE) {
                        const int a0 = ao % N1E, a1 = (ao / N1E) % N1E, a2 = D == 3 ? ao / (N1E * N1E) : 0;
                        T acc = 0;
#pragma unroll
                        for (int j = 0; j < NC; ++j) {
                            const int j0 = j % N1, j1 = (j / N1) % N1, j2 = D == 3 ? j / (N1 * N1) : 0;
                            T w = sP[((o & 1) * N1E + a0) * N1 + j0] * sP[(((o >> 1) & 1) * N1E + a1) * N1 + j1];
                            if (D == 3) w *= sP[(((o >> 2) & 1) * N1E + a2) * N1 + j2];
                            acc += w * sb[lc][j];
                        }
                        e.zf[(size_t)efc * NCE + ao] = ezf[k] + acc;
                    }
                }
            }
        }
    }
}

template <typename T, int EMIT>
struct EmitParam {
    using type = EmitArgs<T>;
};
template <typename T>
struct EmitParam<T, EMIT_NONE> {
    using type = int;
};

// Occupancy floor handed to the register allocator (waves per SIMD): the 3D
// Q2 colour updates are otherwise allocated just above a boundary, 170 VGPRs
// in FP64 and 97 in FP32, and fit 168 (3 waves) and 96 (5 waves); measured on
// the 3D Q2 solve: FP64 10 % and FP32 4 % faster.
// (The p-prolongation form, which would spill, keeps the default.)
// The 3D Q3 FP32 kernels ask for 5: the colour update then fits 76 VGPRs (6
// waves) instead of the 120 it is given by default, with no spill (3D Q3 FP32
// solve 8 % faster).  The FP64 forms would fit 96 only by spilling, which was
// 1.5 % faster but doubled the apply's HBM traffic, so they keep 4 waves.
template <int D, int P, typename T, int OP, int EMIT>
constexpr int cell_min_waves() {
    return (D == 3 && P == 2 && OP == OP_SMOOTH && EMIT != EMIT_P) ? (sizeof(T) == 8 ? 3 : 5)
         : (D == 3 && P == 3 && sizeof(T) == 4) ? 5 : 1;
}

template <int D, int P, typename T, int OP, int EMIT = EMIT_NONE>
__global__ __launch_bounds__((64 * Sh<D, P>::WAVES))
__attribute__((amdgpu_waves_per_eu(cell_min_waves<D, P, T, OP, EMIT>(), 8))) void cellop_kernel(int cell0, int ncells, const T *xin, T *out,
                                                    const T *__restrict__ b, CellArgs<T> a, KRef<T> Rarg,
                                                    typename EmitParam<T, EMIT>::type e) {
    using S = Sh<D, P>;
    constexpr int N1 = S::N1, NC = S::NC, CPB = S::CPB;
    constexpr bool EPRO = EMIT == EMIT_H || EMIT == EMIT_P;
    constexpr int N1E = EMIT == EMIT_P ? N1 + 1 : N1;
    __shared__ CellLds<D, P, T, S::WAVES> L;
    // shared interior-cell inverse (up to 27 DoFs per cell; 64-DoF cells read its
    // columns from memory like the boundary blocks: staging 16-32 KB per block
    // cost more than it saved)
    constexpr bool SB = OP == OP_SMOOTH && NC <= 27;
    __shared__ T sB[SB ? NC * NC : 1];
    __shared__ KRef<T> sR;
    __shared__ T sP[EPRO ? 2 * N1E * N1 : 1];     // embedding for the emission
    // The reference data are indexed per lane; read from the kernel arguments
    // every access would be a memory round trip on the critical path.  Their
    // loads go out first; the LDS writes follow the cell data loads.
    static_assert(sizeof(KRef<T>) % 4 == 0, "KRef is copied as 32-bit words");
    constexpr int NT = 64 * S::WAVES;
    Stager<(int)(sizeof(KRef<T>) / 4), NT> kst;
    kst.load(&Rarg);
    Stager<SB ? (int)(NC * NC * sizeof(T) / 4) : 1, NT> bst;
    if constexpr (SB) bst.load(a.Bint_t);
    static_assert(!EPRO || 2 * N1E * N1 <= NT, "one embedding entry per thread");
    T pv = 0;
    if constexpr (EPRO) {
        const int t = threadIdx.x;
        if (t < 2 * N1E * N1) pv = e.P1[t / (N1E * N1)][(t / N1) % N1E][t % N1];
    }
    auto stage = [&]() {
        kst.store(&sR);
        if constexpr (SB) bst.store(sB);
        if constexpr (EPRO) {
            if ((int)threadIdx.x < 2 * N1E * N1) sP[threadIdx.x] = pv;
        }
    };
    // One batch per block.  (A batch loop would cost registers even when it runs
    // once: the compiler keeps per-batch values live across iterations, e.g.
    // 62 -> 128 VGPRs for the 2D Q2 FP32 smoother, halving its occupancy.)  The
    // remap gives every XCD a contiguous range of cells.
    const int bb = xcd_remap(blockIdx.x, gridDim.x);
    int bstart, bend;
    if (a.perm != nullptr) {
        bstart = bb * CPB;
        bend = ncells;
    } else if (a.batch_start != nullptr) {
        bstart = a.batch_start[bb];
        bend = min(bstart + CPB, bstart < a.split ? a.split : cell0 + ncells);
    } else {
        bstart = cell0 + bb * CPB;
        bend = cell0 + ncells;
    }
    cell_batch<D, P, T, OP, S::WAVES, EMIT, typename EmitParam<T, EMIT>::type, NoHook, decltype(stage)>(
        L, sB, bstart, bend, xin, out, b, a, sR, a.perm, e, sP, NoHook(), stage);
}

// A whole-level operation (apply, residual) or a colour update of a 3D Q2/Q3
// level in one launch (FP32; the FP64 forms run as two launches, whose
// separate register budgets measured faster): its first nb_bnd blocks take the boundary cells
// (bcells, one thread per DoF, four waves per block), the others the interior
// cells (pcells, the pencil form).  The boundary blocks come first, so that
// their longer dependent chains start early and the interior blocks fill the
// machine around them; nb_bnd is a multiple of 8, so the interior blocks keep
// the XCD-contiguous order.  The two kinds of block never share a block, so
// their LDS is one union.
template <int P, typename T, int OP>
struct FusedCellLds {
    CellLds<3, P, T, 4> L;
    KRef<T> sR;
};
template <int P, typename T, int OP>
union FusedLds {
    PencilShared<P, T, OP> p;
    FusedCellLds<P, T, OP> c;
};

// occupancy floor for the FP32 forms (Q3: 6 waves per SIMD, the LDS limit of
// its 4-wave blocks, both parts within 80 VGPRs without a spill; Q2: 5); the
// FP64 forms would spill
template <int P, typename T>
constexpr int fused_min_waves() {
    return sizeof(T) == 4 ? (P == 3 ? 6 : 5) : 1;
}

template <int P, typename T, int OP, int EMIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fused_min_waves<P, T>(), 8))) void fused_cell_kernel(int nb_bnd, int nbnd, const int *__restrict__ bcells,
                                                         int npen, const int *__restrict__ pcells, const T *xin,
                                                         T *out, const T *__restrict__ b, CellArgs<T> a, KRef<T> R,
                                                         typename EmitParam<T, EMIT>::type e) {
    static_assert(EMIT == EMIT_NONE || EMIT == EMIT_F64, "the pencil form sends values on in FP64 only");
    __shared__ FusedLds<P, T, OP> U;
    // Blocks go in groups of 8 consecutive ones (one per XCD), each group all
    // boundary or all interior.  Q3: the nb_bnd / 8 boundary groups are spread
    // evenly over the first three quarters of the grid (boundary group i at
    // group floor(i * span / nbg)), so the boundary cells' long dependent
    // chains overlap the interior blocks' streaming (96^3 sphere colour update
    // 69.8 -> 65.8 us; spread over the whole grid the last boundary blocks
    // start late and form a tail).  Q2 keeps them first (span = nbg): its
    // smaller grids lost 0.5-1.5 us with either spread.  The last, possibly
    // partial, group is always interior, and an interior block's index keeps
    // the XCD of its position, as the tile mapping of pencil_block expects.
    constexpr int SPREAD_NUM = P == 3 ? 3 : 0, SPREAD_DEN = 4;
    const int S = (int)(blockIdx.x >> 3), x = (int)(blockIdx.x & 7);
    const int ng = (int)((gridDim.x + 7) >> 3), nbg = nb_bnd >> 3;
    const int span = max(nbg, ng * SPREAD_NUM / SPREAD_DEN);
    // boundary groups before group S, and whether S is one
    const int gi = nbg == 0 ? 0 : min((int)(((long long)S * nbg + span - 1) / span), nbg);
    const bool isb = gi < nbg && (int)(((long long)gi * span) / nbg) == S;
    if (isb) {
        const int blk = gi * 8 + x;
        constexpr int NW = 4, CPB = Sh<3, P>::CPW * NW;
        Stager<(int)(sizeof(KRef<T>) / 4), 64 * NW> kst;
        kst.load(&R);
        auto stage = [&]() { kst.store(&U.c.sR); };
        cell_batch<3, P, T, OP, NW, EMIT, typename EmitParam<T, EMIT>::type, NoHook, decltype(stage)>(
            U.c.L, nullptr, blk * CPB, nbnd, xin, out, b, a, U.c.sR, bcells, e, nullptr, NoHook(), stage);
    } else {
        double *z64 = nullptr;
        if constexpr (EMIT == EMIT_F64) z64 = e.z64;
        const int nbp = (int)gridDim.x - nb_bnd;
        pencil_block<P, T, OP, EMIT == EMIT_F64>(xcd_remap((S - gi) * 8 + x, nbp), U.p, npen, pcells, xin, out, b, a.nbr,
                                                 a.Bint_t, R, z64, nullptr, nullptr, TransferArgs<T>{});
    }
}

template <int P, typename T>
static int launch_fused_p(int op, int nbnd, const int *bcells, int npen, const int *pcells, const T *x, T *y,
                          const T *b, const CellArgs<T> &a, const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e) {
    constexpr int BCPB = Sh<3, P>::CPW * 4;
    const int nb_bnd = ((nbnd + BCPB - 1) / BCPB + 7) / 8 * 8;
    const int nb_pen = (npen + PSh<P>::CPB - 1) / PSh<P>::CPB;
    if (nb_pen == 0 && nbnd == 0) return 0;
    const dim3 g(nb_bnd + nb_pen), bl(256);
    const bool f64 = e != nullptr;
    if (f64 && (e->kind != EMIT_F64 || e->z64 == nullptr || op != OP_SMOOTH)) return -1;
    if (op == OP_APPLY)
        hipLaunchKernelGGL((fused_cell_kernel<P, T, OP_APPLY, EMIT_NONE>), g, bl, 0, st, nb_bnd, nbnd, bcells, npen,
                           pcells, x, y, b, a, R, 0);
    else if (op == OP_RESID)
        hipLaunchKernelGGL((fused_cell_kernel<P, T, OP_RESID, EMIT_NONE>), g, bl, 0, st, nb_bnd, nbnd, bcells, npen,
                           pcells, x, y, b, a, R, 0);
    else if (op == OP_SMOOTH && !f64)
        hipLaunchKernelGGL((fused_cell_kernel<P, T, OP_SMOOTH, EMIT_NONE>), g, bl, 0, st, nb_bnd, nbnd, bcells, npen,
                           pcells, x, y, b, a, R, 0);
    else if (op == OP_SMOOTH) {
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL((fused_cell_kernel<P, T, OP_SMOOTH, EMIT_F64>), g, bl, 0, st, nb_bnd, nbnd, bcells,
                               npen, pcells, x, y, b, a, R, *e);
        else
            return -1;
    } else {
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_fused(int d, int p, int op, int nbnd, const int *bcells, int npen, const int *pcells, const T *x, T *y,
                 const T *b, const CellArgs<T> &a, const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e) {
    if (!pencil_supported(d, p) || (nbnd > 0 && bcells == nullptr) || (npen > 0 && pcells == nullptr)) return -1;
    return p == 3 ? launch_fused_p<3, T>(op, nbnd, bcells, npen, pcells, x, y, b, a, R, st, e)
                  : launch_fused_p<2, T>(op, nbnd, bcells, npen, pcells, x, y, b, a, R, st, e);
}
template int launch_fused<float>(int, int, int, int, const int *, int, const int *, const float *, float *,
                                 const float *, const CellArgs<float> &, const KRef<float> &, hipStream_t,
                                 const EmitArgs<float> *);
template int launch_fused<double>(int, int, int, int, const int *, int, const int *, const double *, double *,
                                 const double *, const CellArgs<double> &, const KRef<double> &, hipStream_t,
                                 const EmitArgs<double> *);

// Residual and restriction in one launch (Sec. 3.2: the restriction is the
// transpose of the embedding); the residual is not written to memory.
//  h-transfer (nch = 2^d children): batches walk groups of child cells,
//    perm[g * nch + o] (-1 for an inactive child) of the coarse cell grp[g], so
//    that the children of a coarse cell sit in one wave; their residuals stay
//    in LDS and the wave forms bc = sum_o E_o^T r_o.
//  p-transfer (same cells, perm = nullptr): batches follow the whole-level
//    batch table and every cell restricts its own residual; or, with nch = 1
//    and perm = grp a list of cells, only those cells.
// (occupancy floor as for the cell kernels: the 3D Q2 FP64 form fits 3 waves
// per SIMD without spilling but is otherwise allocated 169 VGPRs, 2 waves; the
// 3D Q3 FP32 form fits 78 VGPRs, 6 waves, instead of 122)
template <int D, int P, typename T>
__global__ __launch_bounds__((64 * Sh<D, P>::WAVES))
__attribute__((amdgpu_waves_per_eu((D == 3 && P == 2 && sizeof(T) == 8) ? 3 : (D == 3 && P == 3 && sizeof(T) == 4) ? 5 : 1, 8))) void resid_restrict_kernel(int n_coarse, int nch, int n1c,
                                                             const int *__restrict__ perm,
                                                             const int *__restrict__ grp, const T *xin,
                                                             const T *__restrict__ b, T *__restrict__ bc,
                                                             CellArgs<T> a, KRef<T> Rarg, TransferArgs<T> tr,
                                                             ZeroStartArgs<T> zs, int c1_only) {
    using S = Sh<D, P>;
    constexpr int N1 = S::N1, NC = S::NC, CPW = S::CPW, CPB = S::CPB;
    // coarse DoFs per cell when the zero-start update is formed: h-transfers
    // are Q1 -> Q1, p-transfers Q(P) -> Q(P-1)
    constexpr int NCC = P == 1 ? NC : (D == 2 ? P * P : P * P * P);
    constexpr bool ZPRE = NCC <= 16;   // inverse column in registers
    __shared__ CellLds<D, P, T, S::WAVES> L;
    __shared__ KRef<T> sR;
    __shared__ T sP[2][N1][MAXN1];
    // staging loads first, their LDS writes after the batch's cell data loads
    constexpr int NT = 64 * S::WAVES;
    Stager<(int)(sizeof(KRef<T>) / 4), NT> kst;
    kst.load(&Rarg);
    static_assert(2 * N1 * MAXN1 <= NT, "one embedding entry per thread");
    T pv = 0;
    {
        const int t = threadIdx.x;
        if (t < 2 * N1 * MAXN1) pv = tr.P1[t / (N1 * MAXN1)][(t / MAXN1) % N1][t % MAXN1];
    }
    auto stage = [&]() {
        kst.store(&sR);
        const int t = threadIdx.x;
        if (t < 2 * N1 * MAXN1) sP[t / (N1 * MAXN1)][(t / MAXN1) % N1][t % MAXN1] = pv;
    };
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int bstart, bend;
    if (perm != nullptr) {
        bstart = blk * CPB;
        bend = n_coarse * nch;
    } else if (c1_only) {
        // the colour-0 residual vanishes: colour-1 batches only, and the
        // colour-0 part of bc (and of the zero-start z) is zero
        bstart = a.split + blk * CPB;
        bend = min(bstart + CPB, n_coarse);
        const long long nz = (long long)a.split * (D == 2 ? n1c * n1c : n1c * n1c * n1c);
        for (long long t = (long long)blk * blockDim.x + threadIdx.x; t < nz; t += (long long)gridDim.x * blockDim.x) {
            bc[t] = T(0);
            if (zs.z != nullptr) zs.z[t] = T(0);
        }
    } else {
        bstart = a.batch_start[blk];
        bend = min(bstart + CPB, bstart < a.split ? a.split : n_coarse);
    }
    // coarse DoFs of this wave's parents: CPW / nch parents, ncc DoFs each;
    // lane pp * ncc + jq forms DoF jq of parent pp
    const int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int npar = CPW / nch;
    const bool plane = lane < npar * ncc;
    const int pp = plane ? lane / ncc : 0, jq = plane ? lane % ncc : 0;
    const int g = (bstart + wave * CPW) / nch + pp;   // group (h) or cell (p) of this parent
    const bool pvalid = plane && (perm != nullptr ? g < n_coarse : g < bend);
    const bool zero_start = zs.z != nullptr;
    // read unconditionally (at a clamped group): a guarded load is sunk by the
    // compiler to its use at the end, one more dependent round trip there
    const int gc = pvalid ? g : 0;
    const int Kc = perm != nullptr ? grp[gc] : gc;
    const int zbi = zero_start ? (perm != nullptr ? zs.grp_bnd[gc] : zs.bnd_of[gc]) : -1;
    T zcol[ZPRE ? NCC : 1];
    auto hook = [&]() {
        if constexpr (ZPRE) {
            if (zero_start && pvalid) {
                const T *Bt = zbi < 0 ? zs.Bint_t : zs.Bbnd_t + (size_t)zbi * NCC * NCC;
#pragma unroll
                for (int j = 0; j < NCC; ++j) zcol[j] = Bt[(size_t)j * NCC + jq];
            }
        }
    };
    cell_batch<D, P, T, OP_RESTRICT, S::WAVES, EMIT_NONE, int, decltype(hook), decltype(stage)>(
        L, nullptr, bstart, bend, xin, nullptr, b, a, sR, perm, 0, nullptr, hook, stage);
    T acc = 0;
    if (pvalid) {
        const int j0 = jq % n1c, j1 = (jq / n1c) % n1c, j2 = D == 3 ? jq / (n1c * n1c) : 0;
        for (int o = 0; o < nch; ++o) {
            const int lc = wave * CPW + pp * nch + o;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int i0 = i % N1, i1 = (i / N1) % N1, i2 = D == 3 ? i / (N1 * N1) : 0;
                T w = sP[o & 1][i0][j0] * sP[(o >> 1) & 1][i1][j1];
                if (D == 3) w *= sP[(o >> 2) & 1][i2][j2];
                acc += w * L.sa[lc][i];
            }
        }
        bc[(size_t)Kc * ncc + jq] = acc;
    }
    if (zero_start) {
        // z_K = omega B_K bc_K (colour 0) or 0 (colour 1), in the order of the
        // zero-start smoothing kernel; the wave's bc values through its LDS slice
        T *sz = &L.sb[wave * CPW][0];
        wave_sync();
        if (pvalid) sz[lane] = acc;
        wave_sync();
        if (pvalid) {
            T zv = 0;
            if (Kc < zs.split) {
                T corr = 0;
                if constexpr (ZPRE) {
#pragma unroll
                    for (int j = 0; j < NCC; ++j) corr += zcol[j] * sz[pp * NCC + j];
                } else {
                    const T *Bt = zbi < 0 ? zs.Bint_t : zs.Bbnd_t + (size_t)zbi * NCC * NCC;
#pragma unroll 9
                    for (int j = 0; j < NCC; ++j) corr += Bt[(size_t)j * NCC + jq] * sz[pp * NCC + j];
                }
                zv = T(0) + zs.omega * corr;
            }
            zs.z[(size_t)Kc * NCC + jq] = zv;
        }
    }
}

template <int D, int P, typename T>
static int launch_rr(int n_coarse, int nch, int n1c, const int *perm, const int *grp, const T *x, const T *b, T *bc,
                     const CellArgs<T> &a, const KRef<T> &R, const TransferArgs<T> &tr, hipStream_t st,
                     const ZeroStartArgs<T> *zsp, bool c1_only) {
    using S = Sh<D, P>;
    if (n_coarse <= 0) return 0;
    if (S::CPW % nch != 0) return -1;   // a wave must hold whole child groups
    if (perm == nullptr && (nch != 1 || a.batch_start == nullptr)) return -1;
    if (c1_only && (perm != nullptr || a.split < 0 || a.split > n_coarse)) return -1;
    ZeroStartArgs<T> zs{};
    if (zsp != nullptr) {
        // the zero-start update is sized for Q1 -> Q1 (h) and Q(P) -> Q(P-1) (p);
        // with a cell list the coarse blocks come per group
        const bool h = nch != 1;
        const bool listed = !h && perm != nullptr;   // n_coarse counts the listed cells
        if ((h ? (P != 1 || n1c != 2) : (P < 2 || n1c != P)) || (perm != nullptr && zsp->grp_bnd == nullptr) ||
            zsp->z == nullptr ||
            zsp->bnd_of == nullptr || zsp->Bint_t == nullptr || zsp->split < 0 ||
            (!listed && zsp->split > n_coarse))
            return -1;
        zs = *zsp;
    }
    int nb = perm != nullptr ? (int)(((long long)n_coarse * nch + S::CPB - 1) / S::CPB) : a.nbatch;
    if (c1_only) nb = std::max(1, (n_coarse - a.split + S::CPB - 1) / S::CPB);
    hipLaunchKernelGGL((resid_restrict_kernel<D, P, T>), dim3(nb), dim3(64 * S::WAVES), 0, st, n_coarse, nch, n1c, perm, grp,
                       x, b, bc, a, R, tr, zs, c1_only ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_resid_restrict(int d, int p, int n_coarse, int nch, int n1c, const int *perm, const int *grp, const T *x,
                          const T *b, T *bc, const CellArgs<T> &a, const KRef<T> &R, const TransferArgs<T> &tr,
                          hipStream_t st, const ZeroStartArgs<T> *zs, bool c1_only) {
    if (n1c < 1 || n1c > p + 1) return -1;
    if (d == 2) {
        if (p == 1) return launch_rr<2, 1, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
        if (p == 2) return launch_rr<2, 2, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
        if (p == 3) return launch_rr<2, 3, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
    } else {
        if (p == 1) return launch_rr<3, 1, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
        if (p == 2) return launch_rr<3, 2, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
        if (p == 3) return launch_rr<3, 3, T>(n_coarse, nch, n1c, perm, grp, x, b, bc, a, R, tr, st, zs, c1_only);
    }
    return -1;
}
template int launch_resid_restrict<double>(int, int, int, int, int, const int *, const int *, const double *,
                                           const double *,
                                           double *, const CellArgs<double> &, const KRef<double> &,
                                           const TransferArgs<double> &, hipStream_t, const ZeroStartArgs<double> *,
                                           bool);
template int launch_resid_restrict<float>(int, int, int, int, int, const int *, const int *, const float *,
                                          const float *, float *,
                                          const CellArgs<float> &, const KRef<float> &, const TransferArgs<float> &,
                                          hipStream_t, const ZeroStartArgs<float> *, bool);

template <int D, int P, typename T>
static int launch_dp(int op, int cell0, int ncells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                     const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e) {
    if (ncells <= 0) return 0;
    using S = Sh<D, P>;
    int nb = a.perm == nullptr && a.batch_start != nullptr ? a.nbatch : (ncells + S::CPB - 1) / S::CPB;
    const dim3 g(nb), bl(64 * S::WAVES);
    const int kind = e != nullptr ? e->kind : EMIT_NONE;
    if (op != OP_SMOOTH && kind != EMIT_NONE) return -1;
    if (op == OP_APPLY)
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_APPLY>), g, bl, 0, st, cell0, ncells, x, y, b, a, R, 0);
    else if (op == OP_RESID)
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_RESID>), g, bl, 0, st, cell0, ncells, x, y, b, a, R, 0);
    else if (kind == EMIT_NONE)
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_SMOOTH>), g, bl, 0, st, cell0, ncells, x, y, b, a, R, 0);
    else if (kind == EMIT_F64) {
        if constexpr (std::is_same<T, float>::value) {
            if (e->z64 == nullptr) return -1;
            hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_SMOOTH, EMIT_F64>), g, bl, 0, st, cell0, ncells, x, y, b,
                               a, R, *e);
        } else {
            return -1;
        }
    } else if (kind == EMIT_H) {
        if constexpr (P == 1) {
            if (e->zf == nullptr || e->children == nullptr) return -1;
            hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_SMOOTH, EMIT_H>), g, bl, 0, st, cell0, ncells, x, y, b, a,
                               R, *e);
        } else {
            return -1;
        }
    } else if (kind == EMIT_P) {
        if constexpr (P <= 2) {
            if (e->zf == nullptr || e->children == nullptr) return -1;
            hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_SMOOTH, EMIT_P>), g, bl, 0, st, cell0, ncells, x, y, b, a,
                               R, *e);
        } else {
            return -1;
        }
    } else {
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_cellop(int d, int p, int op, int cell0, int ncells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                  const KRef<T> &R, hipStream_t st, const EmitArgs<T> *e) {
    if (d == 2) {
        if (p == 1) return launch_dp<2, 1, T>(op, cell0, ncells, x, y, b, a, R, st, e);
        if (p == 2) return launch_dp<2, 2, T>(op, cell0, ncells, x, y, b, a, R, st, e);
        if (p == 3) return launch_dp<2, 3, T>(op, cell0, ncells, x, y, b, a, R, st, e);
    } else {
        if (p == 1) return launch_dp<3, 1, T>(op, cell0, ncells, x, y, b, a, R, st, e);
        if (p == 2) return launch_dp<3, 2, T>(op, cell0, ncells, x, y, b, a, R, st, e);
        if (p == 3) return launch_dp<3, 3, T>(op, cell0, ncells, x, y, b, a, R, st, e);
    }
    return -1;
}
template int launch_cellop<double>(int, int, int, int, int, const double *, double *, const double *,
                                   const CellArgs<double> &, const KRef<double> &, hipStream_t,
                                   const EmitArgs<double> *);
template int launch_cellop<float>(int, int, int, int, int, const float *, float *, const float *,
                                  const CellArgs<float> &, const KRef<float> &, hipStream_t, const EmitArgs<float> *);

// First colour-0 update of a smoothing step that starts from z = 0: the
// residual is b itself, so colour-0 cells get z_K = omega B_K b_K (with the
// learned correction where present) and colour-1 cells z_K = 0.  One thread
// per DoF; replaces clearing z plus a full colour-0 update.
template <int D, int P, typename T, typename TB>
__device__ __forceinline__ void smooth_zero_dof(long long t, int split, const TB *__restrict__ b, T *__restrict__ z,
                                                const CellArgs<T> &a, T omega, T *__restrict__ bcopy) {
    constexpr int NC = Sh<D, P>::NC;
    const int cell = (int)(t / NC), i = (int)(t % NC);
    // the first loads together (block index, the cell's right-hand side), the
    // inverse column, whose address needs the block index, after them
    const bool c0 = cell < split;
    const int bi = a.bnd_of[cell];   // (read for every cell: no branch, no wait)
    const TB *bc = b + (size_t)cell * NC;
    // up to 16 values per cell: all loaded up front (unconditionally: every
    // cell's values are valid memory, and a guarded load would be a branch
    // with its own wait); larger cells stream them with the inverse column
    // (held in registers they would spill)
    constexpr bool PRE = NC <= 16;
    T bv[PRE ? NC : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int j = 0; j < NC; ++j) bv[j] = (T)bc[j];
    }
    if (bcopy != nullptr) bcopy[t] = (T)b[t];
    if (c0 && bi < 0 && a.skip_interior) return;   // the pencil kernel's cell
    T out = 0;
    if (c0) {
        const T *Bt = bi < 0 ? a.Bint_t : a.Bbnd_t + (size_t)bi * NC * NC;
        T corr = 0;
#pragma unroll
        for (int j = 0; j < NC; ++j) corr += Bt[(size_t)j * NC + i] * (PRE ? bv[PRE ? j : 0] : (T)bc[j]);
        if (a.lw != nullptr && bi >= 0) {
            const T *U = a.lU + (size_t)bi * NC * 4;
            const T *V = a.lV + (size_t)bi * NC * 4;
            T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
#pragma unroll 8
            for (int j = 0; j < NC; ++j) {
                T r = PRE ? bv[PRE ? j : 0] : (T)bc[j];
                v0 += V[j * 4 + 0] * r;
                v1 += V[j * 4 + 1] * r;
                v2 += V[j * 4 + 2] * r;
                v3 += V[j * 4 + 3] * r;
            }
            corr += U[i * 4 + 0] * v0 + U[i * 4 + 1] * v1 + U[i * 4 + 2] * v2 + U[i * 4 + 3] * v3;
            corr *= a.lw[bi];
        }
        out = T(0) + omega * corr;
    }
    z[t] = out;
}

// bcopy (optional): the right-hand side in the cycle precision, written as it
// is read (the FP32 cycle takes its FP64 input here instead of a cast kernel)
template <int D, int P, typename T, typename TB>
__global__ __launch_bounds__(256) void smooth_zero_kernel(int n_act, int split, const TB *__restrict__ b,
                                                          T *__restrict__ bcopy, T *__restrict__ z, CellArgs<T> a,
                                                          T omega) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n_act * Sh<D, P>::NC) return;
    smooth_zero_dof<D, P, T, TB>(t, split, b, z, a, omega, bcopy);
}

template <int D, int P, typename T, typename TB>
static int launch_sz(int n_act, int split, const TB *b, T *bcopy, T *z, const CellArgs<T> &a, T omega,
                     hipStream_t st) {
    long long n = (long long)n_act * Sh<D, P>::NC;
    if (n <= 0) return 0;
    hipLaunchKernelGGL((smooth_zero_kernel<D, P, T, TB>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_act,
                       split, b, bcopy, z, a, omega);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, typename TB>
int launch_smooth_zero(int d, int p, int n_act, int split, const TB *b, T *bcopy, T *z, const CellArgs<T> &a, T omega,
                       hipStream_t st) {
    if (d == 2) {
        if (p == 1) return launch_sz<2, 1, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
        if (p == 2) return launch_sz<2, 2, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
        if (p == 3) return launch_sz<2, 3, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
    } else {
        if (p == 1) return launch_sz<3, 1, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
        if (p == 2) return launch_sz<3, 2, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
        if (p == 3) return launch_sz<3, 3, T, TB>(n_act, split, b, bcopy, z, a, omega, st);
    }
    return -1;
}
template int launch_smooth_zero<double, double>(int, int, int, int, const double *, double *, double *,
                                                const CellArgs<double> &, double, hipStream_t);
template int launch_smooth_zero<float, float>(int, int, int, int, const float *, float *, float *,
                                              const CellArgs<float> &, float, hipStream_t);
template int launch_smooth_zero<float, double>(int, int, int, int, const double *, float *, float *,
                                               const CellArgs<float> &, float, hipStream_t);

// --------------------------------------------------------------------------
// Transfers (Sec. 3.2): prolongation = embedding of the coarse cell polynomial
// into the fine cell(s), restriction = its transpose; inactive parents give
// zero and restriction into inactive coarse cells is dropped.
template <typename T>
using P1Table = T[2][MAXN1][MAXN1];

// fine DoF gid (cell K, node i) += coarse parent polynomial at that node
template <int D, typename T>
__device__ __forceinline__ void prolong_dof(long long gid, int n1f, int n1c, const int *__restrict__ parent,
                                            const int *__restrict__ childpos, const T *__restrict__ zc,
                                            T *__restrict__ zf, const P1Table<T> &P1t) {
    int ncf = D == 2 ? n1f * n1f : n1f * n1f * n1f;
    int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    int K = (int)(gid / ncf), i = (int)(gid % ncf);
    int pc = parent[K];
    if (pc < 0) return;
    int o = childpos[K];
    int i0 = i % n1f, i1 = (i / n1f) % n1f, i2 = D == 3 ? i / (n1f * n1f) : 0;
    const T *P0 = P1t[o & 1][i0];
    const T *P1 = P1t[(o >> 1) & 1][i1];
    const T *P2 = P1t[(o >> 2) & 1][i2];
    const T *src = zc + (size_t)pc * ncc;
    T acc = 0;
    for (int j = 0; j < ncc; ++j) {
        int j0 = j % n1c, j1 = (j / n1c) % n1c, j2 = D == 3 ? j / (n1c * n1c) : 0;
        T w = P0[j0] * P1[j1];
        if (D == 3) w *= P2[j2];
        acc += w * src[j];
    }
    zf[(size_t)K * ncf + i] += acc;
}

// coarse DoF gid (cell Kc, node j) = sum over the children of the transposed embedding
template <int D, typename T>
__device__ __forceinline__ void restrict_dof(long long gid, int n1f, int n1c, int nch,
                                             const int *__restrict__ children, const T *__restrict__ rf,
                                             T *__restrict__ bc, const P1Table<T> &P1t) {
    int ncf = D == 2 ? n1f * n1f : n1f * n1f * n1f;
    int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    int Kc = (int)(gid / ncc), j = (int)(gid % ncc);
    int j0 = j % n1c, j1 = (j / n1c) % n1c, j2 = D == 3 ? j / (n1c * n1c) : 0;
    T acc = 0;
    for (int o = 0; o < nch; ++o) {
        int K = children[(size_t)Kc * nch + o];
        if (K < 0) continue;
        const T *src = rf + (size_t)K * ncf;
        for (int i = 0; i < ncf; ++i) {
            int i0 = i % n1f, i1 = (i / n1f) % n1f, i2 = D == 3 ? i / (n1f * n1f) : 0;
            T w = P1t[o & 1][i0][j0] * P1t[(o >> 1) & 1][i1][j1];
            if (D == 3) w *= P1t[(o >> 2) & 1][i2][j2];
            acc += w * src[i];
        }
    }
    bc[(size_t)Kc * ncc + j] = acc;
}

template <int D, typename T>
__global__ __launch_bounds__(256) void prolong_kernel(int n_fine, int n1f, int n1c, const int *__restrict__ parent,
                                                      const int *__restrict__ childpos, const T *__restrict__ zc,
                                                      T *__restrict__ zf, TransferArgs<T> tr) {
    int ncf = D == 2 ? n1f * n1f : n1f * n1f * n1f;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)n_fine * ncf) return;
    prolong_dof<D, T>(gid, n1f, n1c, parent, childpos, zc, zf, tr.P1);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void restrict_kernel(int n_coarse, int n1f, int n1c, int nch,
                                                       const int *__restrict__ children, const T *__restrict__ rf,
                                                       T *__restrict__ bc, TransferArgs<T> tr) {
    int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)n_coarse * ncc) return;
    restrict_dof<D, T>(gid, n1f, n1c, nch, children, rf, bc, tr.P1);
}

// The transfers that occur (h: Q1 -> Q1 with 2^d children; p: Q2 -> Q1 and
// Q3 -> Q2 on the same cell) are instantiated with their sizes fixed, so that
// every load of a thread is issued before the first product and the 1D
// embedding sits in LDS (lane-indexed reads of kernel arguments would each be
// a memory round trip).
template <int D, int N1F, int N1C, typename T>
__global__ __launch_bounds__(256) void prolong_fixed_kernel(int n_fine, const int *__restrict__ parent,
                                                            const int *__restrict__ childpos,
                                                            const T *__restrict__ zc, T *__restrict__ zf,
                                                            TransferArgs<T> tr) {
    constexpr int NCF = D == 2 ? N1F * N1F : N1F * N1F * N1F;
    constexpr int NCC = D == 2 ? N1C * N1C : N1C * N1C * N1C;
    __shared__ T sP[2][N1F][N1C];
    // every load first (the embedding entry of this thread, the parent, its
    // values, the old fine value), then the LDS write and the barrier
    static_assert(2 * N1F * N1C <= 256, "one embedding entry per thread");
    const int tp = threadIdx.x;
    const T pv = tp < 2 * N1F * N1C ? tr.P1[tp / (N1F * N1C)][(tp / N1C) % N1F][tp % N1C] : T(0);
    const long long gid0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gid0 < (long long)n_fine * NCF;
    const long long gid = live ? gid0 : 0;
    const int K = (int)(gid / NCF), i = (int)(gid % NCF);
    const T zold = zf[(size_t)K * NCF + i];
    const int pc = parent[K];
    const int o = childpos[K];
    T src[NCC];
    const T *zp = zc + (size_t)(pc < 0 ? 0 : pc) * NCC;
#pragma unroll
    for (int j = 0; j < NCC; ++j) src[j] = pc < 0 ? T(0) : zp[j];
    if (tp < 2 * N1F * N1C) sP[tp / (N1F * N1C)][(tp / N1C) % N1F][tp % N1C] = pv;
    __syncthreads();
    const int i0 = i % N1F, i1 = (i / N1F) % N1F, i2 = D == 3 ? i / (N1F * N1F) : 0;
    T acc = 0;
#pragma unroll
    for (int j = 0; j < NCC; ++j) {
        const int j0 = j % N1C, j1 = (j / N1C) % N1C, j2 = D == 3 ? j / (N1C * N1C) : 0;
        T w = sP[o & 1][i0][j0] * sP[(o >> 1) & 1][i1][j1];
        if (D == 3) w *= sP[(o >> 2) & 1][i2][j2];
        acc += w * src[j];
    }
    if (live && pc >= 0) zf[(size_t)K * NCF + i] = zold + acc;
}

template <int D, int N1F, int N1C, int NCH, typename T>
__global__ __launch_bounds__(256) void restrict_fixed_kernel(int n_coarse, const int *__restrict__ children,
                                                             const T *__restrict__ rf, T *__restrict__ bc,
                                                             TransferArgs<T> tr) {
    constexpr int NCF = D == 2 ? N1F * N1F : N1F * N1F * N1F;
    constexpr int NCC = D == 2 ? N1C * N1C : N1C * N1C * N1C;
    __shared__ T sP[2][N1F][N1C];
    for (int t = threadIdx.x; t < 2 * N1F * N1C; t += blockDim.x)
        sP[t / (N1F * N1C)][(t / N1C) % N1F][t % N1C] = tr.P1[t / (N1F * N1C)][(t / N1C) % N1F][t % N1C];
    const long long gid0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gid0 < (long long)n_coarse * NCC;
    const long long gid = live ? gid0 : 0;
    const int Kc = (int)(gid / NCC), j = (int)(gid % NCC);
    int K[NCH];
#pragma unroll
    for (int o = 0; o < NCH; ++o) K[o] = children[(size_t)Kc * NCH + o];
    T src[NCH][NCF];
#pragma unroll
    for (int o = 0; o < NCH; ++o) {
        const T *rp = rf + (size_t)(K[o] < 0 ? 0 : K[o]) * NCF;
#pragma unroll
        for (int i = 0; i < NCF; ++i) src[o][i] = K[o] < 0 ? T(0) : rp[i];
    }
    __syncthreads();
    const int j0 = j % N1C, j1 = (j / N1C) % N1C, j2 = D == 3 ? j / (N1C * N1C) : 0;
    T acc = 0;
#pragma unroll
    for (int o = 0; o < NCH; ++o) {
        if (K[o] < 0) continue;
#pragma unroll
        for (int i = 0; i < NCF; ++i) {
            const int i0 = i % N1F, i1 = (i / N1F) % N1F, i2 = D == 3 ? i / (N1F * N1F) : 0;
            T w = sP[o & 1][i0][j0] * sP[(o >> 1) & 1][i1][j1];
            if (D == 3) w *= sP[(o >> 2) & 1][i2][j2];
            acc += w * src[o][i];
        }
    }
    if (live) bc[(size_t)Kc * NCC + j] = acc;
}

template <typename T>
int launch_prolong(int d, int n_fine, int n1f, int n1c, const int *parent, const int *childpos, const T *zc, T *zf,
                   const TransferArgs<T> &tr, hipStream_t st) {
    long long n = (long long)n_fine * (d == 2 ? n1f * n1f : n1f * n1f * n1f);
    if (n <= 0) return 0;
    const dim3 g((unsigned)((n + 255) / 256)), bl(256);
#define SBM_PROLONG(DD, F, C)                                                                                  \
    if (d == DD && n1f == F && n1c == C) {                                                                    \
        hipLaunchKernelGGL((prolong_fixed_kernel<DD, F, C, T>), g, bl, 0, st, n_fine, parent, childpos, zc, zf, tr); \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                                      \
    }
    SBM_PROLONG(2, 2, 2) SBM_PROLONG(2, 3, 2) SBM_PROLONG(2, 4, 3)
    SBM_PROLONG(3, 2, 2) SBM_PROLONG(3, 3, 2) SBM_PROLONG(3, 4, 3)
#undef SBM_PROLONG
    if (d == 2)
        hipLaunchKernelGGL((prolong_kernel<2, T>), g, bl, 0, st, n_fine, n1f, n1c, parent, childpos, zc, zf, tr);
    else
        hipLaunchKernelGGL((prolong_kernel<3, T>), g, bl, 0, st, n_fine, n1f, n1c, parent, childpos, zc, zf, tr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_restrict(int d, int n_coarse, int n1f, int n1c, int nch, const int *children, const T *rf, T *bc,
                    const TransferArgs<T> &tr, hipStream_t st) {
    long long n = (long long)n_coarse * (d == 2 ? n1c * n1c : n1c * n1c * n1c);
    if (n <= 0) return 0;
    const dim3 g((unsigned)((n + 255) / 256)), bl(256);
#define SBM_RESTRICT(DD, F, C, H)                                                                              \
    if (d == DD && n1f == F && n1c == C && nch == H) {                                                        \
        hipLaunchKernelGGL((restrict_fixed_kernel<DD, F, C, H, T>), g, bl, 0, st, n_coarse, children, rf, bc, tr); \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                                      \
    }
    SBM_RESTRICT(2, 2, 2, 4) SBM_RESTRICT(2, 3, 2, 1) SBM_RESTRICT(2, 4, 3, 1)
    SBM_RESTRICT(3, 2, 2, 8) SBM_RESTRICT(3, 3, 2, 1) SBM_RESTRICT(3, 4, 3, 1)
#undef SBM_RESTRICT
    if (d == 2)
        hipLaunchKernelGGL((restrict_kernel<2, T>), g, bl, 0, st, n_coarse, n1f, n1c, nch, children, rf, bc, tr);
    else
        hipLaunchKernelGGL((restrict_kernel<3, T>), g, bl, 0, st, n_coarse, n1f, n1c, nch, children, rf, bc, tr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_prolong<double>(int, int, int, int, const int *, const int *, const double *, double *,
                                    const TransferArgs<double> &, hipStream_t);
template int launch_prolong<float>(int, int, int, int, const int *, const int *, const float *, float *,
                                   const TransferArgs<float> &, hipStream_t);
template int launch_restrict<double>(int, int, int, int, int, const int *, const double *, double *,
                                     const TransferArgs<double> &, hipStream_t);
template int launch_restrict<float>(int, int, int, int, int, const int *, const float *, float *,
                                    const TransferArgs<float> &, hipStream_t);

// --------------------------------------------------------------------------
// Coarsest level: z = A0^{-1} b with the dense inverse, accumulated in the
// matrix type TA (the FP32 cycle passes FP32 vectors and the FP64 inverse).
template <typename TA, typename TX>
__device__ __forceinline__ void gemv_row(int n, int row, const TA *__restrict__ A, const TX *__restrict__ x,
                                         TX *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const TA *a = A + (size_t)row * n;
    TA acc = 0;
    // lane sum over j = lane, lane + 64, ... in that order; 16 loads in flight
    // (loads at clamped indices, out-of-range products dropped after)
    for (int j0 = lane; j0 < n; j0 += 64 * 16) {
        TA av[16], xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = min(j0 + 64 * u, n - 1);
            av[u] = a[j];
            xv[u] = (TA)x[j];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += j0 + 64 * u < n ? av[u] * xv[u] : TA(0);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = (TX)acc;
}

template <typename TA, typename TX>
__global__ __launch_bounds__(256) void dense_gemv_kernel(int n, const TA *__restrict__ A, const TX *__restrict__ x,
                                                         TX *__restrict__ y) {
    // one wave per row: the lanes stride over the row (coalesced), then reduce
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    gemv_row(n, row, A, x, y);
}

template <typename TA, typename TX>
int launch_dense_gemv(int n, const TA *A, const TX *x, TX *y, hipStream_t st) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL((dense_gemv_kernel<TA, TX>), dim3((n + 3) / 4), dim3(256), 0, st, n, A, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_dense_gemv<double, double>(int, const double *, const double *, double *, hipStream_t);
template int launch_dense_gemv<double, float>(int, const double *, const float *, float *, hipStream_t);

// Coarsest-level solve y = Ainv x with the prolongation into the next level
// in the same launch: block K computes the rows of coarse cell K (Q1, one wave
// per row), then adds E y_K into the fine cells of K (h: its 2^d children, p:
// the same cell in Q2), as the prolongation kernel does.
template <int D, typename TX, int EMIT>
__global__ __launch_bounds__(64 * (1 << D)) void coarse_solve_prolong_kernel(int n, const double *__restrict__ A,
                                                                             const TX *__restrict__ x,
                                                                             TX *__restrict__ y, EmitArgs<TX> e) {
    static_assert(EMIT == EMIT_H || EMIT == EMIT_P, "prolongation only");
    constexpr int NCC = 1 << D;                       // Q1 coarse cell
    constexpr int N1E = EMIT == EMIT_P ? 3 : 2;       // fine nodes per direction
    constexpr int NCE = D == 2 ? N1E * N1E : N1E * N1E * N1E;
    constexpr int NOUT = EMIT == EMIT_H ? NCC * NCE : NCE;
    __shared__ TX sP[2 * N1E * 2];
    __shared__ TX sy[NCC];
    const int K = blockIdx.x, t = threadIdx.x;
    const TX pv = t < 2 * N1E * 2 ? e.P1[t / (N1E * 2)][(t / 2) % N1E][t % 2] : TX(0);
    // the fine cell this thread updates (its old value is loaded once the
    // first group of row loads is out)
    const int o = EMIT == EMIT_H ? t / NCE : 0, ao = t % NCE;
    int F = -1;
    TX zold = 0;
    if (t < NOUT) F = EMIT == EMIT_H ? e.children[(size_t)K * NCC + o] : e.children[K];
    const int row = K * NCC + (t >> 6);
    {
        // a lane's share of the row in groups of 32 loads in flight (a row of
        // up to 2048 DoFs is one group); loads at clamped indices,
        // out-of-range products dropped after (a guarded load is a branch
        // with its own wait)
        const int lane = t & 63;
        const double *a = A + (size_t)row * n;
        double acc = 0;
        for (int j0 = lane; j0 < n; j0 += 64 * 32) {
            double av[32], xv[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int j = min(j0 + 64 * u, n - 1);
                av[u] = a[j];
                xv[u] = (double)x[j];
            }
            if (j0 == lane && F >= 0) zold = e.zf[(size_t)F * NCE + ao];
#pragma unroll
            for (int u = 0; u < 32; ++u) acc += j0 + 64 * u < n ? av[u] * xv[u] : 0.0;
        }
        // lanes at or beyond the coarse DoF count never enter the row loop
        // (a coarsest level of fewer than 64 DoFs) but may still own a child
        if (lane >= n && F >= 0) zold = e.zf[(size_t)F * NCE + ao];
        if (t < 2 * N1E * 2) sP[t] = pv;
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) {
            y[row] = (TX)acc;
            sy[t >> 6] = (TX)acc;
        }
    }
    __syncthreads();
    if (F >= 0) {
        const int a0 = ao % N1E, a1 = (ao / N1E) % N1E, a2 = D == 3 ? ao / (N1E * N1E) : 0;
        TX acc = 0;
#pragma unroll
        for (int j = 0; j < NCC; ++j) {
            const int j0 = j & 1, j1 = (j >> 1) & 1, j2 = (j >> 2) & 1;
            TX w = sP[((o & 1) * N1E + a0) * 2 + j0] * sP[(((o >> 1) & 1) * N1E + a1) * 2 + j1];
            if (D == 3) w *= sP[(((o >> 2) & 1) * N1E + a2) * 2 + j2];
            acc += w * sy[j];
        }
        e.zf[(size_t)F * NCE + ao] = zold + acc;
    }
}

template <typename TX>
int launch_coarse_solve_prolong(int d, int n, const double *A, const TX *x, TX *y, const EmitArgs<TX> &e,
                                hipStream_t st) {
    const int ncc = 1 << d;
    if (n <= 0) return 0;
    if (n % ncc != 0 || e.children == nullptr || e.zf == nullptr) return -1;
    const dim3 g(n / ncc), bl(64 * ncc);
    if (d == 2 && e.kind == EMIT_H)
        hipLaunchKernelGGL((coarse_solve_prolong_kernel<2, TX, EMIT_H>), g, bl, 0, st, n, A, x, y, e);
    else if (d == 2 && e.kind == EMIT_P)
        hipLaunchKernelGGL((coarse_solve_prolong_kernel<2, TX, EMIT_P>), g, bl, 0, st, n, A, x, y, e);
    else if (d == 3 && e.kind == EMIT_H)
        hipLaunchKernelGGL((coarse_solve_prolong_kernel<3, TX, EMIT_H>), g, bl, 0, st, n, A, x, y, e);
    else if (d == 3 && e.kind == EMIT_P)
        hipLaunchKernelGGL((coarse_solve_prolong_kernel<3, TX, EMIT_P>), g, bl, 0, st, n, A, x, y, e);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_coarse_solve_prolong<double>(int, int, const double *, const double *, double *,
                                                 const EmitArgs<double> &, hipStream_t);
template int launch_coarse_solve_prolong<float>(int, int, const double *, const float *, float *,
                                                const EmitArgs<float> &, hipStream_t);

// --------------------------------------------------------------------------
// Additive cell-wise correction (Sec. 3.1, the additive subspace correction
// P = sum_i R_i^T A_i^{-1} R_i), one thread per DoF, a cell's residual staged
// in LDS by its threads; cells never straddle a wave (64 / nc cells each).
template <typename T, int NC>
__global__ __launch_bounds__(256) void block_jacobi_kernel(int n_act, const int *__restrict__ bnd_of,
                                                           const T *__restrict__ Bint_t,
                                                           const T *__restrict__ Bbnd_t, const T *__restrict__ r,
                                                           T *__restrict__ d, T *__restrict__ z, T alpha, T beta,
                                                           const int *__restrict__ list) {
    constexpr int CPW = 64 / NC;                 // cells per wave
    __shared__ T rs[4 * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane / NC, i = lane % NC;
    const int kx = (blockIdx.x * 4 + wave) * CPW + c;   // cell, or position in the list
    const bool live = c < CPW && kx < n_act;
    const int K = list != nullptr ? (live ? list[kx] : 0) : kx;
    const int Kc = live ? K : 0;
    T ri = live ? r[(size_t)Kc * NC + i] : T(0);
    const int bo = live ? bnd_of[Kc] : -1;
    rs[threadIdx.x] = ri;
    __syncthreads();
    if (!live) return;
    const T *B = bo < 0 ? Bint_t : Bbnd_t + (size_t)bo * NC * NC;
    const T *rc = rs + wave * 64 + c * NC;
    T acc = 0;
#pragma unroll 8
    for (int j = 0; j < NC; ++j) acc += B[(size_t)j * NC + i] * rc[j];
    const size_t g = (size_t)K * NC + i;
    const T dn = alpha == T(0) ? beta * acc : alpha * d[g] + beta * acc;
    d[g] = dn;
    if (z != nullptr) z[g] += dn;
}

template <typename T>
int launch_block_jacobi(int n_act, int nc, const int *bnd_of, const T *Bint_t, const T *Bbnd_t, const T *r, T *d,
                        T *z, T alpha, T beta, hipStream_t st, const int *list) {
    if (n_act <= 0) return 0;
    const int cpw = 64 / nc;
    const dim3 g((n_act + 4 * cpw - 1) / (4 * cpw)), bl(256);
#define BJ_CASE(NCV)                                                                                               \
    case NCV:                                                                                                      \
        hipLaunchKernelGGL((block_jacobi_kernel<T, NCV>), g, bl, 0, st, n_act, bnd_of, Bint_t, Bbnd_t, r, d, z,   \
                           alpha, beta, list);                                                                     \
        break;
    switch (nc) {
        BJ_CASE(4)
        BJ_CASE(8)
        BJ_CASE(9)
        BJ_CASE(16)
        BJ_CASE(27)
        BJ_CASE(64)
        default:
            return -1;
    }
#undef BJ_CASE
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_block_jacobi<double>(int, int, const int *, const double *, const double *, const double *,
                                         double *, double *, double, double, hipStream_t, const int *);
template int launch_block_jacobi<float>(int, int, const int *, const float *, const float *, const float *, float *,
                                        float *, float, float, hipStream_t, const int *);

// --------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(long long n, T *x, T v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) x[i] = v;
}
template <typename T>
int launch_fill(long long n, T *x, T v, hipStream_t st) {
    if (n <= 0) return 0;
    int nb = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((fill_kernel<T>), dim3(nb), dim3(256), 0, st, n, x, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_fill<double>(long long, double *, double, hipStream_t);
template int launch_fill<float>(long long, float *, float, hipStream_t);

// x[0..n) = y[0..n) = 0 in one launch, 16-byte stores (x and y 16-byte
// aligned; the last n % (16 / sizeof(T)) entries one at a time)
template <typename T>
__global__ void zero2_kernel(long long n, T *__restrict__ x, T *__restrict__ y) {
    constexpr int W = 16 / sizeof(T);
    const long long nv = n / W;
    const long long st = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (long long i = t0; i < nv; i += st) {
        reinterpret_cast<float4 *>(x)[i] = z4;
        if (y != nullptr) reinterpret_cast<float4 *>(y)[i] = z4;
    }
    for (long long i = nv * W + t0; i < n; i += st) {
        x[i] = T(0);
        if (y != nullptr) y[i] = T(0);
    }
}
template <typename T>
int launch_zero2(long long n, T *x, T *y, hipStream_t st) {
    if (n <= 0) return 0;
    if (((uintptr_t)x & 15) != 0 || ((uintptr_t)y & 15) != 0) return -1;
    const long long nv = std::max<long long>(n / (16 / sizeof(T)), 1);
    const int nb = (int)std::min<long long>((nv + 255) / 256, 8192);
    hipLaunchKernelGGL((zero2_kernel<T>), dim3(nb), dim3(256), 0, st, n, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_zero2<double>(long long, double *, double *, hipStream_t);
template int launch_zero2<float>(long long, float *, float *, hipStream_t);

template <typename A, typename B>
__global__ void cast_kernel(long long n, const A *__restrict__ x, B *__restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = (B)x[i];
}
int launch_cast_d2f(long long n, const double *x, float *y, hipStream_t st) {
    if (n <= 0) return 0;
    int nb = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nb), dim3(256), 0, st, n, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_cast_f2d(long long n, const float *x, double *y, hipStream_t st) {
    if (n <= 0) return 0;
    int nb = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nb), dim3(256), 0, st, n, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// --------------------------------------------------------------------------
// FGMRES vector kernels (FP64).
//
// Sums are deterministic: each block of a streaming kernel stores its partial
// sums (plain stores), and the partials are added in one fixed order either
// by the next streaming kernel, in every block (it needs the result to go on),
// or by a small reduction kernel when only the host needs it.
constexpr int GS_BLOCKS = 256;   // one 16-wave block per CU
constexpr int GS_THREADS = 1024;
constexpr int GS_WAVES = GS_THREADS / 64;
constexpr int GS_MAXV = 32;      // sums per launch: up to 31 basis vectors plus one norm

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// partial[blockIdx.x * nv + i] = sum over the block's threads of acc[i], i < nv
// (NW waves per block)
template <int NW>
__device__ __forceinline__ void block_partials(const double (&acc)[GS_MAXV], int nv, double *partial) {
    __shared__ double red[NW][GS_MAXV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < GS_MAXV; ++i) {
        if (i < nv) {
            double v = wave_sum(acc[i]);
            if (lane == 0) red[wave][i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        const int i = threadIdx.x;
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) v += red[w][i];
        partial[(size_t)blockIdx.x * nv + i] = v;
    }
}

// dst[i] = sum_b partial[b * nv + i] over nblk <= GS_BLOCKS blocks, i < nv, in
// one fixed order whatever the block size (lane l adds blocks l, l + 64, ...;
// then a butterfly over the lanes; wave w of NW takes sums w, w + NW, ...).
// dst may be LDS or global memory; the caller synchronises before reading it.
template <int NW>
__device__ __forceinline__ void sum_partials(const double *__restrict__ partial, int nblk, int nv, double *dst) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int PER_LANE = GS_BLOCKS / 64, PER_WAVE = GS_MAXV / NW;
    double t[PER_WAVE][PER_LANE];
#pragma unroll
    for (int r = 0; r < PER_WAVE; ++r) {
        const int i = wave + NW * r;
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const int b = lane + 64 * u;
            // (loaded at a clamped index and weighted by 0 or 1: a guarded
            // load, or a select the compiler turns into one, is a branch with
            // its own wait; the clamped duplicates are finite partial sums)
            const double pv = partial[(size_t)min(b, nblk - 1) * nv + min(i, nv - 1)];
            t[r][u] = pv * (i < nv && b < nblk ? 1.0 : 0.0);
        }
    }
    // all sums before the first store (a store between the groups of loads
    // kept the compiler from issuing them together)
    double v[PER_WAVE];
#pragma unroll
    for (int r = 0; r < PER_WAVE; ++r) {
        v[r] = 0.0;
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) v[r] += t[r][u];
        v[r] = wave_sum(v[r]);
    }
#pragma unroll
    for (int r = 0; r < PER_WAVE; ++r) {
        const int i = wave + NW * r;
        if (lane == 0 && i < nv) dst[i] = v[r];
    }
}

static int gs_grid(long long n) {
    return (int)std::max<long long>(1, std::min<long long>((n + GS_THREADS - 1) / GS_THREADS, GS_BLOCKS));
}

// The streaming kernels are instantiated for a bound MB >= m on the number of
// basis vectors.  Rows i >= m read row m - 1 instead (a valid address, already
// in cache) with a zero weight or an unused sum, so every load of an element
// step is unconditional and all of them are in flight together.
static int gs_bucket(int m) { return m == 0 ? 0 : m <= 4 ? 4 : m <= 8 ? 8 : m <= 16 ? 16 : 32; }

// partials of V_i . w (i < m) and of w . w (slot m)
template <int MB>
__global__ __launch_bounds__(GS_THREADS) void gs_dots_kernel(long long n, int m, const double *__restrict__ V,
                                                             const double *__restrict__ w, double *__restrict__ part) {
    double acc[GS_MAXV];
#pragma unroll
    for (int i = 0; i < GS_MAXV; ++i) acc[i] = 0.0;
    double ww = 0.0;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        const double wk = w[k];
#pragma unroll
        for (int i = 0; i < MB; ++i) acc[i] += V[(size_t)(i < m ? i : m - 1) * n + k] * wk;
        ww += wk * wk;
    }
#pragma unroll
    for (int i = 0; i < GS_MAXV; ++i)
        if (i == m) acc[i] = ww;
    block_partials<GS_WAVES>(acc, m + 1, part);
}

// h = sums of the nblk_in x (m + 1) partials hpart (block 0 also stores all
// m + 1 of them in hout); w <- w - sum_i h[i] V_i; partials of V_i . w (i < m)
// and of w . w (slot m)
template <int MB>
__global__ __launch_bounds__(GS_THREADS) void gs_axpy_dots_kernel(long long n, int m, const double *__restrict__ V,
                                                                  const double *__restrict__ hpart, int nblk_in,
                                                                  double *__restrict__ hout, double *__restrict__ w,
                                                                  double *__restrict__ part) {
    __shared__ double hs[GS_MAXV];
    sum_partials<GS_WAVES>(hpart, nblk_in, m + 1, hs);
    __syncthreads();
    if (blockIdx.x == 0 && (int)threadIdx.x <= m) hout[threadIdx.x] = hs[threadIdx.x];
    // (instantiated up to 16 vectors: weights and loaded elements stay in registers)
    static_assert(MB <= 16, "larger bases use gs_axpy_kernel + gs_dots_kernel");
    double hh[MB > 0 ? MB : 1], acc[GS_MAXV];
#pragma unroll
    for (int i = 0; i < MB; ++i) hh[i] = i < m ? hs[i] : 0.0;
#pragma unroll
    for (int i = 0; i < GS_MAXV; ++i) acc[i] = 0.0;
    double ww = 0.0;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        double vk[MB > 0 ? MB : 1];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            vk[i] = V[(size_t)(i < m ? i : m - 1) * n + k];
            s += hh[i] * vk[i];
        }
        const double wk = w[k] - s;
        w[k] = wk;
#pragma unroll
        for (int i = 0; i < MB; ++i) acc[i] += vk[i] * wk;
        ww += wk * wk;
    }
#pragma unroll
    for (int i = 0; i < GS_MAXV; ++i)
        if (i == m) acc[i] = ww;
    block_partials<GS_WAVES>(acc, m + 1, part);
}

// h = sums of the partials hpart (block 0 stores them in hout); w <- w - V h.
// The subtraction of larger bases (17..31 vectors), whose dots then follow in
// gs_dots_kernel: two streaming launches instead of one that would spill.
template <int MB>
__global__ __launch_bounds__(GS_THREADS) void gs_axpy_kernel(long long n, int m, const double *__restrict__ V,
                                                             const double *__restrict__ hpart, int nblk_in,
                                                             double *__restrict__ hout, double *__restrict__ w) {
    __shared__ double hs[GS_MAXV];
    sum_partials<GS_WAVES>(hpart, nblk_in, m + 1, hs);
    __syncthreads();
    if (blockIdx.x == 0 && (int)threadIdx.x <= m) hout[threadIdx.x] = hs[threadIdx.x];
    double hh[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) hh[i] = i < m ? hs[i] : 0.0;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) s += hh[i] * V[(size_t)(i < m ? i : m - 1) * n + k];
        w[k] -= s;
    }
}

__global__ __launch_bounds__(GS_THREADS) void gs_reduce_kernel(const double *__restrict__ part, int nblk, int nv,
                                                               double *__restrict__ out) {
    sum_partials<GS_WAVES>(part, nblk, nv, out);
}

int launch_gs_dots(long long n, int m, const double *V, const double *w, double *part, hipStream_t st) {
    if (m < 0 || m > GS_MAXV - 1 || n < 0) return -1;
    const dim3 g(gs_grid(n)), bl(GS_THREADS);
    switch (gs_bucket(m)) {
        case 0: hipLaunchKernelGGL(gs_dots_kernel<0>, g, bl, 0, st, n, m, V, w, part); break;
        case 4: hipLaunchKernelGGL(gs_dots_kernel<4>, g, bl, 0, st, n, m, V, w, part); break;
        case 8: hipLaunchKernelGGL(gs_dots_kernel<8>, g, bl, 0, st, n, m, V, w, part); break;
        case 16: hipLaunchKernelGGL(gs_dots_kernel<16>, g, bl, 0, st, n, m, V, w, part); break;
        default: hipLaunchKernelGGL(gs_dots_kernel<32>, g, bl, 0, st, n, m, V, w, part);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gs_axpy_dots(long long n, int m, const double *V, const double *hpart, double *hout, double *w,
                        double *part, hipStream_t st) {
    if (m < 1 || m > GS_MAXV - 1 || n < 0) return -1;
    const int nb = gs_grid(n);
    const dim3 g(nb), bl(GS_THREADS);
    switch (gs_bucket(m)) {
        case 4: hipLaunchKernelGGL(gs_axpy_dots_kernel<4>, g, bl, 0, st, n, m, V, hpart, nb, hout, w, part); break;
        case 8: hipLaunchKernelGGL(gs_axpy_dots_kernel<8>, g, bl, 0, st, n, m, V, hpart, nb, hout, w, part); break;
        case 16: hipLaunchKernelGGL(gs_axpy_dots_kernel<16>, g, bl, 0, st, n, m, V, hpart, nb, hout, w, part); break;
        default:
            hipLaunchKernelGGL(gs_axpy_kernel<32>, g, bl, 0, st, n, m, V, hpart, nb, hout, w);
            hipLaunchKernelGGL(gs_dots_kernel<32>, g, bl, 0, st, n, m, V, w, part);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gs_reduce(long long n, int nv, const double *part, double *out, hipStream_t st) {
    if (nv < 1 || nv > GS_MAXV) return -1;
    hipLaunchKernelGGL(gs_reduce_kernel, dim3(1), dim3(GS_THREADS), 0, st, part, gs_grid(n), nv, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// v = (w - sum_i h[i] V_i) * inv
template <int MB>
__global__ __launch_bounds__(256) void gs_axpy_scale_kernel(long long n, int m, const double *__restrict__ V,
                                                            const double *__restrict__ h, double inv,
                                                            const double *__restrict__ w, double *__restrict__ v) {
    double hh[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const double hv = h[i < m ? i : m - 1];   // (clamped, not guarded)
        hh[i] = i < m ? hv : 0.0;
    }
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        // all loads of the element first (left to itself the compiler issues
        // the 32-vector case one load at a time)
        double vk[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) vk[i] = V[(size_t)(i < m ? i : m - 1) * n + k];
        const double wk = w[k];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) s += hh[i] * vk[i];
        v[k] = (wk - s) * inv;
    }
}
int launch_gs_axpy_scale(long long n, int m, const double *V, const double *h, double inv, const double *w, double *v,
                         hipStream_t st) {
    if (m < 1 || m > GS_MAXV - 1) return -1;
    if (n <= 0) return 0;
    const dim3 g((unsigned)std::min<long long>((n + 255) / 256, 8192)), bl(256);
    switch (gs_bucket(m)) {
        case 4: hipLaunchKernelGGL(gs_axpy_scale_kernel<4>, g, bl, 0, st, n, m, V, h, inv, w, v); break;
        case 8: hipLaunchKernelGGL(gs_axpy_scale_kernel<8>, g, bl, 0, st, n, m, V, h, inv, w, v); break;
        case 16: hipLaunchKernelGGL(gs_axpy_scale_kernel<16>, g, bl, 0, st, n, m, V, h, inv, w, v); break;
        default: hipLaunchKernelGGL(gs_axpy_scale_kernel<32>, g, bl, 0, st, n, m, V, h, inv, w, v);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// w += sign * sum_i h[i] V_i
// (instantiated for a bound MB >= m like the Gram-Schmidt kernels, all loads
// of an element issued before the products)
template <int MB>
__global__ __launch_bounds__(256) void multiaxpy_kernel(long long n, int m, double sign, const double *__restrict__ h,
                                                        const double *__restrict__ V, double *__restrict__ w) {
    double hh[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const double hv = h[i < m ? i : m - 1];   // (clamped, not guarded)
        hh[i] = i < m ? hv : 0.0;
    }
    long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        double vk[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) vk[i] = V[(size_t)(i < m ? i : m - 1) * n + k];
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) acc += hh[i] * vk[i];
        w[k] += sign * acc;
    }
}
int launch_multiaxpy(long long n, int m, double sign, const double *h, const double *V, double *w, hipStream_t st) {
    if (n <= 0 || m <= 0) return 0;
    if (m > GS_MAXV) return -1;
    const dim3 g((unsigned)std::min<long long>((n + 255) / 256, 8192)), bl(256);
    switch (gs_bucket(m)) {
        case 4: hipLaunchKernelGGL(multiaxpy_kernel<4>, g, bl, 0, st, n, m, sign, h, V, w); break;
        case 8: hipLaunchKernelGGL(multiaxpy_kernel<8>, g, bl, 0, st, n, m, sign, h, V, w); break;
        case 16: hipLaunchKernelGGL(multiaxpy_kernel<16>, g, bl, 0, st, n, m, sign, h, V, w); break;
        default: hipLaunchKernelGGL(multiaxpy_kernel<32>, g, bl, 0, st, n, m, sign, h, V, w);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// v = w / sqrt(nrm2[0]) (v = w if the norm is zero)
__global__ __launch_bounds__(256) void scale_kernel(long long n, const double *__restrict__ nrm2,
                                                    const double *__restrict__ w, double *__restrict__ v) {
    double s = nrm2[0];
    double inv = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) v[k] = w[k] * inv;
}
int launch_scale(long long n, const double *nrm2, const double *w, double *v, hipStream_t st) {
    if (n <= 0) return 0;
    int nb = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, st, n, nrm2, w, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sbm
