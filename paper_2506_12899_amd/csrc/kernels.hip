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
// block barriers), 4 waves per block; cell data staged in LDS.  The
// block index is remapped so that each of the 8 XCDs works on a contiguous
// range of cells (neighbour traces then hit that XCD's L2).
#include "kernels.hpp"

namespace sbm {

template <int D, int P>
struct Sh {
    static constexpr int N1 = P + 1;
    static constexpr int NC = D == 2 ? N1 * N1 : N1 * N1 * N1;
    static constexpr int NF = D == 2 ? N1 : N1 * N1;
    static constexpr int CPW = 64 / NC;
    static constexpr int WAVES = 4;
    static constexpr int CPB = CPW * WAVES;
    static constexpr int NFACE = 2 * D;
};

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    // blocks are dispatched round-robin over the 8 XCDs; give XCD x a contiguous range
    int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The threads of one cell always sit in one wave, so data exchanged through
// LDS between them needs no block barrier: LDS instructions of a wave complete
// in order, and this only keeps the compiler from moving memory operations
// across the exchange point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

template <typename T>
__device__ __forceinline__ void lagrange_dev(const T *nodes, int n1, T x, T *v) {
    for (int a = 0; a < n1; ++a) {
        T num = 1, den = 1;
        for (int b = 0; b < n1; ++b) {
            if (b == a) continue;
            num *= x - nodes[b];
            den *= nodes[a] - nodes[b];
        }
        v[a] = num / den;
    }
}

// --------------------------------------------------------------------------
// Cell operator kernel.
//  OP_APPLY : out = A x
//  OP_RESID : out = b - A x
//  OP_SMOOTH: x (= out, in place) += omega * B_K (b - A x)_K on cells [cell0, cell0+ncells)
template <int D, int P, typename T, int OP>
__global__ __launch_bounds__(256) void cellop_kernel(int cell0, int ncells, const T *xin, T *out,
                                                    const T *__restrict__ b, CellArgs<T> a, KRef<T> R) {
    using S = Sh<D, P>;
    constexpr int N1 = S::N1, NC = S::NC, NF = S::NF, CPB = S::CPB, NFACE = S::NFACE;
    __shared__ T su[CPB][NC];
    __shared__ T sa[CPB][NC];
    __shared__ T sb[CPB][NC];
    __shared__ T fa[CPB][NFACE][NF];
    __shared__ T fb[CPB][NFACE][NF];
    __shared__ T ga[CPB][NFACE][NF];
    __shared__ T gb[CPB][NFACE][NF];
    __shared__ int snb[CPB][NFACE];
    __shared__ T sB[OP == OP_SMOOTH ? NC * NC : 1];  // shared interior-cell inverse

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool slot = lane < S::CPW * NC;
    const int lc = slot ? wave * S::CPW + lane / NC : 0;
    const int i = slot ? lane % NC : 0;
    if (OP == OP_SMOOTH) {
        for (int t = threadIdx.x; t < NC * NC; t += blockDim.x) sB[t] = a.Bint_t[t];
        __syncthreads();
    }
    // Each block owns a contiguous chunk of cell batches (one batch per block
    // for the apply, several for the smoother so that sB is staged once per
    // chunk); the remap gives every XCD a contiguous range of cells.
    const int nbatch = a.batch_start != nullptr ? a.nbatch : (ncells + CPB - 1) / CPB;
    const int chunk = OP == OP_SMOOTH ? (nbatch + gridDim.x - 1) / gridDim.x : 1;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int bb0 = blk * chunk;
    const int bb1 = OP == OP_SMOOTH ? min(nbatch, bb0 + chunk) : bb0 + 1;
#pragma unroll 1
    for (int bb = bb0; bb < bb1; ++bb) {
        int bstart, bend;
        if (a.batch_start != nullptr) {
            bstart = a.batch_start[bb];
            bend = min(bstart + CPB, bstart < a.split ? a.split : cell0 + ncells);
        } else {
            bstart = cell0 + bb * CPB;
            bend = cell0 + ncells;
        }
        const int cell = bstart + lc;
        const bool live = slot && cell < bend;
        wave_sync();  // the previous batch is done with this wave's LDS slices

        if (live) {
            su[lc][i] = xin[(size_t)cell * NC + i];
            if (i < NFACE) snb[lc][i] = a.nbr[(size_t)cell * NFACE + i];
        }
        wave_sync();

        // neighbour data for the face couplings: the loads are issued here and
        // consumed after the volume stage, so their latency overlaps it
        constexpr int ITEMS = (NFACE * NF + NC - 1) / NC;
        T raw[ITEMS][N1];
        if (live) {
#pragma unroll
            for (int q = 0; q < ITEMS; ++q) {
                int it = i + q * NC;
                if (it < NFACE * NF) {
                    int f = it / NF, j = it % NF, k = f >> 1;
                    int nb = snb[lc][f];
                    if (nb >= 0) {
                        const T *un = xin + (size_t)nb * NC;
#pragma unroll
                        for (int m = 0; m < N1; ++m) raw[q][m] = un[compose<D, P>(k, m, j)];
                    }
                }
            }
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
                int it = i + q * NC;
                if (it >= NFACE * NF) break;
                int f = it / NF, j = it % NF, s = f & 1;
                int nb = snb[lc][f];
                T va = 0, vb = 0;
                if (nb >= 0) {
                    const T *gN = R.g[s == 1 ? 0 : 1];
                    T t = s == 1 ? raw[q][0] : raw[q][P];
                    T dn = 0;
#pragma unroll
                    for (int m = 0; m < N1; ++m) dn += gN[m] * raw[q][m];
                    T sg = s == 1 ? T(1) : T(-1);
                    va = T(-0.5) * sg * dn - R.sigF * t;
                    vb = T(0.5) * t;
                }
                fa[lc][f][j] = va;
                fb[lc][f][j] = vb;
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
            for (int it = i; it < NFACE * NF; it += NC) {
                int f = it / NF, q = it % NF, k = f >> 1, s = f & 1;
                int nb = snb[lc][f];
                T zeta = 0;
                if (nb < 0) {
                    int rec = -nb - 1;
                    const T *dq = a.shift + ((size_t)rec * NF + q) * D;
                    int q1 = q % N1, q2 = D == 3 ? q / N1 : 0;
                    T wq = R.w[q1] * (D == 3 ? R.w[q2] : T(1));
                    const int layer = s ? P : 0;
                    T E = 0;
                    // boundary cells only: loops stay rolled to keep register pressure
                    // of the whole kernel low
                    if (R.ext == 0) {
                        // gradient of u at the face Gauss point
                        T dk = 0, dt1 = 0, dt2 = 0;
#pragma unroll 1
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
                        E = dq[k] * dk + dq[t1] * dt1;
                        if (D == 3) E += dq[t2] * dt2;
                    } else {
                        // cell polynomial at the shifted point minus its value at the face point
                        T lv[3][N1];
                        const int t1 = k == 0 ? 1 : 0;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            T xc = c == k ? T(s) : (c == t1 ? R.gq[q1] : R.gq[q2]);
                            lagrange_dev<T>(R.x, N1, xc + dq[c], lv[c]);
                        }
                        T acc = 0, face = 0;
#pragma unroll 1
                        for (int jj = 0; jj < NC; ++jj) {
                            int a0 = jj % N1, a1 = (jj / N1) % N1, a2 = D == 3 ? jj / (N1 * N1) : 0;
                            T pv = lv[0][a0] * lv[1][a1];
                            if (D == 3) pv *= lv[2][a2];
                            acc += pv * su[lc][jj];
                        }
#pragma unroll 1
                        for (int j = 0; j < NF; ++j) {
                            int j1 = j % N1, j2 = D == 3 ? j / N1 : 0;
                            T sv = R.S[q1][j1] * (D == 3 ? R.S[q2][j2] : T(1));
                            face += sv * su[lc][compose<D, P>(k, layer, j)];
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
#pragma unroll 1
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
            if (live) out[(size_t)cell * NC + i] = b[(size_t)cell * NC + i] - y;
        } else {
            wave_sync();
            if (live) sa[lc][i] = b[(size_t)cell * NC + i] - y;
            wave_sync();
            if (live) {
                int bi = a.bnd_of[cell];
                T corr = 0;
                if (bi < 0) {
#pragma unroll 4
                    for (int j = 0; j < NC; ++j) corr += sB[j * NC + i] * sa[lc][j];
                } else {
                    const T *Bt = a.Bbnd_t + (size_t)bi * NC * NC;
#pragma unroll 2
                    for (int j = 0; j < NC; ++j) corr += Bt[(size_t)j * NC + i] * sa[lc][j];
                }
                if (a.lw != nullptr && bi >= 0) {
                    const T *U = a.lU + (size_t)bi * NC * 4;
                    const T *V = a.lV + (size_t)bi * NC * 4;
                    T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
#pragma unroll 1
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
                out[(size_t)cell * NC + i] = su[lc][i] + R.omega * corr;
            }
        }
    }  // batch loop
}

template <int D, int P, typename T>
static int launch_dp(int op, int cell0, int ncells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                     const KRef<T> &R, hipStream_t st) {
    if (ncells <= 0) return 0;
    using S = Sh<D, P>;
    int nb = a.batch_start != nullptr ? a.nbatch : (ncells + S::CPB - 1) / S::CPB;
    if (op == OP_SMOOTH) nb = std::min(nb, 2048);
    if (op == OP_APPLY)
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_APPLY>), dim3(nb), dim3(256), 0, st, cell0, ncells, x, y, b, a, R);
    else if (op == OP_RESID)
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_RESID>), dim3(nb), dim3(256), 0, st, cell0, ncells, x, y, b, a, R);
    else
        hipLaunchKernelGGL((cellop_kernel<D, P, T, OP_SMOOTH>), dim3(nb), dim3(256), 0, st, cell0, ncells, x, y, b, a, R);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_cellop(int d, int p, int op, int cell0, int ncells, const T *x, T *y, const T *b, const CellArgs<T> &a,
                  const KRef<T> &R, hipStream_t st) {
    if (d == 2) {
        if (p == 1) return launch_dp<2, 1, T>(op, cell0, ncells, x, y, b, a, R, st);
        if (p == 2) return launch_dp<2, 2, T>(op, cell0, ncells, x, y, b, a, R, st);
        if (p == 3) return launch_dp<2, 3, T>(op, cell0, ncells, x, y, b, a, R, st);
    } else {
        if (p == 1) return launch_dp<3, 1, T>(op, cell0, ncells, x, y, b, a, R, st);
        if (p == 2) return launch_dp<3, 2, T>(op, cell0, ncells, x, y, b, a, R, st);
        if (p == 3) return launch_dp<3, 3, T>(op, cell0, ncells, x, y, b, a, R, st);
    }
    return -1;
}
template int launch_cellop<double>(int, int, int, int, int, const double *, double *, const double *,
                                   const CellArgs<double> &, const KRef<double> &, hipStream_t);
template int launch_cellop<float>(int, int, int, int, int, const float *, float *, const float *,
                                  const CellArgs<float> &, const KRef<float> &, hipStream_t);

// --------------------------------------------------------------------------
// Transfers (Sec. 3.2): prolongation = embedding of the coarse cell polynomial
// into the fine cell(s), restriction = its transpose; inactive parents give
// zero and restriction into inactive coarse cells is dropped.
template <int D, typename T>
__global__ __launch_bounds__(256) void prolong_kernel(int n_fine, int n1f, int n1c, const int *__restrict__ parent,
                                                      const int *__restrict__ childpos, const T *__restrict__ zc,
                                                      T *__restrict__ zf, TransferArgs<T> tr) {
    int ncf = D == 2 ? n1f * n1f : n1f * n1f * n1f;
    int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)n_fine * ncf) return;
    int K = (int)(gid / ncf), i = (int)(gid % ncf);
    int pc = parent[K];
    if (pc < 0) return;
    int o = childpos[K];
    int i0 = i % n1f, i1 = (i / n1f) % n1f, i2 = D == 3 ? i / (n1f * n1f) : 0;
    const T *P0 = tr.P1[o & 1][i0];
    const T *P1 = tr.P1[(o >> 1) & 1][i1];
    const T *P2 = tr.P1[(o >> 2) & 1][i2];
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

template <int D, typename T>
__global__ __launch_bounds__(256) void restrict_kernel(int n_coarse, int n1f, int n1c, int nch,
                                                       const int *__restrict__ children, const T *__restrict__ rf,
                                                       T *__restrict__ bc, TransferArgs<T> tr) {
    int ncf = D == 2 ? n1f * n1f : n1f * n1f * n1f;
    int ncc = D == 2 ? n1c * n1c : n1c * n1c * n1c;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)n_coarse * ncc) return;
    int Kc = (int)(gid / ncc), j = (int)(gid % ncc);
    int j0 = j % n1c, j1 = (j / n1c) % n1c, j2 = D == 3 ? j / (n1c * n1c) : 0;
    T acc = 0;
    for (int o = 0; o < nch; ++o) {
        int K = children[(size_t)Kc * nch + o];
        if (K < 0) continue;
        const T *src = rf + (size_t)K * ncf;
        for (int i = 0; i < ncf; ++i) {
            int i0 = i % n1f, i1 = (i / n1f) % n1f, i2 = D == 3 ? i / (n1f * n1f) : 0;
            T w = tr.P1[o & 1][i0][j0] * tr.P1[(o >> 1) & 1][i1][j1];
            if (D == 3) w *= tr.P1[(o >> 2) & 1][i2][j2];
            acc += w * src[i];
        }
    }
    bc[(size_t)Kc * ncc + j] = acc;
}

template <typename T>
int launch_prolong(int d, int n_fine, int n1f, int n1c, const int *parent, const int *childpos, const T *zc, T *zf,
                   const TransferArgs<T> &tr, hipStream_t st) {
    long long n = (long long)n_fine * (d == 2 ? n1f * n1f : n1f * n1f * n1f);
    if (n <= 0) return 0;
    int nb = (int)((n + 255) / 256);
    if (d == 2)
        hipLaunchKernelGGL((prolong_kernel<2, T>), dim3(nb), dim3(256), 0, st, n_fine, n1f, n1c, parent, childpos, zc, zf, tr);
    else
        hipLaunchKernelGGL((prolong_kernel<3, T>), dim3(nb), dim3(256), 0, st, n_fine, n1f, n1c, parent, childpos, zc, zf, tr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_restrict(int d, int n_coarse, int n1f, int n1c, int nch, const int *children, const T *rf, T *bc,
                    const TransferArgs<T> &tr, hipStream_t st) {
    long long n = (long long)n_coarse * (d == 2 ? n1c * n1c : n1c * n1c * n1c);
    if (n <= 0) return 0;
    int nb = (int)((n + 255) / 256);
    if (d == 2)
        hipLaunchKernelGGL((restrict_kernel<2, T>), dim3(nb), dim3(256), 0, st, n_coarse, n1f, n1c, nch, children, rf, bc, tr);
    else
        hipLaunchKernelGGL((restrict_kernel<3, T>), dim3(nb), dim3(256), 0, st, n_coarse, n1f, n1c, nch, children, rf, bc, tr);
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
// Coarsest level: z = A0^{-1} b with the dense inverse (one row per thread).
template <typename T>
__global__ __launch_bounds__(256) void dense_gemv_kernel(int n, const T *__restrict__ A, const T *__restrict__ x,
                                                         T *__restrict__ y) {
    // one wave per row: the lanes stride over the row (coalesced), then reduce
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= n) return;
    const T *a = A + (size_t)row * n;
    T acc = 0;
    for (int j = lane; j < n; j += 64) acc += a[j] * x[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = acc;
}

template <typename T>
int launch_dense_gemv(int n, const T *A, const T *x, T *y, hipStream_t st) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL((dense_gemv_kernel<T>), dim3((n + 3) / 4), dim3(256), 0, st, n, A, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_dense_gemv<double>(int, const double *, const double *, double *, hipStream_t);
template int launch_dense_gemv<float>(int, const float *, const float *, float *, hipStream_t);

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
// FGMRES vector kernels (FP64).  Deterministic: fixed grid, per-block partial
// sums, one reducing block.
constexpr int RED_BLOCKS = 1024;

// partial[blk * m + i] = sum over the block's slice of V_i . w   (V_i = V + i * n)
__global__ __launch_bounds__(256) void multidot_kernel(long long n, int m, const double *__restrict__ V,
                                                       const double *__restrict__ w, double *__restrict__ partial) {
    __shared__ double red[4][32];
    double acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0.0;
    long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        double wk = w[k];
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < m) acc[i] += V[(size_t)i * n + k] * wk;
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        if (i >= m) break;
        double v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < m)
        partial[(size_t)blockIdx.x * m + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// out[i] = sum_blk partial[blk * m + i]  (one block, fixed order)
__global__ __launch_bounds__(256) void reduce_partials_kernel(int nblk, int m, const double *__restrict__ partial,
                                                              double *__restrict__ out) {
    __shared__ double red[256];
    for (int i = 0; i < m; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)b * m + i];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[i] = red[0];
        __syncthreads();
    }
}

int launch_multidot(long long n, int m, const double *V, const double *w, double *partial, double *out,
                    hipStream_t st) {
    if (m <= 0 || m > 32) return -1;
    long long want = (n + 255) / 256;
    int nb = (int)std::max<long long>(1, std::min<long long>(want, RED_BLOCKS));
    hipLaunchKernelGGL(multidot_kernel, dim3(nb), dim3(256), 0, st, n, m, V, w, partial);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, nb, m, partial, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// w += sign * sum_i h[i] V_i
__global__ __launch_bounds__(256) void multiaxpy_kernel(long long n, int m, double sign, const double *__restrict__ h,
                                                        const double *__restrict__ V, double *__restrict__ w) {
    long long st = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += st) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += h[i] * V[(size_t)i * n + k];
        w[k] += sign * acc;
    }
}
int launch_multiaxpy(long long n, int m, double sign, const double *h, const double *V, double *w, hipStream_t st) {
    if (n <= 0 || m <= 0) return 0;
    int nb = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(nb), dim3(256), 0, st, n, m, sign, h, V, w);
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
