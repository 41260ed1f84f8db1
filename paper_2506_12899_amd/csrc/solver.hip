// C ABI, device upload, V-cycle and FGMRES orchestration.
//
// V-cycle (paper Sec. 3: one V-cycle as the preconditioner; Sec. 3.1 smoother,
// Sec. 3.2 transfers): on level l > 0, z = 0; nu_pre SSOR steps; r = b - A z;
// restrict; recurse; prolongate and add; nu_post SSOR steps.  One SSOR step
// visits the colours (0, 1, 1, 0); each colour is one kernel launch because
// cells of one colour do not couple.  Level 0 applies the dense inverse.
//
// FGMRES(m) (Sec. 3 opening, GMRES with the V-cycle preconditioner): right
// preconditioning, x0 = 0, classical Gram-Schmidt with a selective second
// pass (taken only when the first one cancels, |w'| < 0.1 |w|: the
// Daniel-Gragg-Kaufman-Stewart test) in FP64 on the device, Givens rotations on the
// host (one small device-to-host copy per iteration), stop on the true
// relative residual.
#include <algorithm>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "setup.hpp"

using namespace sbm;

namespace {

#define HIPCHK(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) {                                        \
            pb->last_error = std::string(#call) + ": " + hipGetErrorString(e_); \
            return SBM_EDEVICE;                                        \
        }                                                              \
    } while (0)

#define KCHK(call)                                                     \
    do {                                                               \
        if ((call) != 0) {                                             \
            pb->last_error = std::string("launch failed: ") + #call;   \
            return SBM_EDEVICE;                                        \
        }                                                              \
    } while (0)

template <typename T>
int dalloc(sbm_problem *pb, T **p, size_t n) {
    *p = nullptr;
    if (n == 0) return SBM_OK;
    void *q = nullptr;
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
        pb->last_error = "hipMalloc failed";
        return SBM_ENOMEM;
    }
    pb->allocations.push_back(q);
    *p = (T *)q;
    return SBM_OK;
}

template <typename T, typename S>
int upload(sbm_problem *pb, T **p, const S *src, size_t n) {
    int rc = dalloc(pb, p, n);
    if (rc || n == 0) return rc;
    std::vector<T> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (T)src[i];
    HIPCHK(hipMemcpy(*p, tmp.data(), n * sizeof(T), hipMemcpyHostToDevice));
    return SBM_OK;
}

template <typename T>
void cast_kref(const KRef<double> &a, KRef<T> &b) {
    std::memset(&b, 0, sizeof(b));
    for (int i = 0; i < MAXN1; ++i) {
        for (int j = 0; j < MAXN1; ++j) {
            b.M[i][j] = (T)a.M[i][j];
            b.S[i][j] = (T)a.S[i][j];
            b.Sd[i][j] = (T)a.Sd[i][j];
            for (int v = 0; v < 4; ++v) b.Tv[v][i][j] = (T)a.Tv[v][i][j];
        }
        b.w[i] = (T)a.w[i];
        b.gq[i] = (T)a.gq[i];
        b.g[0][i] = (T)a.g[0][i];
        b.g[1][i] = (T)a.g[1][i];
        b.x[i] = (T)a.x[i];
        b.bw[i] = (T)a.bw[i];
    }
    b.sigF = (T)a.sigF;
    b.sigG = (T)a.sigG;
    b.alpha = (T)a.alpha;
    b.scale = (T)a.scale;
    b.omega = (T)a.omega;
    b.ext = a.ext;
}

// The cells of level l whose inverse the stabilisation changed, by colour
// (buffers sized n_bnd, allocated once; set_shifts refills them)
template <typename T>
int clip_lists(sbm_problem *pb, int l, DevLevel<T> &D, bool alloc) {
    const HostLevel &L = pb->levels[l];
    int rc;
    if (alloc) {
        if ((rc = dalloc(pb, &D.hold, L.n_bnd)) || (rc = dalloc(pb, &D.rep1, L.n_bnd)) ||
            (rc = dalloc(pb, &D.clip0, L.n_bnd)) || (rc = dalloc(pb, &D.clip0_cbnd, L.n_bnd)))
            return rc;
    }
    std::vector<int> hold(L.n_bnd, 0), rep1, clip0, cbnd;
    const bool ptransfer = l > 0 && L.ratio == 1;
    for (int K = 0; K < L.n_act; ++K) {
        const int bi = L.bnd_of[K];
        if (bi < 0 || (size_t)bi >= L.clipped.size() || !L.clipped[bi]) continue;
        hold[bi] = 1;
        if (K >= L.n_col0) {
            rep1.push_back(K);
        } else {
            clip0.push_back(K);
            cbnd.push_back(ptransfer ? pb->levels[l - 1].bnd_of[K] : -1);
        }
    }
    D.n_rep1 = (int)rep1.size();
    D.n_clip0 = (int)clip0.size();
    if (L.n_bnd > 0) HIPCHK(hipMemcpy(D.hold, hold.data(), hold.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!rep1.empty()) HIPCHK(hipMemcpy(D.rep1, rep1.data(), rep1.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!clip0.empty()) {
        HIPCHK(hipMemcpy(D.clip0, clip0.data(), clip0.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.clip0_cbnd, cbnd.data(), cbnd.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    return SBM_OK;
}

template <typename T>
int upload_level(sbm_problem *pb, int l, DevLevel<T> &D) {
    const HostLevel &L = pb->levels[l];
    D.d = L.d;
    D.p = L.p;
    D.nc = L.nc;
    D.nf = L.nf;
    D.n_act = L.n_act;
    D.n_col0 = L.n_col0;
    D.n_bnd = L.n_bnd;
    D.n_surr = L.n_surr;
    int rc;
    if ((rc = upload(pb, &D.nbr, L.nbr.data(), L.nbr.size()))) return rc;
    if ((rc = upload(pb, &D.bnd_of, L.bnd_of.data(), L.bnd_of.size()))) return rc;
    if ((rc = upload(pb, &D.bnd_cells, L.bnd_cells.data(), L.bnd_cells.size()))) return rc;
    if ((rc = clip_lists(pb, l, D, true))) return rc;
    if (pb->opt.pencil && pencil_supported(L.d, L.p)) {
        std::vector<int> col, all, bl;
        for (int c = 0; c < 2; ++c) {
            const int k0 = c == 0 ? 0 : L.n_col0, k1 = c == 0 ? L.n_col0 : L.n_act;
            for (int K = k0; K < k1; ++K) (L.bnd_of[K] < 0 ? col : bl).push_back(K);
            if (c == 0) {
                D.n_int0 = (int)col.size();
                D.n_bl0 = (int)bl.size();
            }
        }
        D.n_int1 = (int)col.size() - D.n_int0;
        D.n_bl1 = (int)bl.size() - D.n_bl0;
        // mesh order in tiles of 8^d cells for whole-level operations (a cell's
        // neighbours, of the other colour, are then near it in the launch, and
        // the cells an XCD has in flight with their neighbours fit its L2),
        // the same tile order inside each colour
        auto key = [&](int K) {
            constexpr int TB = 8;
            const int nt = (L.n + TB - 1) / TB;
            long long tile = 0, in = 0;
            for (int c = L.d - 1; c >= 0; --c) {
                const int v = L.cells[(size_t)K * L.d + c];
                tile = tile * nt + v / TB;
                in = in * TB + v % TB;
            }
            long long cells_per_tile = 1;
            for (int c = 0; c < L.d; ++c) cells_per_tile *= TB;
            return tile * cells_per_tile + in;
        };
        auto by_key = [&](int x, int y) { return key(x) < key(y); };
        std::sort(col.begin(), col.begin() + D.n_int0, by_key);
        std::sort(col.begin() + D.n_int0, col.end(), by_key);
        all = col;
        std::sort(all.begin(), all.end(), by_key);
        if ((rc = upload(pb, &D.pen_all, all.data(), all.size())) || (rc = upload(pb, &D.pen_col, col.data(), col.size())) ||
            (rc = upload(pb, &D.bnd_list, bl.data(), bl.size())))
            return rc;
        if (l > 0 && L.ratio == 1) {
            std::vector<int> cb(bl.size());
            for (size_t t = 0; t < bl.size(); ++t) cb[t] = pb->levels[l - 1].bnd_of[bl[t]];
            if ((rc = upload(pb, &D.bl_cbnd, cb.data(), cb.size()))) return rc;
        }
        D.pencil = true;
    }
    {
        // whole-level batches, the two colours merged by relative position
        const int cpb = cells_per_block(L.d, L.p);
        const int nb0 = (L.n_col0 + cpb - 1) / cpb, nb1 = (L.n_act - L.n_col0 + cpb - 1) / cpb;
        std::vector<int> starts;
        int i0 = 0, i1 = 0;
        while (i0 < nb0 || i1 < nb1) {
            bool take0 = i1 >= nb1 || (i0 < nb0 && (2.0 * i0 + 1.0) * nb1 <= (2.0 * i1 + 1.0) * nb0);
            starts.push_back(take0 ? (i0++) * cpb : L.n_col0 + (i1++) * cpb);
        }
        D.nbatch = (int)starts.size();
        if ((rc = upload(pb, &D.batch_start, starts.data(), starts.size()))) return rc;
    }
    std::vector<double> sh(L.shifts.size());
    for (size_t i = 0; i < sh.size(); ++i) sh[i] = L.shifts[i] / L.h;
    if ((rc = upload(pb, &D.shift, sh.data(), sh.size()))) return rc;
    const int nc = L.nc;
    std::vector<double> bt((size_t)nc * nc);
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) bt[(size_t)j * nc + i] = L.Bint[(size_t)i * nc + j];
    if ((rc = upload(pb, &D.Bint_t, bt.data(), bt.size()))) return rc;
    {
        size_t tot = (size_t)L.n_bnd * nc * nc;
        if ((rc = dalloc(pb, &D.Bbnd_t, tot))) return rc;
        if (tot) {
            std::vector<T> tmp(tot);
            for (int b = 0; b < L.n_bnd; ++b) {
                const double *B = &L.Bbnd[(size_t)b * nc * nc];
                T *o = &tmp[(size_t)b * nc * nc];
                for (int i = 0; i < nc; ++i)
                    for (int j = 0; j < nc; ++j) o[(size_t)j * nc + i] = (T)B[(size_t)i * nc + j];
            }
            HIPCHK(hipMemcpy(D.Bbnd_t, tmp.data(), tot * sizeof(T), hipMemcpyHostToDevice));
        }
    }
    if (l > 0) {
        const HostLevel &Lc = pb->levels[l - 1];
        if ((rc = upload(pb, &D.parent, L.parent.data(), L.parent.size()))) return rc;
        if ((rc = upload(pb, &D.childpos, L.childpos.data(), L.childpos.size()))) return rc;
        if ((rc = upload(pb, &D.children, L.children.data(), L.children.size()))) return rc;
        {
            // coarse cells in lexicographic order of their mesh position (both
            // colours mixed), so that the contiguous batch range an XCD takes in
            // the fused residual-restriction is one spatial region
            const int nch = (int)(L.children.size() / std::max<size_t>(1, Lc.cells.size() / Lc.d));
            std::vector<long long> key(Lc.n_act);
            std::vector<int> ord(Lc.n_act);
            for (int k = 0; k < Lc.n_act; ++k) {
                long long v = 0;
                for (int c = Lc.d - 1; c >= 0; --c) v = v * Lc.n + Lc.cells[(size_t)k * Lc.d + c];
                key[k] = v;
                ord[k] = k;
            }
            std::sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] < key[y]; });
            std::vector<int> perm((size_t)Lc.n_act * nch);
            for (int g = 0; g < Lc.n_act; ++g)
                for (int o = 0; o < nch; ++o) perm[(size_t)g * nch + o] = L.children[(size_t)ord[g] * nch + o];
            std::vector<int> gbnd(Lc.n_act);
            for (int g = 0; g < Lc.n_act; ++g) gbnd[g] = Lc.bnd_of[ord[g]];
            if ((rc = upload(pb, &D.rr_perm, perm.data(), perm.size())) ||
                (rc = upload(pb, &D.rr_grp, ord.data(), ord.size())) ||
                (rc = upload(pb, &D.rr_gbnd, gbnd.data(), gbnd.size())))
                return rc;
        }
        double P1[2][MAXN1][MAXN1];
        embedding_1d(Lc, L, P1);
        for (int o = 0; o < 2; ++o)
            for (int a = 0; a < MAXN1; ++a)
                for (int b = 0; b < MAXN1; ++b) D.P1[o][a][b] = (T)P1[o][a][b];
        D.pc = Lc.p;
    }
    KRef<double> kr;
    double omega = pb->opt.omega;
    make_kref(L, pb->opt, omega, kr);
    cast_kref(kr, D.kref);
    size_t nd = (size_t)L.n_act * nc;
    if ((rc = dalloc(pb, &D.z, nd))) return rc;
    if ((rc = dalloc(pb, &D.b, nd))) return rc;
    if ((rc = dalloc(pb, &D.r, nd))) return rc;
    return SBM_OK;
}

template <typename T>
CellArgs<T> cell_args(const DevLevel<T> &D, bool learned) {
    CellArgs<T> a;
    a.nbr = D.nbr;
    a.shift = D.shift;
    a.bnd_of = D.bnd_of;
    a.Bint_t = D.Bint_t;
    a.Bbnd_t = D.Bbnd_t;
    a.lw = learned ? D.lw : nullptr;
    a.lU = learned ? D.lU : nullptr;
    a.lV = learned ? D.lV : nullptr;
    a.batch_start = nullptr;
    a.nbatch = 0;
    a.split = D.n_col0;
    a.perm = nullptr;
    a.skip_interior = 0;
    return a;
}

template <typename T>
std::vector<DevLevel<T>> &devlevels(sbm_problem *pb);
template <>
std::vector<DevLevel<double>> &devlevels<double>(sbm_problem *pb) { return pb->dev64; }
template <>
std::vector<DevLevel<float>> &devlevels<float>(sbm_problem *pb) { return pb->dev32; }

template <typename T>
int level_apply(sbm_problem *pb, int l, int op, const T *x, T *y, const T *b) {
    auto &D = devlevels<T>(pb)[l];
    CellArgs<T> a = cell_args(D, false);
    if (D.pencil) {
        // boundary cells one thread per DoF, interior cells in the pencil form
        // (disjoint outputs): in one launch, except the FP64 Q3 operator (its
        // one-launch form measured 137.7 against 134.7 us on the 96^3 sphere,
        // the register budget the larger of the two kernels'; on the 64^3 Q2
        // sphere the FP64 one-launch apply takes 22.0 against 23.9 us)
        if (sizeof(T) == 4 || D.p == 2) {
            KCHK(launch_fused<T>(D.d, D.p, op, D.n_bl0 + D.n_bl1, D.bnd_list, D.n_int0 + D.n_int1, D.pen_all, x, y, b,
                                 a, D.kref, pb->stream, nullptr));
        } else {
            a.perm = D.bnd_list;
            KCHK(launch_cellop<T>(D.d, D.p, op, 0, D.n_bl0 + D.n_bl1, x, y, b, a, D.kref, pb->stream));
            KCHK(launch_pencil<T>(D.d, D.p, op, D.n_int0 + D.n_int1, D.pen_all, x, y, b, a, D.kref, pb->stream,
                                  nullptr));
        }
        return SBM_OK;
    }
    a.batch_start = D.batch_start;
    a.nbatch = D.nbatch;
    KCHK(launch_cellop<T>(D.d, D.p, op, 0, D.n_act, x, y, b, a, D.kref, pb->stream));
    return SBM_OK;
}

// em: the updated cells' values also go there (see EmitArgs)
template <typename T>
int colour_update(sbm_problem *pb, int l, int colour, const T *b, T *z, const EmitArgs<T> *em = nullptr) {
    auto &D = devlevels<T>(pb)[l];
    int c0 = colour == 0 ? 0 : D.n_col0;
    int nc = colour == 0 ? D.n_col0 : D.n_act - D.n_col0;
    bool learned = pb->learned_on && D.lw != nullptr && l == (int)pb->levels.size() - 1;
    if (D.pencil && (em == nullptr || em->kind == EMIT_F64)) {
        // the learned correction acts on boundary cells only (the same inputs,
        // disjoint outputs)
        CellArgs<T> a = cell_args(D, learned);
        const int nb = colour == 0 ? D.n_bl0 : D.n_bl1, ni = colour == 0 ? D.n_int0 : D.n_int1;
        const int *bl = D.bnd_list + (colour == 0 ? 0 : D.n_bl0), *il = D.pen_col + (colour == 0 ? 0 : D.n_int0);
        // one launch (FP32: 64^3 Q2 sphere solve 6.06 -> 5.44 ms, 96^3 Q3
        // sphere 86.0 -> 84.7 ms; FP64: 96^3 Q3 sphere solve 120.6 -> 117.0 ms,
        // 64^3 Q2 7.46 -> 7.31 ms)
        KCHK(launch_fused<T>(D.d, D.p, OP_SMOOTH, nb, bl, ni, il, z, z, b, a, D.kref, pb->stream, em));
        return SBM_OK;
    }
    KCHK(launch_cellop<T>(D.d, D.p, OP_SMOOTH, c0, nc, z, z, b, cell_args(D, learned), D.kref, pb->stream, em));
    return SBM_OK;
}

// the block update on the listed cells of level l only (no learned correction)
template <typename T>
int list_update(sbm_problem *pb, int l, const int *cells, int count, const T *b, T *z,
                const EmitArgs<T> *em = nullptr) {
    auto &D = devlevels<T>(pb)[l];
    CellArgs<T> a = cell_args(D, false);
    a.perm = cells;
    KCHK(launch_cellop<T>(D.d, D.p, OP_SMOOTH, 0, count, z, z, b, a, D.kref, pb->stream, em));
    return SBM_OK;
}

// Emission of level l - 1's final z into level l's zf: zf += P z (Sec. 3.2)
template <typename T>
EmitArgs<T> prolong_emit(sbm_problem *pb, int l, T *zf) {
    auto &Df = devlevels<T>(pb)[l];
    EmitArgs<T> e{};
    e.kind = pb->levels[l].ratio == 2 ? EMIT_H : EMIT_P;
    e.children = Df.children;
    e.zf = zf;
    e.z64 = nullptr;
    std::memcpy(e.P1, Df.P1, sizeof(e.P1));
    return e;
}

template <typename T>
int restrict_to(sbm_problem *pb, int l, const T *rf, T *bc) {
    auto &Df = devlevels<T>(pb)[l];
    auto &Dc = devlevels<T>(pb)[l - 1];
    TransferArgs<T> tr;
    std::memcpy(tr.P1, Df.P1, sizeof(tr.P1));
    int nch = pb->levels[l].ratio == 2 ? (1 << Df.d) : 1;
    KCHK(launch_restrict<T>(Df.d, Dc.n_act, Df.p + 1, Dc.p + 1, nch, Df.children, rf, bc, tr, pb->stream));
    return SBM_OK;
}

// bc = R (b - A_l z): residual of level l restricted to level l - 1, one
// launch; with zc also level l - 1's zero-start colour-0 update zc = omega B bc
// (colour 0) and 0 (colour 1)
template <typename T>
int resid_restrict(sbm_problem *pb, int l, const T *z, const T *b, T *bc, T *zc = nullptr) {
    auto &Df = devlevels<T>(pb)[l];
    auto &Dc = devlevels<T>(pb)[l - 1];
    TransferArgs<T> tr;
    std::memcpy(tr.P1, Df.P1, sizeof(tr.P1));
    const int nch = pb->levels[l].ratio == 2 ? (1 << Df.d) : 1;
    // p-transfers keep the cells: the whole-level batch table, no child lists
    CellArgs<T> ca = cell_args(Df, false);
    ca.batch_start = Df.batch_start;
    ca.nbatch = Df.nbatch;
    ZeroStartArgs<T> zs{};
    if (zc != nullptr) {
        zs.z = zc;
        zs.bnd_of = Dc.bnd_of;
        zs.grp_bnd = nch == 1 ? nullptr : Df.rr_gbnd;
        zs.Bint_t = Dc.Bint_t;
        zs.Bbnd_t = Dc.Bbnd_t;
        zs.split = Dc.n_col0;
        zs.omega = Dc.kref.omega;
    }
    // After a smoothing step that ends with a colour-0 block solve (omega = 1,
    // unshifted inverses, no learned correction on this level) the colour-0
    // residual is zero up to rounding on every cell whose inverse is exact: a
    // p-transfer then computes colour 1 (the cells map one to one, so the
    // colour-0 part of bc is zero) and, in a second launch, the colour-0 cells
    // whose inverse the stabilisation changed.
    const bool learned_here = pb->learned_on && l == (int)pb->levels.size() - 1 && Df.lw != nullptr;
    const bool c1_only = nch == 1 && pb->opt.smoother == 0 && pb->opt.nu_pre > 0 && pb->opt.omega == 1.0 &&
                         pb->opt.allow_singular == 0 && !learned_here &&
                         (pb->levels[l].n_clipped == 0 || Df.hold != nullptr);
    if (c1_only && Df.pencil) {
        // colour 0 of bc (and of the zero start) is zero; colour 1: boundary
        // cells by the cell kernel on its list, interior cells by the pencil kernel
        const long long n0 = (long long)Dc.n_col0 * Dc.nc;
        KCHK(launch_zero2<T>(n0, bc, zc, pb->stream));
        ZeroStartArgs<T> zb = zs;
        zb.grp_bnd = Df.bl_cbnd != nullptr ? Df.bl_cbnd + Df.n_bl0 : nullptr;
        if (Df.n_bl1 > 0)
            KCHK(launch_resid_restrict<T>(Df.d, Df.p, Df.n_bl1, 1, Dc.p + 1, Df.bnd_list + Df.n_bl0,
                                          Df.bnd_list + Df.n_bl0, z, b, bc, ca, Df.kref, tr, pb->stream,
                                          zc != nullptr ? &zb : nullptr, false));
        KCHK(launch_pencil_rr<T>(Df.d, Df.p, Df.n_int1, Df.pen_col + Df.n_int0, z, b, bc, zc, ca, Df.kref, tr,
                                 pb->stream));
    } else if (Df.pencil && nch == 1 && zc == nullptr && pb->opt.smoother == 1) {
        // the Chebyshev cycle (transfers never fused): every cell, boundary
        // cells by the cell kernel on their list, interior cells by the pencil
        // kernel.  (The SSOR cycle keeps one kernel for this step whether its
        // transfers are fused or not: the two forms share their arithmetic.)
        if (Df.n_bl0 + Df.n_bl1 > 0)
            KCHK(launch_resid_restrict<T>(Df.d, Df.p, Df.n_bl0 + Df.n_bl1, 1, Dc.p + 1, Df.bnd_list, Df.bnd_list, z, b,
                                          bc, ca, Df.kref, tr, pb->stream, nullptr, false));
        KCHK(launch_pencil_rr<T>(Df.d, Df.p, Df.n_int0 + Df.n_int1, Df.pen_all, z, b, bc, nullptr, ca, Df.kref, tr,
                                 pb->stream));
    } else {
        KCHK(launch_resid_restrict<T>(Df.d, Df.p, Dc.n_act, nch, Dc.p + 1, nch == 1 ? nullptr : Df.rr_perm,
                                      nch == 1 ? nullptr : Df.rr_grp, z, b, bc, ca, Df.kref, tr, pb->stream,
                                      zc != nullptr ? &zs : nullptr, c1_only));
    }
    if (c1_only && Df.n_clip0 > 0) {
        ZeroStartArgs<T> zl = zs;
        zl.grp_bnd = Df.clip0_cbnd;
        KCHK(launch_resid_restrict<T>(Df.d, Df.p, Df.n_clip0, 1, Dc.p + 1, Df.clip0, Df.clip0, z, b, bc, ca, Df.kref,
                                      tr, pb->stream, zc != nullptr ? &zl : nullptr, false));
    }
    return SBM_OK;
}

template <typename T>
int prolong_add(sbm_problem *pb, int l, const T *zc, T *zf) {
    auto &Df = devlevels<T>(pb)[l];
    auto &Dc = devlevels<T>(pb)[l - 1];
    TransferArgs<T> tr;
    std::memcpy(tr.P1, Df.P1, sizeof(tr.P1));
    if (Df.pencil && Dc.pencil && pb->levels[l].ratio == 1 && Dc.p + 1 == Df.p) {
        // p-transfer between pencil levels (which never fold it into their
        // colour updates, so the fused and the separate cycle both come here):
        // sum factorised, one lane per fine line
        KCHK(launch_pencil_prolong<T>(Df.d, Df.p, Df.n_act, Df.parent, zc, zf, tr, pb->stream));
        return SBM_OK;
    }
    KCHK(launch_prolong<T>(Df.d, Df.n_act, Df.p + 1, Dc.p + 1, Df.parent, Df.childpos, zc, zf, tr, pb->stream));
    return SBM_OK;
}

// One SSOR step: colours 0, 1, 1, 0.  With omega = 1, the first colour-1
// update zeroes the residual of every colour-1 cell whose inverse is exact,
// and nothing it depends on changes before the repeated colour-1 update (cells
// of one colour do not couple), so the repeat adds zero there up to rounding:
// it runs only on the colour-1 cells whose inverse the stabilisation changed
// (none: it is skipped), and the first update holds back their emission.
// With omega != 1, allow_singular (every block is then (D_K + eps I)^-1) or
// the learned correction the full repeat is kept.
// from_zero: z starts at zero; with b64 (FP32 cycle only) the right-hand side
// is read in FP64 and its FP32 copy written to b on the way.  started: that
// first colour-0 update from zero was already formed (by the finer level's
// residual-restriction kernel).  em: the last update of each colour also sends
// the values on (they are final after it when this is the last step).
template <typename T>
int ssor_step(sbm_problem *pb, int l, const T *b, T *z, bool from_zero = false, const double *b64 = nullptr,
              bool started = false, const EmitArgs<T> *em = nullptr) {
    const bool learned_here = pb->learned_on && l == (int)pb->levels.size() - 1;
    auto &DL = devlevels<T>(pb)[l];
    const bool exact_repeat = pb->opt.omega == 1.0 && pb->opt.allow_singular == 0 && !learned_here &&
                              (pb->levels[l].n_clipped == 0 || DL.hold != nullptr);
    const bool skip_repeat = exact_repeat && DL.n_rep1 == 0;
    const bool list_repeat = exact_repeat && DL.n_rep1 > 0;
    int rc;
    if (started) {
        // nothing: z holds the zero-start colour-0 update
    } else if (from_zero && DL.pencil) {
        // boundary cells, the colour-1 zeros and the FP32 copy of b by the
        // per-DoF kernel, interior colour-0 cells by the pencil kernel
        CellArgs<T> ca = cell_args(DL, learned_here && DL.lw != nullptr);
        ca.skip_interior = 1;
        const hipStream_t bs = pb->stream;   // (both launches on the problem's stream)
        if (b64 != nullptr) {
            KCHK((launch_smooth_zero<T, double>(DL.d, DL.p, DL.n_act, DL.n_col0, b64, const_cast<T *>(b), z, ca,
                                                DL.kref.omega, bs)));
            KCHK((launch_pencil_zero<T, double>(DL.d, DL.p, DL.n_int0, DL.pen_col, b64, z, DL.Bint_t, DL.kref.omega,
                                                pb->stream)));
        } else {
            KCHK((launch_smooth_zero<T, T>(DL.d, DL.p, DL.n_act, DL.n_col0, b, (T *)nullptr, z, ca, DL.kref.omega, bs)));
            KCHK((launch_pencil_zero<T, T>(DL.d, DL.p, DL.n_int0, DL.pen_col, b, z, DL.Bint_t, DL.kref.omega,
                                           pb->stream)));
        }
    } else if (from_zero) {
        auto &D = devlevels<T>(pb)[l];
        const CellArgs<T> ca = cell_args(D, learned_here && D.lw != nullptr);
        if (b64 != nullptr) {
            KCHK((launch_smooth_zero<T, double>(D.d, D.p, D.n_act, D.n_col0, b64, const_cast<T *>(b), z, ca,
                                                D.kref.omega, pb->stream)));
        } else {
            KCHK((launch_smooth_zero<T, T>(D.d, D.p, D.n_act, D.n_col0, b, (T *)nullptr, z, ca, D.kref.omega,
                                           pb->stream)));
        }
    } else if ((rc = colour_update<T>(pb, l, 0, b, z))) {
        return rc;
    }
    if (list_repeat) {
        EmitArgs<T> eh{};
        if (em != nullptr) {
            eh = *em;
            eh.hold = DL.hold;
        }
        if ((rc = colour_update<T>(pb, l, 1, b, z, em != nullptr ? &eh : nullptr))) return rc;
        if ((rc = list_update<T>(pb, l, DL.rep1, DL.n_rep1, b, z, em))) return rc;
    } else {
        if (!skip_repeat && (rc = colour_update<T>(pb, l, 1, b, z))) return rc;
        if ((rc = colour_update<T>(pb, l, 1, b, z, em))) return rc;
    }
    return colour_update<T>(pb, l, 0, b, z, em);
}

// b64 (FP32 cycle at the finest level only): the FP64 right-hand side; b is
// then the cycle's own FP32 buffer, filled by the first smoothing kernel.
// started: z already holds the zero-start colour-0 update (formed by the finer
// level).  em: where the final z also goes; *emitted says whether it went
// (else the caller moves it itself).  With fused transfers (the default) the
// restriction forms the coarser level's zero-start update and the coarser
// level's last smoothing kernels add its final z into this level's z, so
// neither needs a launch of its own.
// One Chebyshev smoothing step on level l: cheb_degree additive block-Jacobi
// updates z += d_k, d_k = a_k d_(k-1) + c_k B (b - A z), with the weights of
// the Chebyshev iteration for the eigenvalue interval [lmax / range, lmax] of
// B A (theta, delta: its centre and half width; rho_k = 1 / (2 sigma -
// rho_(k-1)), sigma = theta / delta, a_k = rho_k rho_(k-1), c_k = 2 rho_k /
// delta, d_0 = B r / theta).  from_zero: z = 0 on entry (the first residual
// is b).
template <typename T>
int cheb_smooth(sbm_problem *pb, int l, const T *b, T *z, bool from_zero) {
    auto &D = devlevels<T>(pb)[l];
    const double lmax = D.cheb_lmax, lmin = lmax / pb->opt.cheb_range;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho_old = 1.0 / sigma;
    for (int k = 0; k < pb->opt.cheb_degree; ++k) {
        const T *r = b;
        if (!(k == 0 && from_zero)) {
            int rc;
            if ((rc = level_apply<T>(pb, l, OP_RESID, z, D.r, b))) return rc;
            r = D.r;
        }
        double alpha = 0.0, beta = 1.0 / theta;
        if (k > 0) {
            const double rho = 1.0 / (2.0 * sigma - rho_old);
            alpha = rho * rho_old;
            beta = 2.0 * rho / delta;
            rho_old = rho;
        }
        if (D.pencil) {
            // boundary cells on their list, interior cells by the pencil kernel
            KCHK(launch_block_jacobi<T>(D.n_bl0 + D.n_bl1, D.nc, D.bnd_of, D.Bint_t, D.Bbnd_t, r, D.dcheb, z, (T)alpha,
                                        (T)beta, pb->stream, D.bnd_list));
            KCHK(launch_pencil_bj<T>(D.d, D.p, D.n_int0 + D.n_int1, D.pen_all, r, D.dcheb, z, D.Bint_t, (T)alpha,
                                     (T)beta, pb->stream));
        } else {
            KCHK(launch_block_jacobi<T>(D.n_act, D.nc, D.bnd_of, D.Bint_t, D.Bbnd_t, r, D.dcheb, z, (T)alpha, (T)beta,
                                        pb->stream));
        }
    }
    return SBM_OK;
}

template <typename T>
int vcycle_rec(sbm_problem *pb, int l, const T *b, T *z, const double *b64 = nullptr, bool started = false,
               const EmitArgs<T> *em = nullptr, bool *emitted = nullptr);

// V-cycle with the Chebyshev block-Jacobi smoother (separate transfer kernels)
template <typename T>
int vcycle_cheb(sbm_problem *pb, int l, const T *b, T *z, const double *b64) {
    auto &D = devlevels<T>(pb)[l];
    const long long nd = (long long)D.n_act * D.nc;
    if constexpr (std::is_same<T, float>::value) {
        if (b64 != nullptr) KCHK(launch_cast_d2f(nd, b64, const_cast<float *>(b), pb->stream));
    }
    int rc;
    KCHK(launch_fill<T>(nd, z, T(0), pb->stream));
    for (int s = 0; s < pb->opt.nu_pre; ++s)
        if ((rc = cheb_smooth<T>(pb, l, b, z, s == 0))) return rc;
    auto &Dc = devlevels<T>(pb)[l - 1];
    if ((rc = resid_restrict<T>(pb, l, z, b, Dc.b, nullptr))) return rc;
    if ((rc = l - 1 == 0 ? vcycle_rec<T>(pb, 0, Dc.b, Dc.z) : vcycle_cheb<T>(pb, l - 1, Dc.b, Dc.z, nullptr)))
        return rc;
    if ((rc = prolong_add<T>(pb, l, Dc.z, z))) return rc;
    for (int s = 0; s < pb->opt.nu_post; ++s)
        if ((rc = cheb_smooth<T>(pb, l, b, z, false))) return rc;
    return SBM_OK;
}

template <typename T>
int vcycle_rec(sbm_problem *pb, int l, const T *b, T *z, const double *b64, bool started, const EmitArgs<T> *em,
               bool *emitted) {
    auto &D = devlevels<T>(pb)[l];
    if (emitted) *emitted = false;
    if (l > 0 && pb->opt.smoother == 1) return vcycle_cheb<T>(pb, l, b, z, b64);
    // a pencil level keeps its values to itself (the pencil kernel does not
    // embed into the finer level): the caller prolongs them separately
    if (l > 0 && D.pencil && em != nullptr && (em->kind == EMIT_H || em->kind == EMIT_P)) em = nullptr;
    if (l == 0) {
        if constexpr (std::is_same<T, float>::value) {
            // a one-level hierarchy: the FP32 copy of the right-hand side first
            if (b64 != nullptr) KCHK(launch_cast_d2f(pb->coarse.n, b64, const_cast<float *>(b), pb->stream));
        }
        // the coarsest problem is tiny and can be badly conditioned: the FP32
        // cycle also solves it with the FP64 inverse
        if (em != nullptr && (em->kind == EMIT_H || em->kind == EMIT_P) && D.p == 1) {
            KCHK(launch_coarse_solve_prolong<T>(D.d, pb->coarse.n, pb->coarse.Ainv64, b, z, *em, pb->stream));
            if (emitted) *emitted = true;
        } else {
            KCHK((launch_dense_gemv<double, T>(pb->coarse.n, pb->coarse.Ainv64, b, z, pb->stream)));
        }
        return SBM_OK;
    }
    const bool fuse = pb->opt.fuse_transfers != 0;
    const int nu_pre = pb->opt.nu_pre, nu_post = pb->opt.nu_post;
    int rc;
    if (nu_pre > 0) {
        // z starts at zero: the first colour-0 update needs no operator application
        if ((rc = ssor_step<T>(pb, l, b, z, true, b64, started))) return rc;
    } else {
        if constexpr (std::is_same<T, float>::value) {
            if (b64 != nullptr) KCHK(launch_cast_d2f(D.n_act * (long long)D.nc, b64, const_cast<float *>(b), pb->stream));
        }
        KCHK(launch_fill<T>((long long)D.n_act * D.nc, z, T(0), pb->stream));
    }
    for (int s = 1; s < nu_pre; ++s)
        if ((rc = ssor_step<T>(pb, l, b, z))) return rc;
    auto &Dc = devlevels<T>(pb)[l - 1];
    const bool zs = fuse && nu_pre > 0 && l - 1 > 0;
    if ((rc = resid_restrict<T>(pb, l, z, b, Dc.b, zs ? Dc.z : nullptr))) return rc;
    EmitArgs<T> up{};
    if (fuse) up = prolong_emit<T>(pb, l, z);
    bool done = false;
    if ((rc = vcycle_rec<T>(pb, l - 1, Dc.b, Dc.z, nullptr, zs, fuse ? &up : nullptr, &done))) return rc;
    if (!done && (rc = prolong_add<T>(pb, l, Dc.z, z))) return rc;
    for (int s = 0; s < nu_post; ++s)
        if ((rc = ssor_step<T>(pb, l, b, z, false, nullptr, false, s == nu_post - 1 ? em : nullptr))) return rc;
    if (emitted) *emitted = em != nullptr && nu_post > 0;
    return SBM_OK;
}

int check_level(sbm_problem *pb, int &level) {
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) {
        pb->last_error = "level out of range";
        return SBM_EINVAL;
    }
    return SBM_OK;
}

}  // namespace

template <typename T>
int refresh_level(sbm_problem *pb, int l, DevLevel<T> &D) {
    const HostLevel &L = pb->levels[l];
    const int nc = L.nc;
    int rc;
    if ((rc = clip_lists(pb, l, D, false))) return rc;
    if (L.n_surr) {
        std::vector<T> sh(L.shifts.size());
        for (size_t i = 0; i < sh.size(); ++i) sh[i] = (T)(L.shifts[i] / L.h);
        HIPCHK(hipMemcpy(D.shift, sh.data(), sh.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    const size_t tot = (size_t)L.n_bnd * nc * nc;
    if (tot) {
        std::vector<T> tmp(tot);
        for (int b = 0; b < L.n_bnd; ++b) {
            const double *B = &L.Bbnd[(size_t)b * nc * nc];
            T *o = &tmp[(size_t)b * nc * nc];
            for (int i = 0; i < nc; ++i)
                for (int j = 0; j < nc; ++j) o[(size_t)j * nc + i] = (T)B[(size_t)i * nc + j];
        }
        HIPCHK(hipMemcpy(D.Bbnd_t, tmp.data(), tot * sizeof(T), hipMemcpyHostToDevice));
    }
    return SBM_OK;
}

namespace sbm {
int finest_residual(sbm_problem *pb, const double *x, const double *b, double *r) {
    return level_apply<double>(pb, (int)pb->levels.size() - 1, OP_RESID, x, r, b);
}
}  // namespace sbm

extern "C" {

const char *sbm_strerror(int s) {
    switch (s) {
        case SBM_OK: return "ok";
        case SBM_NOT_CONVERGED: return "not converged";
        case SBM_EINVAL: return "invalid argument";
        case SBM_ENOMEM: return "out of memory";
        case SBM_EDEVICE: return "HIP device error";
        case SBM_ESINGULAR: return "singular block";
        case SBM_ENONFINITE: return "non-finite value";
        case SBM_EGEOM: return "closest-point search failed";
    }
    return "unknown status";
}

const char *sbm_last_error(const sbm_problem *pb) { return pb ? pb->last_error.c_str() : ""; }

int sbm_default_options(int dim, int p, sbm_options *o) {
    if (!o || (dim != 2 && dim != 3) || p < 1 || p > 3) return SBM_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->lo = -1.0;
    o->hi = 1.0;
    o->c_F = 2.0;
    o->c_G = 5.0;
    o->alpha = 1.0;
    o->ext = 1;
    o->omega = p >= 3 ? 0.8 : 1.0;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->coarse_min = 3;
    o->coarse_dofs = 2048;
    o->vcycle_fp32 = 0;
    o->allow_singular = 0;
    o->fuse_transfers = 1;
    o->penalty_p = 0;
    o->lambda_frac = 0.0;
    o->frac_m = 16;
    o->min_neighbours = 0;
    o->smoother = 0;
    o->cheb_degree = 3;
    o->cheb_range = 20.0;
    o->pencil = 1;
    o->stab = 0.0;
    o->device = 0;
    o->stream = nullptr;
    return SBM_OK;
}

int sbm_destroy(sbm_problem *pb) {
    if (!pb) return SBM_OK;
    hipSetDevice(pb->opt.device);
    for (void *q : pb->allocations) hipFree(q);
    if (pb->pinned) hipHostFree(pb->pinned);
    delete pb;
    return SBM_OK;
}

// Chebyshev smoother: direction vectors of every smoothed level and the
// largest eigenvalue modulus of B A per level, by 25 power iterations in FP64
// from the normalised all-ones vector (v <- B A v / |B A v|; the estimate is
// the last |B A v|), taken 1.2 times as the interval's upper end.
static int chebyshev_setup(sbm_problem *pb) {
    int rc;
    double *part = nullptr, *scal = nullptr;
    if ((rc = dalloc(pb, &part, (size_t)sbm::gs_partials_max())) || (rc = dalloc(pb, &scal, (size_t)2))) return rc;
    hipStream_t s = pb->stream;
    for (size_t l = 1; l < pb->levels.size(); ++l) {
        auto &D64 = pb->dev64[l];
        auto &D32 = pb->dev32[l];
        const long long nd = (long long)D64.n_act * D64.nc;
        if ((rc = dalloc(pb, &D64.dcheb, (size_t)nd)) || (rc = dalloc(pb, &D32.dcheb, (size_t)nd))) return rc;
        KCHK(launch_fill<double>(nd, D64.b, 1.0 / std::sqrt((double)nd), s));
        for (int it = 0; it < 25; ++it) {
            if ((rc = level_apply<double>(pb, (int)l, OP_APPLY, D64.b, D64.r, nullptr))) return rc;
            KCHK(launch_block_jacobi<double>(D64.n_act, D64.nc, D64.bnd_of, D64.Bint_t, D64.Bbnd_t, D64.r, D64.dcheb,
                                             nullptr, 0.0, 1.0, s));
            KCHK(launch_gs_dots(nd, 0, nullptr, D64.dcheb, part, s));
            KCHK(launch_gs_reduce(nd, 1, part, scal, s));
            KCHK(launch_scale(nd, scal, D64.dcheb, D64.b, s));
        }
        double lam2 = 0.0;
        HIPCHK(hipMemcpyAsync(&lam2, scal, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!(lam2 > 0.0) || !std::isfinite(lam2)) {
            pb->last_error = "Chebyshev smoother: eigenvalue estimate failed on level " + std::to_string(l);
            return SBM_ENONFINITE;
        }
        D64.cheb_lmax = D32.cheb_lmax = 1.2 * std::sqrt(lam2);
    }
    return SBM_OK;
}

static int setup_body(const sbm_geometry *g, int n, int p, const sbm_options *o, sbm_problem **out, sbm_problem **live) {
    if (!g || !out || n < 1 || p < 1 || p > 3 || (g->dim != 2 && g->dim != 3)) return SBM_EINVAL;
    // cells are indexed by int: the background mesh holds at most 2^31 - 1 cells
    if ((g->dim == 2 ? (double)n * n : (double)n * n * n) > 2147483647.0) return SBM_EINVAL;
    *out = nullptr;
    sbm_problem *pb = new (std::nothrow) sbm_problem();
    if (!pb) return SBM_ENOMEM;
    *live = pb;
    if (o)
        pb->opt = *o;
    else
        sbm_default_options(g->dim, p, &pb->opt);
    sbm_options &op = pb->opt;
    if (!(op.hi > op.lo) || op.nu_pre < 0 || op.nu_post < 0 || op.coarse_min < 1 || op.coarse_dofs < 0 ||
        (op.ext != 0 && op.ext != 1) || op.penalty_p < 0 || op.penalty_p > 3 || !(op.lambda_frac >= 0.0) ||
        op.lambda_frac > 1.0 || op.frac_m < 1 || op.frac_m > 64 || !(op.stab >= 0.0) || op.min_neighbours < 0 ||
        op.min_neighbours > 2 * g->dim || (op.smoother != 0 && op.smoother != 1) || op.cheb_degree < 1 ||
        op.cheb_degree > 64 || !(op.cheb_range > 1.0) || (op.pencil != 0 && op.pencil != 1)) {
        delete pb;
        return SBM_EINVAL;
    }
    Geometry &G = pb->geom;
    G.dim = g->dim;
    G.kind = g->kind;
    if (g->kind == SBM_GEOM_BALLS) {
        if (g->n_balls < 1 || !g->centers || !g->radii) { delete pb; return SBM_EINVAL; }
        G.centers.assign(g->centers, g->centers + (size_t)g->n_balls * g->dim);
        G.radii.assign(g->radii, g->radii + g->n_balls);
    } else if (g->kind == SBM_GEOM_STAR2D) {
        if (g->dim != 2) { delete pb; return SBM_EINVAL; }
        G.r0 = g->star_r0;
        G.a = g->star_a;
        G.k = g->star_k;
    } else if (g->kind == SBM_GEOM_ELLIPSOID) {
        if (g->dim != 3 || !g->centers || !g->radii || !g->rotation) { delete pb; return SBM_EINVAL; }
        G.centers.assign(g->centers, g->centers + 3);
        G.radii.assign(g->radii, g->radii + 3);
        G.rot.assign(g->rotation, g->rotation + 9);
        for (double r : G.radii)
            if (!(r > 0)) { delete pb; return SBM_EINVAL; }
    } else if (g->kind == SBM_GEOM_CALLBACK) {
        if (!g->phi || !g->grad || !g->hess) { delete pb; return SBM_EINVAL; }
        G.cb_phi = g->phi;
        G.cb_grad = g->grad;
        G.cb_hess = g->hess;
        G.user = g->user;
    } else {
        delete pb;
        return SBM_EINVAL;
    }
    pb->dim = g->dim;
    pb->n = n;
    pb->p = p;
    const bool host_only = op.device < 0;
    if (!host_only && hipSetDevice(op.device) != hipSuccess) {
        delete pb;
        return SBM_EDEVICE;
    }
    pb->stream = (hipStream_t)op.stream;
    // finest first: p-levels on the finest mesh, then halve n with p = 1 while
    // n is even, n/2 >= coarse_min and the current level has more than
    // coarse_dofs active DoFs
    {
        std::vector<HostLevel> f2c;
        int nn = n;
        for (int q = p;; ) {
            f2c.emplace_back();
            std::string err;
            int rc = build_level(G, op, nn, q, nn == n, f2c.back(), err);
            if (rc) {
                pb->last_error = err;
                *out = pb;  // caller can read the message, must destroy
                return rc;
            }
            if (q > 1) {
                --q;
                continue;
            }
            const HostLevel &Lc = f2c.back();
            if (nn % 2 != 0 || nn / 2 < op.coarse_min || (long long)Lc.n_act * Lc.nc <= op.coarse_dofs) break;
            nn /= 2;
        }
        pb->levels.assign(f2c.rbegin(), f2c.rend());
    }
    // every level must hold unknowns: the centre rule can leave a level empty
    // (no cell centre inside the domain: an empty domain, or a small one on a
    // coarse mesh when coarse_dofs / coarse_min allow coarsening that far)
    for (const HostLevel &L : pb->levels) {
        if (L.n_act == 0) {
            pb->last_error = "level n = " + std::to_string(L.n) + ", p = " + std::to_string(L.p) +
                             " has no active cell (no cell centre inside the domain): refine the mesh or raise "
                             "coarse_dofs / coarse_min";
            *out = pb;
            return SBM_EINVAL;
        }
    }
    for (size_t l = 1; l < pb->levels.size(); ++l) build_transfer(pb->levels[l - 1], pb->levels[l]);
    const size_t nlev = pb->levels.size();
    // coarsest dense matrix and its inverse
    const HostLevel &L0 = pb->levels[0];
    long long n0 = (long long)L0.n_act * L0.nc;
    if (n0 > 4096) {
        pb->last_error = "coarsest level too large for the dense solver (raise coarse_min)";
        *out = pb;
        return SBM_EINVAL;
    }
    coarse_matrix(L0, op.alpha, op.ext, pb->A0);
    std::vector<double> Ainv = pb->A0;
    if (n0 > 0 && !invert(Ainv.data(), (int)n0, 1e-14, 0.0)) {
        pb->last_error = "singular coarsest-level matrix";
        *out = pb;
        return SBM_ESINGULAR;
    }
    pb->coarse.n = (int)n0;
    pb->host_only = host_only;
    if (host_only) {
        *out = pb;
        return SBM_OK;
    }
    int rc;
    if ((rc = upload(pb, &pb->coarse.Ainv64, Ainv.data(), Ainv.size()))) {
        *out = pb;
        return rc;
    }
    pb->dev64.resize(nlev);
    pb->dev32.resize(nlev);
    for (size_t l = 0; l < nlev; ++l) {
        if ((rc = upload_level<double>(pb, (int)l, pb->dev64[l])) || (rc = upload_level<float>(pb, (int)l, pb->dev32[l]))) {
            *out = pb;
            return rc;
        }
        if (l > 0) {
            std::vector<double>().swap(pb->levels[l].Dbnd);  // only the coarsest keeps D
        }
    }
    if (op.smoother == 1 && (rc = chebyshev_setup(pb))) {
        *out = pb;
        return rc;
    }
    const HostLevel &Lf = pb->levels.back();
    size_t nd = (size_t)Lf.n_act * Lf.nc;
    if ((rc = dalloc(pb, &pb->f32_in, nd)) || (rc = dalloc(pb, &pb->f32_out, nd))) {
        *out = pb;
        return rc;
    }
    pb->arnoldi.assign(sbm::ARNOLDI_DOUBLES, 0.0);
    if (hipHostMalloc((void **)&pb->pinned, sbm::SOLVE_SCALARS * sizeof(double)) != hipSuccess) {
        *out = pb;
        return SBM_ENOMEM;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        *out = pb;
        return SBM_EDEVICE;
    }
    *out = pb;
    return SBM_OK;
}

// Host containers throw std::bad_alloc; nothing may leave through the C ABI:
// a failed setup releases what it had built.
int sbm_setup(const sbm_geometry *g, int n, int p, const sbm_options *o, sbm_problem **out) {
    sbm_problem *live = nullptr;
    int rc = SBM_ENOMEM;
    try {
        return setup_body(g, n, p, o, out, &live);
    } catch (const std::bad_alloc &) {
        rc = SBM_ENOMEM;
    } catch (...) {
        rc = SBM_EINVAL;
    }
    if (out) *out = nullptr;
    if (live) sbm_destroy(live);
    return rc;
}

int sbm_layout_info(const sbm_problem *pb, sbm_layout *o) {
    if (!pb || !o) return SBM_EINVAL;
    const HostLevel &L = pb->levels.back();
    o->n_dofs = (long long)L.n_act * L.nc;
    o->n_active = L.n_act;
    o->n_colour0 = L.n_col0;
    o->dofs_per_cell = L.nc;
    o->n_levels = (int)pb->levels.size();
    o->n_boundary_cells = L.n_bnd;
    o->n_surrogate_faces = L.n_surr;
    return SBM_OK;
}

int sbm_level_info(const sbm_problem *pb, int level, int *n, int *p, int *n_active, int *n_colour0, int *n_surr) {
    if (!pb) return SBM_EINVAL;
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    const HostLevel &L = pb->levels[level];
    if (n) *n = L.n;
    if (p) *p = L.p;
    if (n_active) *n_active = L.n_act;
    if (n_colour0) *n_colour0 = L.n_col0;
    if (n_surr) *n_surr = L.n_surr;
    return SBM_OK;
}

int sbm_level_blocks(const sbm_problem *pb, int level, int *n_boundary, int *n_clipped, int *n_clipped_colour0) {
    if (!pb) return SBM_EINVAL;
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    const HostLevel &L = pb->levels[level];
    int c0 = 0;
    for (int K = 0; K < L.n_col0; ++K) {
        const int bi = L.bnd_of[K];
        if (bi >= 0 && (size_t)bi < L.clipped.size() && L.clipped[bi]) ++c0;
    }
    if (n_boundary) *n_boundary = L.n_bnd;
    if (n_clipped) *n_clipped = L.n_clipped;
    if (n_clipped_colour0) *n_clipped_colour0 = c0;
    return SBM_OK;
}

int sbm_active_cells(const sbm_problem *pb, int level, int *ijk, long long cap) {
    if (!pb) return SBM_EINVAL;
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    const HostLevel &L = pb->levels[level];
    if (cap < (long long)L.cells.size() || (!ijk && !L.cells.empty())) return SBM_EINVAL;
    if (!L.cells.empty()) std::memcpy(ijk, L.cells.data(), L.cells.size() * sizeof(int));
    return SBM_OK;
}

int sbm_shifts(const sbm_problem *pb, int level, double *out, long long cap) {
    if (!pb) return SBM_EINVAL;
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    const HostLevel &L = pb->levels[level];
    if (cap < (long long)L.shifts.size() || (!out && !L.shifts.empty())) return SBM_EINVAL;
    if (!L.shifts.empty()) std::memcpy(out, L.shifts.data(), L.shifts.size() * sizeof(double));
    return SBM_OK;
}

static int rhs_body(sbm_problem *pb, sbm_field_fn f, sbm_field_fn g, void *user, double *b_dev) {
    if (!pb || pb->host_only || !f || !g || !b_dev) return SBM_EINVAL;
    const HostLevel &L = pb->levels.back();
    const int d = L.d, n1 = L.n1, nc = L.nc, nf = L.nf;
    const Ref1D &r = L.ref;
    const double h = L.h, alpha = pb->opt.alpha;
    std::vector<double> b((size_t)L.n_act * nc, 0.0);
    // volume: h^d sum_q w_q f(x_q) phi_i(x_q), (p+1)^d Gauss points
    const int nq = nc;
    const long long chunk = 1 << 16;
    std::vector<double> X, F;
    for (long long c0 = 0; c0 < L.n_act; c0 += chunk) {
        long long c1 = std::min<long long>(L.n_act, c0 + chunk);
        long long np = (c1 - c0) * nq;
        X.resize((size_t)np * d);
        F.resize((size_t)np);
        for (long long K = c0; K < c1; ++K)
            for (int q = 0; q < nq; ++q) {
                int qq[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
                for (int c = 0; c < d; ++c)
                    X[((K - c0) * nq + q) * d + c] = L.lo + h * (L.cells[K * d + c] + r.gq[qq[c]]);
            }
        f(X.data(), np, F.data(), user);
        for (long long K = c0; K < c1; ++K)
            for (int i = 0; i < nc; ++i) {
                int ii[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
                double acc = 0.0;
                for (int q = 0; q < nq; ++q) {
                    int qq[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
                    double w = 1.0;
                    for (int c = 0; c < d; ++c) w *= r.wq[qq[c]] * r.S[qq[c]][ii[c]];
                    acc += w * F[(K - c0) * nq + q];
                }
                b[K * nc + i] = std::pow(h, d) * acc;
            }
    }
    // surrogate faces: h^(d-2) sum_q w_q [-alpha dn phi_i + sigma phi_i] g(x~ + d)
    if (L.n_surr) {
        long long np = (long long)L.n_surr * nf;
        X.resize((size_t)np * d);
        F.resize((size_t)np);
        for (int fc = 0; fc < L.n_surr; ++fc) {
            int K = L.surr_cell[fc], k = L.surr_k[fc], s = L.surr_s[fc];
            int tang[2], nt = 0;
            for (int c = 0; c < d; ++c)
                if (c != k) tang[nt++] = c;
            for (int q = 0; q < nf; ++q) {
                int qq[2] = {q % n1, q / n1};
                double x[3];
                x[k] = L.lo + h * (L.cells[K * d + k] + s);
                for (int t = 0; t < nt; ++t) x[tang[t]] = L.lo + h * (L.cells[K * d + tang[t]] + r.gq[qq[t]]);
                for (int c = 0; c < d; ++c) X[((size_t)fc * nf + q) * d + c] = x[c] + L.shifts[((size_t)fc * nf + q) * d + c];
            }
        }
        g(X.data(), np, F.data(), user);
        double sc = std::pow(h, d - 2);
        for (int fc = 0; fc < L.n_surr; ++fc) {
            int K = L.surr_cell[fc], k = L.surr_k[fc], s = L.surr_s[fc];
            double sg = s == 1 ? 1.0 : -1.0;
            int tang[2], nt = 0;
            for (int c = 0; c < d; ++c)
                if (c != k) tang[nt++] = c;
            for (int i = 0; i < nc; ++i) {
                int ii[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
                double coef = -alpha * sg * r.g[s][ii[k]] + L.sigG * r.e[s][ii[k]];
                if (coef == 0.0) continue;
                double acc = 0.0;
                for (int q = 0; q < nf; ++q) {
                    int qq[2] = {q % n1, q / n1};
                    double w = 1.0;
                    for (int t = 0; t < nt; ++t) w *= r.wq[qq[t]] * r.S[qq[t]][ii[tang[t]]];
                    acc += w * F[(size_t)fc * nf + q];
                }
                b[(size_t)K * nc + i] += sc * coef * acc;
            }
        }
    }
    hipSetDevice(pb->opt.device);
    HIPCHK(hipMemcpyAsync(b_dev, b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice, pb->stream));
    HIPCHK(hipStreamSynchronize(pb->stream));
    return SBM_OK;
}

// (host containers throw std::bad_alloc; nothing may leave through the C ABI)
int sbm_rhs(sbm_problem *pb, sbm_field_fn f, sbm_field_fn g, void *user, double *b_dev) {
    try {
        return rhs_body(pb, f, g, user, b_dev);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

int sbm_apply(sbm_problem *pb, const void *x, void *y, int fp32) {
    if (!pb || pb->host_only || !x || !y || x == y) return SBM_EINVAL;
    int l = (int)pb->levels.size() - 1;
    return fp32 ? level_apply<float>(pb, l, OP_APPLY, (const float *)x, (float *)y, nullptr)
                : level_apply<double>(pb, l, OP_APPLY, (const double *)x, (double *)y, nullptr);
}

int sbm_level_apply(sbm_problem *pb, int level, const void *x, void *y, int fp32) {
    if (!pb || pb->host_only || !x || !y || x == y) return SBM_EINVAL;
    int rc = check_level(pb, level);
    if (rc) return rc;
    return fp32 ? level_apply<float>(pb, level, OP_APPLY, (const float *)x, (float *)y, nullptr)
                : level_apply<double>(pb, level, OP_APPLY, (const double *)x, (double *)y, nullptr);
}

int sbm_colour_update(sbm_problem *pb, int level, int colour, const void *b, void *z, int fp32) {
    if (!pb || pb->host_only || !b || !z || b == z || (colour != 0 && colour != 1)) return SBM_EINVAL;
    int rc = check_level(pb, level);
    if (rc) return rc;
    return fp32 ? colour_update<float>(pb, level, colour, (const float *)b, (float *)z)
                : colour_update<double>(pb, level, colour, (const double *)b, (double *)z);
}

int sbm_restrict(sbm_problem *pb, int level, const void *r, void *bc, int fp32) {
    if (!pb || pb->host_only || !r || !bc) return SBM_EINVAL;
    int rc = check_level(pb, level);
    if (rc) return rc;
    if (level == 0) return SBM_EINVAL;
    return fp32 ? restrict_to<float>(pb, level, (const float *)r, (float *)bc)
                : restrict_to<double>(pb, level, (const double *)r, (double *)bc);
}

int sbm_prolong_add(sbm_problem *pb, int level, const void *zc, void *zf, int fp32) {
    if (!pb || pb->host_only || !zc || !zf) return SBM_EINVAL;
    int rc = check_level(pb, level);
    if (rc) return rc;
    if (level == 0) return SBM_EINVAL;
    return fp32 ? prolong_add<float>(pb, level, (const float *)zc, (float *)zf)
                : prolong_add<double>(pb, level, (const double *)zc, (double *)zf);
}

int sbm_vcycle(sbm_problem *pb, const void *r, void *z, int fp32) {
    if (!pb || pb->host_only || !r || !z || r == z) return SBM_EINVAL;
    int l = (int)pb->levels.size() - 1;
    return fp32 ? vcycle_rec<float>(pb, l, (const float *)r, (float *)z)
                : vcycle_rec<double>(pb, l, (const double *)r, (double *)z);
}

static int set_shifts_body(sbm_problem *pb, int level, const double *shifts, long long count) {
    if (!pb || !shifts) return SBM_EINVAL;
    const int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    HostLevel &L = pb->levels[level];
    if (count != (long long)L.shifts.size()) {
        pb->last_error = "sbm_set_shifts: expected " + std::to_string(L.shifts.size()) + " values";
        return SBM_EINVAL;
    }
    for (long long i = 0; i < count; ++i)
        if (!std::isfinite(shifts[i])) {
            pb->last_error = "sbm_set_shifts: non-finite shift";
            return SBM_EINVAL;
        }
    std::vector<double> keep(L.shifts);
    std::copy(shifts, shifts + count, L.shifts.begin());
    std::string err;
    int rc = build_blocks(L, pb->opt, err);
    if (rc) {
        // leave the problem as it was
        L.shifts.swap(keep);
        std::string e2;
        build_blocks(L, pb->opt, e2);
        pb->last_error = "sbm_set_shifts: " + err;
        return rc;
    }
    std::vector<double> Ainv;
    if (level == 0) {
        coarse_matrix(L, pb->opt.alpha, pb->opt.ext, pb->A0);
        Ainv = pb->A0;
        if (!invert(Ainv.data(), pb->coarse.n, 1e-14, 0.0)) {
            pb->last_error = "sbm_set_shifts: singular coarsest-level matrix";
            return SBM_ESINGULAR;
        }
    }
    if (!pb->host_only) {
        HIPCHK(hipSetDevice(pb->opt.device));
        HIPCHK(hipStreamSynchronize(pb->stream));
        if ((rc = refresh_level<double>(pb, level, pb->dev64[level])) ||
            (rc = refresh_level<float>(pb, level, pb->dev32[level])))
            return rc;
        if (level == 0)
            HIPCHK(hipMemcpy(pb->coarse.Ainv64, Ainv.data(), Ainv.size() * sizeof(double), hipMemcpyHostToDevice));
        if (level > 0) std::vector<double>().swap(L.Dbnd);  // only the coarsest keeps D
    }
    return SBM_OK;
}

int sbm_set_shifts(sbm_problem *pb, int level, const double *shifts, long long count) {
    try {
        return set_shifts_body(pb, level, shifts, count);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

int sbm_cell_block(const sbm_problem *pb, int level, int cell, int inverse, double *out) {
    if (!pb || !out) return SBM_EINVAL;
    int nl = (int)pb->levels.size();
    if (level == -1) level = nl - 1;
    if (level < 0 || level >= nl) return SBM_EINVAL;
    const HostLevel &L = pb->levels[level];
    if (cell < 0 || cell >= L.n_act) return SBM_EINVAL;
    const size_t nn = (size_t)L.nc * L.nc;
    int b = L.bnd_of[cell];
    if (inverse) {
        const double *src = b < 0 ? L.Bint.data() : &L.Bbnd[(size_t)b * nn];
        std::memcpy(out, src, nn * sizeof(double));
    } else if (b < 0) {
        std::memcpy(out, L.Dint.data(), nn * sizeof(double));
    } else {
        cell_block(L, pb->opt.alpha, pb->opt.ext, cell, out);
    }
    return SBM_OK;
}

int sbm_set_vcycle_fp32(sbm_problem *pb, int fp32) {
    if (!pb || (fp32 != 0 && fp32 != 1)) return SBM_EINVAL;
    pb->opt.vcycle_fp32 = fp32;
    return SBM_OK;
}

int sbm_coarse_matrix(const sbm_problem *pb, double *out, long long cap) {
    if (!pb || !out || cap < (long long)pb->A0.size()) return SBM_EINVAL;
    std::memcpy(out, pb->A0.data(), pb->A0.size() * sizeof(double));
    return SBM_OK;
}

int sbm_sync(sbm_problem *pb) {
    if (!pb) return SBM_EINVAL;
    HIPCHK(hipStreamSynchronize(pb->stream));
    return SBM_OK;
}

// FGMRES workspace: the Krylov bases V ((m+1) x n) and Z (m x n), the work
// vector w (n), two partial-sum buffers (2 gs_partials_max) and 128 doubles
// of device scalars.  None of it needs to start at zero: every entry is
// written before it is read.
struct SolveWork {
    double *V = nullptr, *Z = nullptr, *w = nullptr, *red = nullptr, *hdev = nullptr;
};

static constexpr int MAX_RESTART = SBM_MAX_RESTART;
// offsets into the device scalars (and the pinned staging buffer)
static constexpr int HD_P1 = 0;                         // pass-1 sums: V^T w, then |w|^2
static constexpr int HD_P2 = MAX_RESTART + 1;           // pass-2 sums
static constexpr int HD_P3 = 2 * (MAX_RESTART + 1);     // explicit norm pass / true residual
static constexpr int HD_Y = 3 * (MAX_RESTART + 1);      // least-squares coefficients
static constexpr int HD_BETA = 4 * (MAX_RESTART + 1);   // beta^2
static_assert(HD_BETA + 1 == sbm::SOLVE_SCALARS, "device scalar layout");

// One Gram-Schmidt launch sums at most GS_CHUNK basis vectors (plus the norm
// slot).  Longer bases run chunk by chunk through the same launches; bases of
// up to GS_CHUNK vectors take the single launches, so restarts up to 31 keep
// their arithmetic.
static constexpr int GS_CHUNK = 31;

// out[i] = V_i . w (i < nv), out[nv] = w . w.  Each chunk's reduction also
// writes its norm slot, which the next chunk's first sum overwrites.
static int gs_project(sbm_problem *pb, long long n, int nv, const double *V, const double *w, double *part,
                      double *out, hipStream_t s) {
    for (int c0 = 0; c0 < nv; c0 += GS_CHUNK) {
        const int mc = std::min(GS_CHUNK, nv - c0);
        KCHK(launch_gs_dots(n, mc, V + (size_t)c0 * n, w, part, s));
        KCHK(launch_gs_reduce(n, mc + 1, part, out + c0, s));
    }
    return SBM_OK;
}

// w -= sum_{i < nv} h[i] V_i, in place
static int gs_subtract(sbm_problem *pb, long long n, int nv, const double *V, const double *h, double *w,
                       hipStream_t s) {
    for (int c0 = 0; c0 < nv; c0 += GS_CHUNK)
        KCHK(launch_multiaxpy(n, std::min(GS_CHUNK, nv - c0), -1.0, h + c0, V + (size_t)c0 * n, w, s));
    return SBM_OK;
}

// v = (w - sum_{i < nv} h[i] V_i) * inv; the leading chunks of a long basis
// are subtracted from w in place first
static int gs_subtract_scale(sbm_problem *pb, long long n, int nv, const double *V, const double *h, double inv,
                             double *w, double *v, hipStream_t s) {
    const int last = (nv - 1) / GS_CHUNK * GS_CHUNK;
    int rc;
    if (last > 0 && (rc = gs_subtract(pb, n, last, V, h, w, s))) return rc;
    KCHK(launch_gs_axpy_scale(n, nv - last, V + (size_t)last * n, h + last, inv, w, v, s));
    return SBM_OK;
}

static int solve_body(sbm_problem *pb, const double *b, double *x, double tol, int m, int max_iter, sbm_stats *st,
                      const SolveWork &ws) {
    if (!pb || pb->host_only || !b || !x || b == x || m < 1 || m > MAX_RESTART || max_iter < 1 || !(tol > 0) ||
        !pb->pinned || pb->arnoldi.size() < sbm::ARNOLDI_DOUBLES)
        return SBM_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    const HostLevel &L = pb->levels.back();
    const long long n = (long long)L.n_act * L.nc;
    const int lf = (int)pb->levels.size() - 1;
    hipStream_t s = pb->stream;
    int rc;
    double *V = ws.V, *Z = ws.Z, *w = ws.w, *hd = ws.hdev, *hp = pb->pinned;
    // two partial-sum buffers: the passes of one Arnoldi step alternate between them
    double *pa = ws.red, *pq = ws.red + sbm::gs_partials_max();
    const bool f32 = pb->opt.vcycle_fp32 != 0;
    // ||b||
    KCHK(launch_gs_dots(n, 0, nullptr, b, pa, s));
    KCHK(launch_gs_reduce(n, 1, pa, hd, s));
    HIPCHK(hipMemcpyAsync(hp, hd, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double nb = std::sqrt(hp[0]);
    KCHK(launch_fill<double>(n, x, 0.0, s));
    sbm_stats local{0, 0, 0.0, 0.0};
    if (!std::isfinite(nb)) return SBM_ENONFINITE;
    if (nb == 0.0) {
        local.converged = 1;
        if (st) *st = local;
        HIPCHK(hipStreamSynchronize(s));
        return SBM_OK;
    }
    // Hessenberg matrix (row stride m), Givens rotations, the reduced
    // right-hand side and the coefficients in the problem's own storage, sized
    // for MAX_RESTART at setup: the solve allocates nothing on the host
    double *H = pb->arnoldi.data();
    double *cs = H + (size_t)(MAX_RESTART + 1) * MAX_RESTART, *sn = cs + MAX_RESTART, *gv = sn + MAX_RESTART,
           *y = gv + MAX_RESTART + 1;
    // r = b (x0 = 0); v0 = r / ||r||
    HIPCHK(hipMemcpyAsync(w, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double beta = nb;
    int its = 0;
    double rel = 1.0;
    int status = SBM_NOT_CONVERGED;
    for (;;) {
        hp[HD_BETA] = beta * beta;
        HIPCHK(hipMemcpyAsync(hd + HD_BETA, hp + HD_BETA, sizeof(double), hipMemcpyHostToDevice, s));
        KCHK(launch_scale(n, hd + HD_BETA, w, V, s));
        std::fill(H, H + (size_t)(m + 1) * m, 0.0);
        std::fill(gv, gv + m + 1, 0.0);
        gv[0] = beta;
        int j = 0;
        bool est_ok = false;
        while (j < m && its < max_iter) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            if (f32) {
                // the cycle reads v_j in FP64 and keeps its own FP32 copy; its
                // last smoothing kernels write z_j in FP64
                EmitArgs<float> e64{};
                e64.kind = EMIT_F64;
                e64.z64 = zj;
                bool done = false;
                if ((rc = vcycle_rec<float>(pb, lf, pb->f32_in, pb->f32_out, vj, false,
                                            pb->opt.fuse_transfers ? &e64 : nullptr, &done)))
                    return rc;
                if (!done) KCHK(launch_cast_f2d(n, pb->f32_out, zj, s));
            } else {
                if ((rc = vcycle_rec<double>(pb, lf, vj, zj))) return rc;
            }
            if ((rc = level_apply<double>(pb, lf, OP_APPLY, zj, w, nullptr))) return rc;
            // Classical Gram-Schmidt with a selective second pass (the
            // reorthogonalisation test of Daniel, Gragg, Kaufman and Stewart,
            // with a looser threshold eta).  Pass 1 forms h1 = V^T w and |w|^2 in
            // one sweep.  When the projection keeps |w'|^2 = |w|^2 - |h1|^2 >=
            // eta^2 |w|^2, the computed w' = w - V h1 is orthogonal to V up to
            // a loss of order eps |w| / |w'| <= eps / eta, and that identity
            // gives its norm to about eps / eta^2: the subtraction is fused with
            // the normalisation and the step ends after two sweeps over V.
            // Otherwise the second pass runs: it subtracts h1 and forms
            // h2 = V^T w' with |w'|^2 in the same sweep; the pass-2 subtraction
            // is fused with the normalisation, the norm following from
            // |w''|^2 = |w'|^2 - |h2|^2 (w'' orthogonal to V), or, when h2 is
            // not small against w' and that identity loses digits, from an
            // explicit measurement of w''.  (In the preconditioned iterations
            // measured here |w'| / |w| stays within 0.17-0.43 and the second
            // pass changes w' by about 1e-15 of its norm.)
            // At tight tolerances (below 1e-10) the norm identity delays the
            // Arnoldi residual estimate (measured on the paper's 2D disk at
            // 1e-12: 33 iterations against 18 with the norm measured), so
            // there every step takes the second pass and measures |w''|.
            // The one-pass step's loss of orthogonality compounds along the
            // basis: classical Gram-Schmidt loses about eps kappa^2 (Giraud,
            // Langou and Rozloznik, 2005), and the condition of the Arnoldi
            // basis grows like the residual reduction R = beta / |g_j| within
            // the cycle (Greenbaum, Rozloznik and Strakos, 1997).  On a weakly
            // preconditioned 2D disk (FGMRES(100)) one pass throughout drifts
            // 1.4e-6 from orthogonal by vector 40 and 0.16 by vector 80 (R =
            // 3e4, 2e7), and the residual estimate stalls: 100 iterations
            // against 87.  The estimate stays sound while eps R^2 < 1e-3 / R,
            // so beyond the 30th vector one pass is kept only for R < (1e-3 /
            // eps)^(1/3) = 1.6e4 (87 iterations there; basis loss 4e-7).
            // Bases of up to 30 vectors keep the one-pass test alone.
            constexpr double eta = 0.1;
            constexpr int one_pass_max = 30;
            constexpr double one_pass_reduction = 1.6e4;
            const bool norm_identity = tol >= 1e-10;
            const int nv = j + 1;
            double *vnext = V + (size_t)(j + 1) * n;
            if ((rc = gs_project(pb, n, nv, V, w, pa, hd + HD_P1, s))) return rc;
            HIPCHK(hipMemcpyAsync(hp, hd, (size_t)(nv + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            double h1sq = 0.0;
            for (int i = 0; i <= j; ++i) h1sq += hp[i] * hp[i];
            const double wsq = hp[nv];
            if (!std::isfinite(wsq) || !std::isfinite(h1sq)) return SBM_ENONFINITE;
            double hn;
            const bool one_pass_ok = nv <= one_pass_max || one_pass_reduction * std::fabs(gv[j]) > beta;
            if (norm_identity && one_pass_ok && wsq - h1sq >= eta * eta * wsq) {
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hp[i];
                hn = std::sqrt(wsq - h1sq);
                if ((rc = gs_subtract_scale(pb, n, nv, V, hd + HD_P1, hn > 0.0 ? 1.0 / hn : 1.0, w, vnext, s)))
                    return rc;
            } else {
                if (nv <= GS_CHUNK) {
                    KCHK(launch_gs_axpy_dots(n, nv, V, pa, hd + HD_P1, w, pq, s));
                    KCHK(launch_gs_reduce(n, nv + 1, pq, hd + HD_P2, s));
                } else if ((rc = gs_subtract(pb, n, nv, V, hd + HD_P1, w, s)) ||
                           (rc = gs_project(pb, n, nv, V, w, pq, hd + HD_P2, s))) {
                    return rc;
                }
                HIPCHK(hipMemcpyAsync(hp + HD_P2, hd + HD_P2, (size_t)(nv + 1) * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hp[i] + hp[HD_P2 + i];
                double h2sq = 0.0;
                for (int i = 0; i <= j; ++i) h2sq += hp[HD_P2 + i] * hp[HD_P2 + i];
                const double w1sq = hp[HD_P2 + nv];
                if (!std::isfinite(w1sq) || !std::isfinite(h2sq)) return SBM_ENONFINITE;
                if (h2sq <= 0.5 * w1sq) {
                    hn = std::sqrt(w1sq - h2sq);
                    if ((rc = gs_subtract_scale(pb, n, nv, V, hd + HD_P2, hn > 0.0 ? 1.0 / hn : 1.0, w, vnext,
                                                s)))
                        return rc;
                } else {
                    if (nv <= GS_CHUNK) {
                        KCHK(launch_gs_axpy_dots(n, nv, V, pq, hd + HD_P3, w, pa, s));
                        KCHK(launch_gs_reduce(n, nv + 1, pa, hd + HD_P3, s));
                    } else if ((rc = gs_subtract(pb, n, nv, V, hd + HD_P2, w, s)) ||
                               (rc = gs_project(pb, n, nv, V, w, pa, hd + HD_P3, s))) {
                        return rc;
                    }
                    HIPCHK(hipMemcpyAsync(hp + HD_P3, hd + HD_P3 + nv, sizeof(double), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    hn = std::sqrt(hp[HD_P3]);
                    if (!std::isfinite(hn)) return SBM_ENONFINITE;
                    KCHK(launch_scale(n, hd + HD_P3 + nv, w, vnext, s));
                }
            }
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double den = std::hypot(a, bb);
            cs[j] = den > 0 ? a / den : 1.0;
            sn[j] = den > 0 ? bb / den : 0.0;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++j;
            ++its;
            if (std::fabs(gv[j]) / nb <= tol) {
                est_ok = true;
                break;
            }
        }
        // y = R^{-1} g ; x += Z y
        for (int i = j - 1; i >= 0; --i) {
            double acc = gv[i];
            for (int k2 = i + 1; k2 < j; ++k2) acc -= H[(size_t)i * m + k2] * y[k2];
            y[i] = acc / H[(size_t)i * m + i];
        }
        for (int i = 0; i < j; ++i) hp[HD_Y + i] = y[i];
        HIPCHK(hipMemcpyAsync(hd + HD_Y, hp + HD_Y, j * sizeof(double), hipMemcpyHostToDevice, s));
        for (int c0 = 0; c0 < j; c0 += GS_CHUNK)
            KCHK(launch_multiaxpy(n, std::min(GS_CHUNK, j - c0), 1.0, hd + HD_Y + c0, Z + (size_t)c0 * n, x, s));
        // true residual
        if ((rc = level_apply<double>(pb, lf, OP_RESID, x, w, b))) return rc;
        KCHK(launch_gs_dots(n, 0, nullptr, w, pa, s));
        KCHK(launch_gs_reduce(n, 1, pa, hd + HD_P3, s));
        HIPCHK(hipMemcpyAsync(hp, hd + HD_P3, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        beta = std::sqrt(hp[0]);
        if (!std::isfinite(beta)) return SBM_ENONFINITE;
        rel = beta / nb;
        (void)est_ok;
        if (rel <= tol) {
            status = SBM_OK;
            break;
        }
        if (its >= max_iter) break;
    }
    local.iterations = its;
    local.converged = status == SBM_OK;
    local.rel_residual_true = rel;
    local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = local;
    return status;
}

// (host containers throw std::bad_alloc; nothing may leave through the C ABI)
int sbm_solve(sbm_problem *pb, const double *b, double *x, double tol, int m, int max_iter, sbm_stats *st) {
    try {
        if (!pb || pb->host_only) return SBM_EINVAL;
        if (m < 1 || m > MAX_RESTART) {
            pb->last_error = "restart length " + std::to_string(m) + " outside 1.." + std::to_string(MAX_RESTART);
            return SBM_EINVAL;
        }
        const HostLevel &L = pb->levels.back();
        const long long n = (long long)L.n_act * L.nc;
        int rc;
        if (pb->ws_restart < m) {
            if ((rc = dalloc(pb, &pb->V, (size_t)(m + 1) * n)) || (rc = dalloc(pb, &pb->Z, (size_t)m * n)) ||
                (rc = dalloc(pb, &pb->w, (size_t)n)) ||
                (rc = dalloc(pb, &pb->red, (size_t)2 * sbm::gs_partials_max())) ||
                (rc = dalloc(pb, &pb->hdev, (size_t)sbm::SOLVE_SCALARS)))
                return rc;
            pb->ws_restart = m;
        }
        SolveWork ws;
        ws.V = pb->V;
        ws.Z = pb->Z;
        ws.w = pb->w;
        ws.red = pb->red;
        ws.hdev = pb->hdev;
        return solve_body(pb, b, x, tol, m, max_iter, st, ws);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solve.  The FGMRES workspace lives in one file-scope device
// array of SBM_NOALLOC_SCRATCH_BYTES, which every GPU the library runs on
// holds from the module's load until the process ends.  In host code the
// array's name only stands for the device symbol: its device address is
// looked up once per device (with that device current) and kept, and only
// that address ever reaches a kernel or a copy.
static __device__ __align__(256) double scratch[SBM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

static constexpr int MAX_DEVICES = 64;
static double *scratch_dev[MAX_DEVICES];
static std::mutex scratch_mutex;

static int scratch_address(sbm_problem *pb, double **out) {
    const int dev = pb->opt.device;
    if (dev < 0 || dev >= MAX_DEVICES) {
        pb->last_error = "device ordinal out of range for the allocation-free solve";
        return SBM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_dev[dev] == nullptr) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || (cur != dev && hipSetDevice(dev) != hipSuccess)) return SBM_EDEVICE;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) {
            pb->last_error = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return SBM_EDEVICE;
        }
        scratch_dev[dev] = (double *)p;
    }
    *out = scratch_dev[dev];
    return SBM_OK;
}

extern "C" {

long long sbm_solve_noalloc_doubles(const sbm_problem *pb, int m) {
    if (!pb || pb->host_only || m < 1 || m > MAX_RESTART) return -1;
    const HostLevel &L = pb->levels.back();
    const long long n = (long long)L.n_act * L.nc;
    auto up = [](long long k) { return (k + 31) / 32 * 32; };   // 256-byte sections
    return up((long long)(m + 1) * n) + up((long long)m * n) + up(n) + up(2LL * sbm::gs_partials_max()) +
           up(sbm::SOLVE_SCALARS);
}

int sbm_solve_noalloc(sbm_problem *pb, const double *b, double *x, double tol, int m, int max_iter, sbm_stats *st) {
    try {
        if (!pb || pb->host_only) return SBM_EINVAL;
        if (m < 1 || m > MAX_RESTART) {
            pb->last_error = "restart length " + std::to_string(m) + " outside 1.." + std::to_string(MAX_RESTART);
            return SBM_EINVAL;
        }
        const long long need = sbm_solve_noalloc_doubles(pb, m);
        const long long cap = (long long)(SBM_NOALLOC_SCRATCH_BYTES / sizeof(double));
        if (need > cap) {
            pb->last_error = "allocation-free solve: the FGMRES(" + std::to_string(m) + ") workspace needs " +
                             std::to_string(need * 8) + " bytes, the scratch array holds " +
                             std::to_string(cap * 8) + " (fewer DoFs or a shorter restart)";
            return SBM_EINVAL;
        }
        double *base = nullptr;
        int rc;
        if ((rc = scratch_address(pb, &base))) return rc;
        const HostLevel &L = pb->levels.back();
        const long long n = (long long)L.n_act * L.nc;
        auto up = [](long long k) { return (k + 31) / 32 * 32; };
        SolveWork ws;
        ws.V = base;
        ws.Z = ws.V + up((long long)(m + 1) * n);
        ws.w = ws.Z + up((long long)m * n);
        ws.red = ws.w + up(n);
        ws.hdev = ws.red + up(2LL * sbm::gs_partials_max());
        return solve_body(pb, b, x, tol, m, max_iter, st, ws);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

}  // extern "C"
