// C ABI of the learned boundary-cell correction (features, training kernels,
// BF16 inference and installation into the smoother).  See mlp.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

using namespace sbm;

namespace {

template <typename T>
int lalloc(sbm_problem *pb, T **p, size_t n) {
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

// Per boundary cell of the finest level, per face (k, s) in order: surrogate
// mask, mean / min / max of d . n~ / h, mean d / h, mean unit normal of Gamma at
// the projections (recovered as -sign(phi(x~)) d / |d|: the segment from x~ to
// its closest point is normal to Gamma).
void features(const sbm_problem *pb, std::vector<double> &F) {
    const HostLevel &L = pb->levels.back();
    const int d = L.d, nf = L.nf, n1 = L.n1, fd = feature_dim(d);
    F.assign((size_t)L.n_bnd * fd, 0.0);
    for (int b = 0; b < L.n_bnd; ++b) {
        int K = L.bnd_cells[b];
        double *o = &F[(size_t)b * fd];
        for (int f = 0; f < 2 * d; ++f) {
            double *of = o + f * (4 + 2 * d);
            int nb = L.nbr[(size_t)K * 2 * d + f];
            if (nb >= 0) continue;
            int rec = -nb - 1, k = f / 2, s = f % 2;
            double sg = s == 1 ? 1.0 : -1.0;
            int tang[2], nt = 0;
            for (int c = 0; c < d; ++c)
                if (c != k) tang[nt++] = c;
            double mean = 0, mn = 1e300, mx = -1e300, md[3] = {0, 0, 0}, nrm[3] = {0, 0, 0};
            for (int q = 0; q < nf; ++q) {
                const double *dq = &L.shifts[((size_t)rec * nf + q) * d];
                double dn = dq[k] * sg / L.h;
                mean += dn;
                mn = std::fmin(mn, dn);
                mx = std::fmax(mx, dn);
                double x[3], len = 0;
                int qq[2] = {q % n1, q / n1};
                x[k] = L.lo + L.h * (L.cells[(size_t)K * d + k] + s);
                for (int t = 0; t < nt; ++t) x[tang[t]] = L.lo + L.h * (L.cells[(size_t)K * d + tang[t]] + L.ref.gq[qq[t]]);
                for (int c = 0; c < d; ++c) {
                    md[c] += dq[c] / L.h;
                    len += dq[c] * dq[c];
                }
                len = std::sqrt(len);
                double ph = pb->geom.phi(x);
                double sgn = ph > 0 ? -1.0 : (ph < 0 ? 1.0 : 0.0);
                if (len > 0)
                    for (int c = 0; c < d; ++c) nrm[c] += sgn * dq[c] / len;
            }
            of[0] = 1.0;
            of[1] = mean / nf;
            of[2] = mn;
            of[3] = mx;
            for (int c = 0; c < d; ++c) {
                of[4 + c] = md[c] / nf;
                of[4 + d + c] = nrm[c] / nf;
            }
        }
    }
}

// One block per finest-level boundary cell K: R = r_K, BR = B_K r_K,
// E = x*_K - z_K, all three scaled by 1 / |E| (the loss is invariant to a
// per-sample scale); valid = 0 (and the rows zero) when |E| = 0 or any entry
// is not finite.
__global__ __launch_bounds__(64) void collect_pairs_kernel(int nc, const int *__restrict__ bnd_cells,
                                                           const double *__restrict__ Bt, const double *__restrict__ r,
                                                           const double *__restrict__ xs,
                                                           const double *__restrict__ z, double *__restrict__ R,
                                                           double *__restrict__ BR, double *__restrict__ E,
                                                           int *__restrict__ valid) {
    __shared__ double rs[64], e2[64];
    __shared__ int ok;
    const int b = blockIdx.x, i = threadIdx.x;
    const int K = bnd_cells[b];
    double ri = 0, ei = 0;
    if (i < nc) {
        ri = r[(size_t)K * nc + i];
        ei = xs[(size_t)K * nc + i] - z[(size_t)K * nc + i];
    }
    rs[i] = ri;
    e2[i] = ei * ei;
    if (i == 0) ok = 1;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        if (i < off) e2[i] += e2[i + off];
        __syncthreads();
    }
    double acc = 0;
    if (i < nc) {
        const double *B = Bt + (size_t)b * nc * nc;
        for (int j = 0; j < nc; ++j) acc += B[(size_t)j * nc + i] * rs[j];
    }
    const double n2 = e2[0];
    if (!std::isfinite(ri) || !std::isfinite(acc) || !std::isfinite(ei) || !(n2 > 0) || !std::isfinite(n2)) ok = 0;
    __syncthreads();
    const double sc = ok ? 1.0 / std::sqrt(n2) : 0.0;
    if (i < nc) {
        R[(size_t)b * nc + i] = ri * sc;
        BR[(size_t)b * nc + i] = acc * sc;
        E[(size_t)b * nc + i] = ei * sc;
    }
    if (i == 0) valid[b] = ok;
}

__global__ void axpy_kernel(long long n, const double *__restrict__ t, double *__restrict__ z) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) z[i] += t[i];
}

int pair_vectors(sbm_problem *pb) {
    if (pb->pair_r) return SBM_OK;
    const HostLevel &L = pb->levels.back();
    const size_t n = (size_t)L.n_act * L.nc;
    int rc;
    if ((rc = lalloc(pb, &pb->pair_r, n)) || (rc = lalloc(pb, &pb->pair_t, n))) return rc;
    return SBM_OK;
}

}  // namespace

extern "C" {

int sbm_collect_pairs(sbm_problem *pb, const double *x_star, const double *b, const double *z, double *R, double *BR,
                      double *E, int *valid) {
    if (!pb || pb->host_only || !x_star || !b || !z || !R || !BR || !E || !valid) return SBM_EINVAL;
    int rc;
    if ((rc = pair_vectors(pb))) return rc;
    if ((rc = finest_residual(pb, z, b, pb->pair_r))) return rc;
    auto &D = pb->dev64.back();
    if (D.n_bnd == 0) return SBM_OK;
    if (D.nc > 64) return SBM_EINVAL;
    hipLaunchKernelGGL(collect_pairs_kernel, dim3(D.n_bnd), dim3(64), 0, pb->stream, D.nc, D.bnd_cells, D.Bbnd_t,
                       pb->pair_r, x_star, z, R, BR, E, valid);
    if (hipGetLastError() != hipSuccess) {
        pb->last_error = "collect_pairs launch failed";
        return SBM_EDEVICE;
    }
    return SBM_OK;
}

int sbm_richardson(sbm_problem *pb, const double *b, double *z, int steps) {
    if (!pb || pb->host_only || !b || !z || b == z || steps < 0) return SBM_EINVAL;
    int rc;
    if ((rc = pair_vectors(pb))) return rc;
    const HostLevel &L = pb->levels.back();
    const long long n = (long long)L.n_act * L.nc;
    for (int s = 0; s < steps; ++s) {
        if ((rc = finest_residual(pb, z, b, pb->pair_r))) return rc;
        if ((rc = sbm_vcycle(pb, pb->pair_r, pb->pair_t, 0))) return rc;
        const int nbk = (int)std::min<long long>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(axpy_kernel, dim3(nbk), dim3(256), 0, pb->stream, n, pb->pair_t, z);
        if (hipGetLastError() != hipSuccess) {
            pb->last_error = "richardson update launch failed";
            return SBM_EDEVICE;
        }
    }
    return SBM_OK;
}

int sbm_feature_dim(int dim) { return (dim == 2 || dim == 3) ? feature_dim(dim) : SBM_EINVAL; }

int sbm_boundary_cells(const sbm_problem *pb, int *n_boundary, int *cells, long long cap) {
    if (!pb || !n_boundary) return SBM_EINVAL;
    const HostLevel &L = pb->levels.back();
    *n_boundary = L.n_bnd;
    if (cells) {
        if (cap < L.n_bnd) return SBM_EINVAL;
        std::memcpy(cells, L.bnd_cells.data(), sizeof(int) * L.n_bnd);
    }
    return SBM_OK;
}

static int boundary_features_body(const sbm_problem *pb, double *out, long long cap) {
    if (!pb || !out) return SBM_EINVAL;
    std::vector<double> F;
    features(pb, F);
    if (cap < (long long)F.size()) return SBM_EINVAL;
    std::memcpy(out, F.data(), F.size() * sizeof(double));
    return SBM_OK;
}

// (host containers throw std::bad_alloc; nothing may leave through the C ABI)
int sbm_boundary_features(const sbm_problem *pb, double *out, long long cap) {
    try {
        return boundary_features_body(pb, out, cap);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

int sbm_boundary_samples(sbm_problem *pb, const double *r, const double *e, double *R, double *BR, double *E) {
    if (!pb || pb->host_only || !r || !e || !R || !BR || !E) return SBM_EINVAL;
    auto &D = pb->dev64.back();
    if (launch_boundary_samples(D.n_bnd, D.nc, D.bnd_cells, D.Bbnd_t, r, e, R, BR, E, pb->stream)) {
        pb->last_error = "boundary_samples launch failed";
        return SBM_EDEVICE;
    }
    return SBM_OK;
}

static int set_learned_body(sbm_problem *pb, const float *params, int width) {
    if (!pb || pb->host_only) return SBM_EINVAL;
    if (!params) {
        pb->learned_on = false;
        return SBM_OK;
    }
    if (width != 64) return SBM_EINVAL;
    auto &D64 = pb->dev64.back();
    auto &D32 = pb->dev32.back();
    const int nb = D64.n_bnd, nc = D64.nc, n_in = feature_dim(D64.d), n_out = 1 + 8 * nc;
    if (nb == 0) {
        pb->learned_on = true;
        return SBM_OK;
    }
    int rc;
    if (!D64.lw) {
        if ((rc = lalloc(pb, &D64.lw, nb)) || (rc = lalloc(pb, &D64.lU, (size_t)nb * nc * 4)) ||
            (rc = lalloc(pb, &D64.lV, (size_t)nb * nc * 4)) || (rc = lalloc(pb, &D32.lw, nb)) ||
            (rc = lalloc(pb, &D32.lU, (size_t)nb * nc * 4)) || (rc = lalloc(pb, &D32.lV, (size_t)nb * nc * 4)))
            return rc;
    }
    if (!pb->lrn_X) {
        if ((rc = lalloc(pb, &pb->lrn_X, (size_t)nb * n_in)) || (rc = lalloc(pb, &pb->lrn_O, (size_t)nb * n_out)) ||
            (rc = lalloc(pb, &pb->lrn_wbuf, mlp_infer_wbuf_elems(n_out))))
            return rc;
    }
    std::vector<double> F;
    features(pb, F);
    std::vector<float> Ff(F.begin(), F.end());
    if (hipMemcpyAsync(pb->lrn_X, Ff.data(), Ff.size() * sizeof(float), hipMemcpyHostToDevice, pb->stream) !=
        hipSuccess)
        return SBM_EDEVICE;
    if (mlp_infer_bf16(n_in, width, n_out, nb, params, pb->lrn_X, pb->lrn_O, pb->lrn_wbuf, pb->stream) ||
        launch_head<double>(nb, nc, pb->lrn_O, D64.lw, D64.lU, D64.lV, pb->stream) ||
        launch_head<float>(nb, nc, pb->lrn_O, D32.lw, D32.lU, D32.lV, pb->stream)) {
        pb->last_error = "learned inference launch failed";
        return SBM_EDEVICE;
    }
    if (hipStreamSynchronize(pb->stream) != hipSuccess) return SBM_EDEVICE;
    pb->learned_nout = n_out;
    pb->learned_on = true;
    return SBM_OK;
}

// (host containers throw std::bad_alloc; nothing may leave through the C ABI)
int sbm_set_learned(sbm_problem *pb, const float *params, int width) {
    try {
        return set_learned_body(pb, params, width);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

static int set_learned_arrays_body(sbm_problem *pb, const double *w, const double *U, const double *V) {
    if (!pb || pb->host_only || !w || !U || !V) return SBM_EINVAL;
    auto &D64 = pb->dev64.back();
    auto &D32 = pb->dev32.back();
    const int nb = D64.n_bnd, nc = D64.nc;
    int rc;
    if (!D64.lw) {
        if ((rc = lalloc(pb, &D64.lw, nb)) || (rc = lalloc(pb, &D64.lU, (size_t)nb * nc * 4)) ||
            (rc = lalloc(pb, &D64.lV, (size_t)nb * nc * 4)) || (rc = lalloc(pb, &D32.lw, nb)) ||
            (rc = lalloc(pb, &D32.lU, (size_t)nb * nc * 4)) || (rc = lalloc(pb, &D32.lV, (size_t)nb * nc * 4)))
            return rc;
    }
    size_t n1 = nb, n4 = (size_t)nb * nc * 4;
    std::vector<float> wf(w, w + n1), Uf(U, U + n4), Vf(V, V + n4);
    if (hipMemcpy(D64.lw, w, n1 * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(D64.lU, U, n4 * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(D64.lV, V, n4 * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(D32.lw, wf.data(), n1 * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(D32.lU, Uf.data(), n4 * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(D32.lV, Vf.data(), n4 * 4, hipMemcpyHostToDevice) != hipSuccess)
        return SBM_EDEVICE;
    pb->learned_on = true;
    return SBM_OK;
}

// (host containers throw std::bad_alloc; nothing may leave through the C ABI)
int sbm_set_learned_arrays(sbm_problem *pb, const double *w, const double *U, const double *V) {
    try {
        return set_learned_arrays_body(pb, w, U, V);
    } catch (const std::bad_alloc &) {
        return SBM_ENOMEM;
    } catch (...) {
        return SBM_EINVAL;
    }
}

int sbm_use_learned(sbm_problem *pb, int on) {
    if (!pb || (on && !pb->dev64.empty() && !pb->dev64.back().lw && pb->dev64.back().n_bnd > 0)) return SBM_EINVAL;
    pb->learned_on = on != 0;
    return SBM_OK;
}

int sbm_mlp_forward(int fp64, int n_in, int width, int n_out, int batch, const void *params, const void *X, void *H1,
                    void *H2, void *O, void *stream) {
    if (n_in < 1 || width < 1 || n_out < 1 || batch < 1 || !params || !X || !H1 || !H2 || !O) return SBM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int rc = fp64 ? mlp_forward<double>(n_in, width, n_out, batch, (const double *)params, (const double *)X,
                                        (double *)H1, (double *)H2, (double *)O, st)
                  : mlp_forward<float>(n_in, width, n_out, batch, (const float *)params, (const float *)X,
                                       (float *)H1, (float *)H2, (float *)O, st);
    return rc ? SBM_EDEVICE : SBM_OK;
}

int sbm_mlp_loss_grad(int fp64, int batch, int n_cell, int train_uv, double omega, const void *O, const void *R,
                      const void *BR, const void *E, void *dO, void *loss_s, void *loss, void *stream) {
    if (batch < 1 || n_cell < 1 || n_cell > 64 || !O || !R || !BR || !E || !dO || !loss_s || !loss) return SBM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int rc = fp64 ? mlp_loss_grad<double>(batch, n_cell, train_uv, omega, (const double *)O, (const double *)R,
                                          (const double *)BR, (const double *)E, (double *)dO, (double *)loss_s,
                                          (double *)loss, st)
                  : mlp_loss_grad<float>(batch, n_cell, train_uv, omega, (const float *)O, (const float *)R, (const float *)BR,
                                         (const float *)E, (float *)dO, (float *)loss_s, (float *)loss, st);
    return rc ? SBM_EDEVICE : SBM_OK;
}

long long sbm_mlp_work_elems(int n_in, int width, int n_out, int batch) {
    long long a = 64LL * n_out * width, b = 64LL * width * width, c = 64LL * width * n_in;
    long long d = (long long)((batch + 511) / 512) * (n_out > width ? n_out : width);
    long long m = a;
    if (b > m) m = b;
    if (c > m) m = c;
    if (d > m) m = d;
    return m;
}

int sbm_mlp_backward(int fp64, int n_in, int width, int n_out, int batch, const void *params, const void *X,
                     const void *H1, const void *H2, const void *dO, void *grads, void *dH, void *work, void *stream) {
    if (n_in < 1 || width < 1 || n_out < 1 || batch < 1 || !params || !X || !H1 || !H2 || !dO || !grads || !dH ||
        !work)
        return SBM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int rc = fp64 ? mlp_backward<double>(n_in, width, n_out, batch, (const double *)params, (const double *)X,
                                         (const double *)H1, (const double *)H2, (const double *)dO, (double *)grads,
                                         (double *)dH, (double *)work, st)
                  : mlp_backward<float>(n_in, width, n_out, batch, (const float *)params, (const float *)X,
                                        (const float *)H1, (const float *)H2, (const float *)dO, (float *)grads,
                                        (float *)dH, (float *)work, st);
    return rc ? SBM_EDEVICE : SBM_OK;
}

int sbm_adam(int n, float *params, const float *grads, float *m, float *v, int t, float lr, float b1, float b2,
             float eps, void *stream) {
    if (n < 1 || t < 1 || !params || !grads || !m || !v) return SBM_EINVAL;
    return adam_step(n, params, grads, m, v, t, lr, b1, b2, eps, (hipStream_t)stream) ? SBM_EDEVICE : SBM_OK;
}

long long sbm_mlp_infer_wbuf_elems(int n_out) { return (long long)mlp_infer_wbuf_elems(n_out); }

int sbm_mlp_infer_bf16(int n_in, int width, int n_out, int batch, const float *params, const float *X, float *O,
                       short *wbuf, void *stream) {
    if (width != 64 || n_in < 1 || n_in > 64 || batch < 1 || !params || !X || !O || !wbuf) return SBM_EINVAL;
    return mlp_infer_bf16(n_in, width, n_out, batch, params, X, O, wbuf, (hipStream_t)stream) ? SBM_EDEVICE : SBM_OK;
}

}  // extern "C"
