// Learned boundary-cell smoother correction: training and inference kernels.
//
// Not part of the paper: the paper finds the cell-wise smoother weak for
// p = 3 in 3D (Sec. 5.3) and leaves better smoothers open (Sec. 6).  The
// correction keeps the successive cell-wise update of Sec. 3.1 and changes
// only the local solve of surrogate-boundary cells of the finest level,
//     z_K += omega * w_K * (B_K + U_K V_K^T) r_K,    w_K = 2 sigmoid(o_0),
// where (o_0, U_K, V_K) come from a 3-layer tanh MLP on per-cell shift
// features.  Training runs in FP32 (or FP64 for exact parity checks) with the
// tiled GEMM, loss and Adam kernels below; inference runs in BF16 on the
// matrix cores (v_mfma_f32_16x16x16_bf16) with FP32 accumulation.
#include <hip/hip_bf16.h>

#include "kernels.hpp"
#include "mlp.hpp"

namespace sbm {

// --------------------------------------------------------------------------
// C[m][n] (+)= sum_k opA(m,k) opB(k,n)  [+ bias[n]] [tanh]
//   opA(m,k) = TA ? A[k*lda + m] : A[m*lda + k]
//   opB(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// blockIdx.z splits the k range into chunks of kchunk; block z writes C + z*M*ldc.
constexpr int GT = 32;

template <typename T, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const T *__restrict__ A, int lda,
                                                   const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc,
                                                   const T *__restrict__ bias, int kchunk) {
    __shared__ T As[GT][GT + 1];
    __shared__ T Bs[GT][GT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    T acc[2][2] = {{0, 0}, {0, 0}};
    for (int k0 = kb; k0 < ke; k0 += GT) {
        for (int t = threadIdx.x; t < GT * GT; t += 256) {
            int r = t / GT, c = t % GT;
            // As[r = m][c = k]
            int m = m0 + r, k = k0 + c;
            As[r][c] = (m < M && k < ke) ? (TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]) : T(0);
            // Bs[r = k][c = n]
            int kk = k0 + r, n = n0 + c;
            Bs[r][c] = (kk < ke && n < N) ? (TB ? B[(size_t)n * ldb + kk] : B[(size_t)kk * ldb + n]) : T(0);
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < GT; ++k) {
            T a0 = As[ty * 2][k], a1 = As[ty * 2 + 1][k];
            T b0 = Bs[k][tx * 2], b1 = Bs[k][tx * 2 + 1];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    T *Cz = C + (size_t)blockIdx.z * M * ldc;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            int m = m0 + ty * 2 + i, n = n0 + tx * 2 + j;
            if (m >= M || n >= N) continue;
            T v = acc[i][j];
            if (EPI >= 1) v += bias[n];
            if (EPI == 2) v = tanh(v);
            Cz[(size_t)m * ldc + n] = v;
        }
}

// out[i] = sum_z part[z * n + i]  (fixed order)
template <typename T>
__global__ void sum_splits_kernel(long long n, int nz, const T *__restrict__ part, T *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = 0;
    for (int z = 0; z < nz; ++z) acc += part[(size_t)z * n + i];
    out[i] = acc;
}

// column sums of Y (M x N): part[z][n] over row chunks
template <typename T>
__global__ void colsum_kernel(int M, int N, const T *__restrict__ Y, int rows_per_z, T *__restrict__ part) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int r0 = blockIdx.y * rows_per_z, r1 = min(M, r0 + rows_per_z);
    T acc = 0;
    for (int m = r0; m < r1; ++m) acc += Y[(size_t)m * N + n];
    part[(size_t)blockIdx.y * N + n] = acc;
}

// d_pre = d_post * (1 - h^2)
template <typename T>
__global__ void tanh_back_kernel(long long n, const T *__restrict__ h, T *__restrict__ d) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] *= T(1) - h[i] * h[i];
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per sample.  O: [S][n_out], n_out = 1 + 2*nc*rank (rank = 4).
template <typename T>
__global__ __launch_bounds__(64) void loss_grad_kernel(int S, int nc, int train_uv, T omega, const T *__restrict__ O,
                                                       const T *__restrict__ R, const T *__restrict__ BR,
                                                       const T *__restrict__ E, T *__restrict__ dO,
                                                       T *__restrict__ loss_s) {
    const int s = blockIdx.x, i = threadIdx.x;
    const int n_out = 1 + 8 * nc;
    const T *o = O + (size_t)s * n_out;
    const bool on = i < nc;
    T r = on ? R[(size_t)s * nc + i] : T(0);
    T br = on ? BR[(size_t)s * nc + i] : T(0);
    T e = on ? E[(size_t)s * nc + i] : T(0);
    T U[4], V[4];
    for (int a = 0; a < 4; ++a) {
        U[a] = on ? o[1 + i * 4 + a] : T(0);
        V[a] = on ? o[1 + 4 * nc + i * 4 + a] : T(0);
    }
    T q[4];
    for (int a = 0; a < 4; ++a) q[a] = wave_sum(V[a] * r);
    T P = br + U[0] * q[0] + U[1] * q[1] + U[2] * q[2] + U[3] * q[3];
    T sig = T(1) / (T(1) + exp(-o[0]));
    T w = T(2) * sig;
    T res = on ? omega * w * P - e : T(0);
    T ne = wave_sum(e * e);
    T inv_ne = ne > T(0) ? T(1) / ne : T(0);  // a zero-error sample contributes nothing
    T ls = wave_sum(res * res) * inv_ne;
    T g = T(2) * res * inv_ne / T(S);
    T dw = omega * wave_sum(g * P);
    T dP = omega * w * g;
    T *d = dO + (size_t)s * n_out;
    T dq[4];
    for (int a = 0; a < 4; ++a) dq[a] = wave_sum(dP * U[a]);
    if (on) {
        // train_uv = 0 trains the relaxation weight only (U, V gradients zero)
        for (int a = 0; a < 4; ++a) {
            d[1 + i * 4 + a] = train_uv ? dP * q[a] : T(0);
            d[1 + 4 * nc + i * 4 + a] = train_uv ? dq[a] * r : T(0);
        }
    }
    if (i == 0) {
        d[0] = dw * T(2) * sig * (T(1) - sig);
        loss_s[s] = ls;
    }
}

template <typename T>
__global__ void mean_kernel(int S, const T *__restrict__ v, T *__restrict__ out) {
    __shared__ T red[256];
    T acc = 0;
    for (int i = threadIdx.x; i < S; i += 256) acc += v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / T(S);
}

__global__ void adam_kernel(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// --------------------------------------------------------------------------
template <typename T, bool TA, bool TB, int EPI>
static int gemm(int M, int N, int K, const T *A, int lda, const T *B, int ldb, T *C, int ldc, const T *bias, int nz,
                hipStream_t st) {
    if (M <= 0 || N <= 0) return 0;
    int kchunk = (K + nz - 1) / nz;
    kchunk = ((kchunk + GT - 1) / GT) * GT;
    nz = (K + kchunk - 1) / kchunk;
    if (nz < 1) nz = 1;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, nz);
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       kchunk);
    return hipGetLastError() == hipSuccess ? nz : -1;
}

template <typename T>
static void offsets(int n_in, int w, int n_out, const T *p, const T *&W1, const T *&b1, const T *&W2, const T *&b2,
                    const T *&W3, const T *&b3) {
    W1 = p;
    b1 = W1 + (size_t)w * n_in;
    W2 = b1 + w;
    b2 = W2 + (size_t)w * w;
    W3 = b2 + w;
    b3 = W3 + (size_t)n_out * w;
}

template <typename T>
int mlp_forward(int n_in, int w, int n_out, int S, const T *p, const T *X, T *H1, T *H2, T *O, hipStream_t st) {
    const T *W1, *b1, *W2, *b2, *W3, *b3;
    offsets(n_in, w, n_out, p, W1, b1, W2, b2, W3, b3);
    if (gemm<T, false, true, 2>(S, w, n_in, X, n_in, W1, n_in, H1, w, b1, 1, st) < 0) return -1;
    if (gemm<T, false, true, 2>(S, w, w, H1, w, W2, w, H2, w, b2, 1, st) < 0) return -1;
    if (gemm<T, false, true, 1>(S, n_out, w, H2, w, W3, w, O, n_out, b3, 1, st) < 0) return -1;
    return 0;
}

// weight gradient gW[n][k] = sum_s dY[s][n] X[s][k] and bias gradient, reduced deterministically
template <typename T>
static int wgrad(int S, int N, int K, const T *dY, const T *X, T *gW, T *gb, T *work, hipStream_t st) {
    int nz = std::max(1, std::min(64, (S + 511) / 512));
    nz = gemm<T, true, false, 0>(N, K, S, dY, N, X, K, work, K, nullptr, nz, st);
    if (nz < 0) return -1;
    long long n = (long long)N * K;
    hipLaunchKernelGGL((sum_splits_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, n, nz, work, gW);
    int rows = 512, nzb = (S + rows - 1) / rows;
    hipLaunchKernelGGL((colsum_kernel<T>), dim3((N + 255) / 256, nzb), dim3(256), 0, st, S, N, dY, rows, work);
    hipLaunchKernelGGL((sum_splits_kernel<T>), dim3((N + 255) / 256), dim3(256), 0, st, (long long)N, nzb, work, gb);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int mlp_backward(int n_in, int w, int n_out, int S, const T *p, const T *X, const T *H1, const T *H2, const T *dO,
                 T *grads, T *dH, T *work, hipStream_t st) {
    const T *W1, *b1, *W2, *b2, *W3, *b3;
    offsets(n_in, w, n_out, p, W1, b1, W2, b2, W3, b3);
    T *gW1 = grads, *gb1 = gW1 + (size_t)w * n_in, *gW2 = gb1 + w, *gb2 = gW2 + (size_t)w * w, *gW3 = gb2 + w,
      *gb3 = gW3 + (size_t)n_out * w;
    T *d2 = dH, *d1 = dH + (size_t)S * w;
    if (wgrad<T>(S, n_out, w, dO, H2, gW3, gb3, work, st)) return -1;
    // d2 = (dO W3) * (1 - H2^2)
    if (gemm<T, false, false, 0>(S, w, n_out, dO, n_out, W3, w, d2, w, nullptr, 1, st) < 0) return -1;
    long long n = (long long)S * w;
    hipLaunchKernelGGL((tanh_back_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, n, H2, d2);
    if (wgrad<T>(S, w, w, d2, H1, gW2, gb2, work, st)) return -1;
    if (gemm<T, false, false, 0>(S, w, w, d2, w, W2, w, d1, w, nullptr, 1, st) < 0) return -1;
    hipLaunchKernelGGL((tanh_back_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, n, H1, d1);
    if (wgrad<T>(S, w, n_in, d1, X, gW1, gb1, work, st)) return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int mlp_loss_grad(int S, int nc, int train_uv, double omega, const T *O, const T *R, const T *BR, const T *E, T *dO,
                  T *loss_s, T *loss, hipStream_t st) {
    if (S <= 0 || nc > 64) return -1;
    hipLaunchKernelGGL((loss_grad_kernel<T>), dim3(S), dim3(64), 0, st, S, nc, train_uv, (T)omega, O, R, BR, E, dO,
                       loss_s);
    hipLaunchKernelGGL((mean_kernel<T>), dim3(1), dim3(256), 0, st, S, loss_s, loss);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int adam_step(int n, float *p, const float *g, float *m, float *v, int t, float lr, float b1, float b2, float eps,
              hipStream_t st) {
    if (n <= 0 || t < 1) return -1;
    float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int mlp_forward<float>(int, int, int, int, const float *, const float *, float *, float *, float *, hipStream_t);
template int mlp_forward<double>(int, int, int, int, const double *, const double *, double *, double *, double *,
                                 hipStream_t);
template int mlp_backward<float>(int, int, int, int, const float *, const float *, const float *, const float *,
                                 const float *, float *, float *, float *, hipStream_t);
template int mlp_backward<double>(int, int, int, int, const double *, const double *, const double *, const double *,
                                  const double *, double *, double *, double *, hipStream_t);
template int mlp_loss_grad<float>(int, int, int, double, const float *, const float *, const float *, const float *, float *,
                                  float *, float *, hipStream_t);
template int mlp_loss_grad<double>(int, int, int, double, const double *, const double *, const double *, const double *,
                                   double *, double *, double *, hipStream_t);

// --------------------------------------------------------------------------
// BF16 inference on the matrix cores.  width = 64, n_in <= 64, n_out <= 16*NT.
// One wave handles 16 samples through the three layers; activations live in
// LDS as bf16, weights are packed once as bf16 [N][64] (zero padded).
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    // round to nearest even
    unsigned u = __float_as_uint(x);
    unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (short)(u >> 16);
}

// pack W (N x K fp32, row-major) into bf16 [Npad][64] with zero padding
__global__ void pack_bf16_kernel(int N, int K, int Npad, const float *__restrict__ W, short *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Npad * 64) return;
    int n = i / 64, k = i % 64;
    out[i] = (n < N && k < K) ? to_bf16(W[(size_t)n * K + k]) : (short)0;
}

__device__ __forceinline__ void mfma_layer(const short (*act)[64 + 8], const short *__restrict__ W, int ntiles,
                                           int lane, f32x4 *acc) {
    // acc[t] = act (16 x 64) * W[t*16 .. t*16+15][0..63]^T
    for (int t = 0; t < ntiles; ++t) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            int k = ks * 16 + 4 * (lane / 16);
            bf16x4 a, b;
            const short *ap = &act[lane % 16][k];
            a[0] = ap[0]; a[1] = ap[1]; a[2] = ap[2]; a[3] = ap[3];
            const short *bp = W + (size_t)(t * 16 + lane % 16) * 64 + k;
            b[0] = bp[0]; b[1] = bp[1]; b[2] = bp[2]; b[3] = bp[3];
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
        }
        acc[t] = c;
    }
}

__global__ __launch_bounds__(256) void infer_bf16_kernel(int S, int n_in, int n_out, const float *__restrict__ X,
                                                         const short *__restrict__ W1, const float *__restrict__ b1,
                                                         const short *__restrict__ W2, const float *__restrict__ b2,
                                                         const short *__restrict__ W3, const float *__restrict__ b3,
                                                         float *__restrict__ O) {
    __shared__ short actA[4][16][64 + 8];
    __shared__ short actB[4][16][64 + 8];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int s0 = (blockIdx.x * 4 + wave) * 16;
    // load inputs (bf16, zero padded)
    for (int t = lane; t < 16 * 64; t += 64) {
        int m = t / 64, k = t % 64, s = s0 + m;
        actA[wave][m][k] = (s < S && k < n_in) ? to_bf16(X[(size_t)s * n_in + k]) : (short)0;
    }
    __syncthreads();
    f32x4 acc[4];
    // layer 1
    mfma_layer(actA[wave], W1, 4, lane, acc);
    for (int t = 0; t < 4; ++t)
        for (int i = 0; i < 4; ++i) {
            int m = 4 * (lane / 16) + i, n = t * 16 + lane % 16;
            actB[wave][m][n] = to_bf16(tanhf(acc[t][i] + b1[n]));
        }
    __syncthreads();
    mfma_layer(actB[wave], W2, 4, lane, acc);
    __syncthreads();
    for (int t = 0; t < 4; ++t)
        for (int i = 0; i < 4; ++i) {
            int m = 4 * (lane / 16) + i, n = t * 16 + lane % 16;
            actA[wave][m][n] = to_bf16(tanhf(acc[t][i] + b2[n]));
        }
    __syncthreads();
    const int ntiles = (n_out + 15) / 16;
    for (int t0 = 0; t0 < ntiles; t0 += 4) {
        int nt = min(4, ntiles - t0);
        mfma_layer(actA[wave], W3 + (size_t)t0 * 16 * 64, nt, lane, acc);
        for (int t = 0; t < nt; ++t)
            for (int i = 0; i < 4; ++i) {
                int m = 4 * (lane / 16) + i, n = (t0 + t) * 16 + lane % 16, s = s0 + m;
                if (s < S && n < n_out) O[(size_t)s * n_out + n] = acc[t][i] + b3[n];
            }
    }
}

int mlp_infer_bf16(int n_in, int w, int n_out, int S, const float *p, const float *X, float *O, short *wbuf,
                   hipStream_t st) {
    if (w != 64 || n_in > 64 || n_in < 1 || S <= 0) return -1;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    offsets(n_in, w, n_out, p, W1, b1, W2, b2, W3, b3);
    int np3 = ((n_out + 15) / 16) * 16;
    short *P1 = wbuf, *P2 = P1 + 64 * 64, *P3 = P2 + 64 * 64;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3((64 * 64 + 255) / 256), dim3(256), 0, st, w, n_in, 64, W1, P1);
    hipLaunchKernelGGL(pack_bf16_kernel, dim3((64 * 64 + 255) / 256), dim3(256), 0, st, w, w, 64, W2, P2);
    hipLaunchKernelGGL(pack_bf16_kernel, dim3((np3 * 64 + 255) / 256), dim3(256), 0, st, n_out, w, np3, W3, P3);
    int nb = (S + 63) / 64;
    hipLaunchKernelGGL(infer_bf16_kernel, dim3(nb), dim3(256), 0, st, S, n_in, n_out, X, P1, b1, P2, b2, P3, b3, O);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t mlp_infer_wbuf_elems(int n_out) { return (size_t)(64 * 64 * 2 + ((n_out + 15) / 16) * 16 * 64); }

// --------------------------------------------------------------------------
// Head: w_K = 2 sigmoid(o_0), U_K, V_K (nc x 4) into the smoother's arrays.
template <typename T>
__global__ void head_kernel(int S, int nc, const float *__restrict__ O, T *__restrict__ lw, T *__restrict__ lU,
                            T *__restrict__ lV) {
    int s = blockIdx.x, t = threadIdx.x;
    if (s >= S) return;
    int n_out = 1 + 8 * nc;
    const float *o = O + (size_t)s * n_out;
    if (t == 0) lw[s] = T(2) / (T(1) + exp(-(T)o[0]));
    for (int i = t; i < nc * 4; i += blockDim.x) {
        lU[(size_t)s * nc * 4 + i] = (T)o[1 + i];
        lV[(size_t)s * nc * 4 + i] = (T)o[1 + nc * 4 + i];
    }
}

template <typename T>
int launch_head(int S, int nc, const float *O, T *lw, T *lU, T *lV, hipStream_t st) {
    if (S <= 0) return 0;
    hipLaunchKernelGGL((head_kernel<T>), dim3(S), dim3(64), 0, st, S, nc, O, lw, lU, lV);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_head<float>(int, int, const float *, float *, float *, float *, hipStream_t);
template int launch_head<double>(int, int, const float *, double *, double *, double *, hipStream_t);

// --------------------------------------------------------------------------
// Training samples of the finest level's boundary cells:
//   R[b] = r_K, BR[b] = B_K r_K, E[b] = e_K   for K = bnd_cells[b].
template <typename T>
__global__ void boundary_samples_kernel(int nb, int nc, const int *__restrict__ bnd_cells, const T *__restrict__ Bt,
                                        const T *__restrict__ r, const T *__restrict__ e, T *__restrict__ R,
                                        T *__restrict__ BR, T *__restrict__ E) {
    __shared__ T rs[64];
    int b = blockIdx.x, i = threadIdx.x;
    int K = bnd_cells[b];
    if (i < nc) rs[i] = r[(size_t)K * nc + i];
    __syncthreads();
    if (i >= nc) return;
    const T *B = Bt + (size_t)b * nc * nc;
    T acc = 0;
    for (int j = 0; j < nc; ++j) acc += B[(size_t)j * nc + i] * rs[j];
    R[(size_t)b * nc + i] = rs[i];
    BR[(size_t)b * nc + i] = acc;
    E[(size_t)b * nc + i] = e[(size_t)K * nc + i];
}

int launch_boundary_samples(int nb, int nc, const int *bnd_cells, const double *Bt, const double *r, const double *e,
                            double *R, double *BR, double *E, hipStream_t st) {
    if (nb <= 0) return 0;
    if (nc > 64) return -1;
    hipLaunchKernelGGL((boundary_samples_kernel<double>), dim3(nb), dim3(64), 0, st, nb, nc, bnd_cells, Bt, r, e, R, BR,
                       E);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sbm
