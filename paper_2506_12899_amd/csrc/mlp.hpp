// Learned boundary-cell correction: kernel launchers (mlp.hip).
#pragma once

#include "common.hpp"

namespace sbm {

template <typename T>
int mlp_forward(int n_in, int w, int n_out, int S, const T *p, const T *X, T *H1, T *H2, T *O, hipStream_t st);
template <typename T>
int mlp_backward(int n_in, int w, int n_out, int S, const T *p, const T *X, const T *H1, const T *H2, const T *dO,
                 T *grads, T *dH, T *work, hipStream_t st);
template <typename T>
int mlp_loss_grad(int S, int nc, int train_uv, double omega, const T *O, const T *R, const T *BR, const T *E, T *dO, T *loss_s,
                  T *loss, hipStream_t st);
int adam_step(int n, float *p, const float *g, float *m, float *v, int t, float lr, float b1, float b2, float eps,
              hipStream_t st);
int mlp_infer_bf16(int n_in, int w, int n_out, int S, const float *p, const float *X, float *O, short *wbuf,
                   hipStream_t st);
size_t mlp_infer_wbuf_elems(int n_out);
template <typename T>
int launch_head(int S, int nc, const float *O, T *lw, T *lU, T *lV, hipStream_t st);
int launch_boundary_samples(int nb, int nc, const int *bnd_cells, const double *Bt, const double *r, const double *e,
                            double *R, double *BR, double *E, hipStream_t st);

inline int feature_dim(int d) { return 2 * d * (4 + 2 * d); }

// r = b - A x on the finest level, FP64 (solver.hip)
int finest_residual(sbm_problem *pb, const double *x, const double *b, double *r);

}  // namespace sbm
