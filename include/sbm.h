/*
 * sbm.h -- C ABI of the MI355X (gfx950) DG Shifted Boundary Method solver.
 *
 * The library solves the Poisson problem -Lap u = f in Omega, u = g on
 * Gamma = boundary of Omega (the paper's Sec. 2, model problem), with Omega
 * = {phi < 0} given by a level set (Sec. 4.1), on a Cartesian background mesh
 * of n^d cells covering [lo, hi]^d (Sec. 5 opening), discretised by the DG
 * shifted boundary method of degree p (Sec. 2.2, full DG-SBM form), and
 * preconditions restarted flexible GMRES with one hp-multigrid V-cycle per
 * iteration whose smoother is the cell-wise successive subspace correction
 * of Sec. 3.1 (red-black ordered, see sbm_options).
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status (SBM_OK = 0, negative = error,
 *    SBM_NOT_CONVERGED = 1); none throws, aborts or exits.
 *  - "device" pointers are HIP device allocations on the problem's device
 *    (for example torch.Tensor.data_ptr() of a cuda tensor); "host" pointers
 *    are ordinary CPU memory.  Unless stated otherwise the caller owns every
 *    buffer it passes; the library never frees or keeps them past the call.
 *  - Vectors on a level are laid out cell-major: active cells in DoF order
 *    (colour (i+j+k) mod 2 = 0 first, then colour 1, each lexicographic with
 *    i fastest), then the (p+1)^d Gauss-Lobatto nodes of the cell
 *    lexicographically with x fastest.  Length = n_active * (p+1)^d.
 *  - fp32 = 1 means the buffers hold float, otherwise double.
 *  - Asynchronous entry points enqueue work on the problem's stream
 *    (sbm_options.stream) and return; the synchronous ones say so.
 *  - One problem must not be used from two threads at the same time.
 */
#ifndef SBM_H
#define SBM_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SBM_OK = 0,
    SBM_NOT_CONVERGED = 1,
    SBM_EINVAL = -1,      /* bad argument, size or unsupported (d, p)           */
    SBM_ENOMEM = -2,      /* host or device allocation failed                   */
    SBM_EDEVICE = -3,     /* a HIP call failed                                  */
    SBM_ESINGULAR = -4,   /* a cell block or the coarse matrix is singular      */
    SBM_ENONFINITE = -5,  /* NaN / Inf met in the solve                         */
    SBM_EGEOM = -6        /* closest-point search failed                        */
};

enum { SBM_GEOM_BALLS = 0, SBM_GEOM_STAR2D = 1, SBM_GEOM_CALLBACK = 2, SBM_GEOM_ELLIPSOID = 3 };

/* Level-set description of Omega = {phi < 0}.  Sec. 4.1 (level set), Sec. 4.2
 * (closest-point projection).  All arrays are host memory, copied at setup.
 *  BALLS:   union of n_balls balls |x - centers[j]| < radii[j]
 *           (centers: n_balls x dim, row-major); one ball = disk / sphere;
 *           closest points are exact (Sec. 4.2 allows exact projections).
 *  STAR2D:  dim = 2, {|x| < r(t)}, r(t) = star_r0 + star_a sin(star_k t).
 *  CALLBACK: phi, grad (dim values) and hess (dim*dim, row-major) of a
 *           general level set, each called for one point; the closest point
 *           solves the Lagrangian stationarity system of Sec. 4.2 by Newton.
 *  ELLIPSOID: dim = 3, phi(x) = |diag(1/radii) R^T (x - centers)|^2 - 1 with
 *           3 semi-axes in radii and R = rotation (3x3 row-major, columns =
 *           principal axes); closest points by the same Newton iteration. */
typedef struct {
    int dim, kind, n_balls;
    const double *centers, *radii, *rotation;
    double star_r0, star_a;
    int star_k;
    double (*phi)(const double *x, void *user);
    void (*grad)(const double *x, double *g, void *user);
    void (*hess)(const double *x, double *H, void *user);
    void *user;
} sbm_geometry;

typedef struct {
    double lo, hi;        /* background box [lo, hi]^dim (default -1, 1)                      */
    double c_F, c_G;      /* sigma_F = c_F (p+1)^2 / h (default 2), sigma_Gamma = c_G (p+1)^2 / h (5) */
    double alpha;         /* Nitsche symmetry parameter alpha (default 1, quasi-symmetric)    */
    int ext;              /* extension operator: 0 = first-order Taylor E u = u + d.grad u
                             (Sec. 2.1), 1 = cell polynomial evaluated at x~ + d (default 1) */
    double omega;         /* smoother relaxation (default 1 for p <= 2, 0.8 for p = 3)        */
    int nu_pre, nu_post;  /* SSOR steps before / after the coarse correction (default 1, 1)   */
    int coarse_min;       /* geometric coarsening (p = 1) halves n while n is even,           */
    int coarse_dofs;      /* n/2 >= coarse_min (default 3) and the level still has more than  */
                          /* coarse_dofs active DoFs (default 2048); the last level is solved */
                          /* with a dense inverse (at most 4096 DoFs)                         */
    int vcycle_fp32;      /* sbm_solve: 0 = FP64 V-cycle, 1 = FP32 V-cycle (default 0)        */
    int allow_singular;   /* 1: do not fail on near-singular blocks; EVERY cell block is then */
                          /* inverted as (D_K + 1e-10 max|D_K| I)^-1 (not only the singular  */
                          /* ones), so the smoothing step keeps its repeated colour update  */
    int fuse_transfers;   /* V-cycle launches (same arithmetic either way).  1 (default): the
                             residual-restriction kernel also forms the coarser level's first
                             colour-0 update from zero, and the last colour updates of a
                             level add its final z into the finer level (the FP32 cycle's
                             finest level writes z in FP64 there).  0: separate kernels   */
    int penalty_p;        /* degree in the penalties: 0 (default) = each level's own degree p_l,
                             q >= 1 = sigma_F = c_F (q+1)^2 / h_l, sigma_Gamma = c_G (q+1)^2 / h_l
                             on every level (one penalty constant across the hierarchy)    */
    double lambda_frac;   /* active-cell rule (Sec. 2.1, Sec. 4.1): 0 (default) = the cell centre
                             lies in Omega; lambda in (0, 1] = the volume fraction of the cell
                             inside Omega exceeds lambda (lambda = 1: the whole cell inside),
                             the fraction taken as the share of frac_m^dim cell-midpoint
                             samples with phi < 0                                           */
    int frac_m;           /* samples per direction for the volume fraction (default 16)     */
    int min_neighbours;   /* 0 (default) or k >= 1: after the active-cell rule, cells with fewer
                             than k active face neighbours are dropped, repeatedly, until every
                             active cell has at least k (the k-core of the face-adjacency graph
                             of the active cells) on the finest mesh (its p-levels); removes
                             cells that hang on by one or two faces, whose blocks and patches
                             are near-singular at p = 3; coarser meshes keep the plain rule */
    double stab;          /* smoother block stabilisation for near-singular cell blocks
                             (Sec. 3.1 asks for one; 0 = none, default): singular values of
                             a cell block below stab * s_int, s_int = smallest singular value
                             of the level's interior block, are raised to that floor in its
                             inverse, B_K = sum_i v_i u_i^T / max(sigma_i, stab s_int); the
                             operator itself is unchanged                                   */
    int smoother;         /* 0 (default): multiplicative cell-wise smoother, red-black SSOR
                             (colours 0, 1, 1, 0 per step); 1: the additive cell-wise
                             smoother (block Jacobi, Sec. 3.1) accelerated by Chebyshev
                             polynomials (Sec. 5.3): one smoothing step is cheb_degree
                             block-Jacobi updates with the Chebyshev weights for the interval
                             [l/cheb_range, l], l = 1.2 x the largest eigenvalue modulus of
                             B A found by 25 power iterations from the all-ones vector at
                             setup (per level); no learned correction; transfers unfused  */
    int cheb_degree;      /* block-Jacobi updates per Chebyshev smoothing step (default 3)   */
    double cheb_range;    /* ratio of the interval's ends (default 20)                       */
    int pencil;           /* 1 (default): on 3D Q2 and Q3 levels the interior cells (no surrogate
                             face) go through a kernel with one lane per line of nodes, the
                             boundary cells through the one-thread-per-DoF kernel; 0: all
                             cells through the latter (same operator and update)          */
    int device;           /* HIP device ordinal (default 0); < 0 = host-only setup for tests:
                             no device data, the device entry points return SBM_EINVAL     */
    void *stream;         /* hipStream_t for all work (default NULL = null stream)            */
} sbm_options;

typedef struct {
    long long n_dofs;     /* finest-level vector length                                       */
    int n_active;         /* active cells on the finest level                                 */
    int n_colour0;        /* active cells of colour 0 on the finest level                     */
    int dofs_per_cell;    /* (p+1)^dim                                                        */
    int n_levels;         /* multigrid levels (coarsest = 0)                                  */
    int n_boundary_cells; /* finest-level cells with at least one surrogate face              */
    int n_surrogate_faces;/* finest-level surrogate faces                                     */
} sbm_layout;

typedef struct {
    int iterations;             /* FGMRES iterations (V-cycles) performed                    */
    int converged;              /* 1 if the true relative residual reached tol               */
    double rel_residual_true;   /* ||b - A x|| / ||b|| computed in FP64 at the end           */
    double seconds;             /* wall time of the solve                                    */
} sbm_stats;

/* Fill *o with the defaults for (dim, p).  Host only. */
int sbm_default_options(int dim, int p, sbm_options *o);

/* Build the hierarchy for geometry g, n^dim background cells and degree p
 * (1 <= p <= 3, dim in {2, 3}; n >= 1 and n^dim < 2^31): per level the centre-inside active
 * set (phi(cell centre) < 0), red-black order, neighbour table, surrogate
 * faces, closest points and shifts at the (p_l+1)^(dim-1) Gauss points of
 * every surrogate face (Sec. 4.2: once per level, stored), the cell blocks
 * D_K (Sec. 3.1, A_i = R_i A R_i^T) with their FP64 LU inverses, the
 * transfer maps (Sec. 3.2) and the dense coarsest-level inverse.  Uploads
 * everything to o->device.  Synchronous.  On success *out owns all of it.
 * Errors: SBM_EINVAL (arguments, or a level with no active cell: an empty
 * domain, or coarsening allowed down to a mesh with no cell centre inside
 * the domain), SBM_ESINGULAR, SBM_EGEOM, SBM_ENOMEM, SBM_EDEVICE. */
int sbm_setup(const sbm_geometry *g, int n, int p, const sbm_options *o, struct sbm_problem **out);

int sbm_layout_info(const struct sbm_problem *pb, sbm_layout *out);

/* Host copies of finest-level metadata (for tests): active cell multi-indices
 * (n_active x dim ints, DoF order) and the surrogate-face shifts d = x - x~
 * of a level (n_surrogate_faces x (p_l+1)^(dim-1) x dim doubles, faces
 * ordered by (cell, direction k, side s)).  level = -1 means the finest.
 * cap = capacity of the output in elements; SBM_EINVAL if too small. */
int sbm_active_cells(const struct sbm_problem *pb, int level, int *ijk, long long cap);
int sbm_level_info(const struct sbm_problem *pb, int level, int *n, int *p, int *n_active,
                   int *n_colour0, int *n_surrogate_faces);
int sbm_shifts(const struct sbm_problem *pb, int level, double *host_out, long long cap);
/* Cell blocks of a level (for tests): boundary blocks (cells with a surrogate
 * face), those whose inverse the singular-value floor changed (stab > 0,
 * Sec. 3.1 stabilisation), and how many of the latter are colour-0 cells.
 * Null outputs are skipped; level = -1 means the finest. */
int sbm_level_blocks(const struct sbm_problem *pb, int level, int *n_boundary, int *n_clipped,
                     int *n_clipped_colour0);

/* Test hook: replace the shifts d of a level's surrogate Gauss points by
 * externally supplied ones (host, count = n_surrogate_faces x (p_l+1)^(dim-1)
 * x dim doubles, physical units, the layout of sbm_shifts), so that kernel
 * parity can be checked independently of the closest-point search (Sec. 4.2).
 * The level's boundary-cell blocks and inverses (and, on level 0, the dense
 * coarse inverse) are rebuilt from them and the device copies of the shifts and
 * inverses overwritten in place (no allocation).  An installed learned
 * correction keeps its w, U, V.  Synchronous.  SBM_EINVAL for a wrong count or
 * non-finite values; on an error the problem keeps its previous shifts. */
int sbm_set_shifts(struct sbm_problem *pb, int level, const double *host_shifts, long long count);

/* Right-hand side of the DG-SBM system (Sec. 2.2): int_K f phi_i plus, on
 * surrogate faces, [-alpha grad phi_i . n~ + sigma_Gamma phi_i] g(x~ + d).
 * f and g are batched host callbacks: called with npts points (npts x dim,
 * row-major) they write npts values.  b_dev: finest-level FP64 device vector.
 * Synchronous. */
typedef void (*sbm_field_fn)(const double *x, long long npts, double *out, void *user);
int sbm_rhs(struct sbm_problem *pb, sbm_field_fn f, sbm_field_fn g, void *user, double *b_dev);

/* y = A x on the finest level (volume + SIPG faces, Sec. 2.2; Nitsche terms
 * with the extended trial function on surrogate faces, Sec. 2.1).  x, y:
 * device vectors of n_dofs; they must not alias.  Asynchronous. */
int sbm_apply(struct sbm_problem *pb, const void *x_dev, void *y_dev, int fp32);

/* z = M^{-1} r: one V(nu_pre, nu_post)-cycle (Sec. 3, one V-cycle as the
 * preconditioner) with the red-black cell-block SSOR smoother.  r, z:
 * device vectors of n_dofs (must not alias).  fp32 selects the precision of
 * the whole cycle (blocks stored in that precision).  Asynchronous. */
int sbm_vcycle(struct sbm_problem *pb, const void *r_dev, void *z_dev, int fp32);

/* Longest FGMRES restart sbm_solve and sbm_solve_noalloc accept. */
#define SBM_MAX_RESTART 256

/* Solve A x = b with FGMRES(restart), right-preconditioned by one V-cycle
 * (FP32 if o->vcycle_fp32), FP64 Arnoldi (classical Gram-Schmidt, second pass
 * only when the first cancels, |w'| < 0.1 |w|, when tol < 1e-10, or beyond
 * the 30th basis vector once the residual has fallen 1.6e4-fold within the
 * cycle), x0 = 0; stops when the TRUE
 * relative residual ||b - A x|| / ||b|| <= tol, or after max_iter
 * iterations (then SBM_NOT_CONVERGED, x holds the last iterate).  b, x: FP64
 * device vectors; restart in 1..SBM_MAX_RESTART (else SBM_EINVAL); the
 * workspace holds 2 restart + 2 vectors of n_dofs.  Synchronous.  st may be
 * NULL. */
int sbm_solve(struct sbm_problem *pb, const double *b_dev, double *x_dev, double tol, int restart,
              int max_iter, sbm_stats *st);

/* Size of the device array that holds the workspace of sbm_solve_noalloc on
 * each GPU (128 MiB). */
#define SBM_NOALLOC_SCRATCH_BYTES (128ull << 20)

/* Allocation-free variant of sbm_solve, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, arithmetic and results as
 * sbm_solve; the FGMRES workspace (Krylov bases, work vector, partial sums,
 * device scalars) lives in one file-scope device array of
 * SBM_NOALLOC_SCRATCH_BYTES instead of buffers owned by the problem, and the
 * call makes no device or host allocation (the problem itself, set up by
 * sbm_setup, already holds every level's data and the pinned staging word).
 * Limit: sbm_solve_noalloc_doubles(pb, restart) * 8 must not exceed
 * SBM_NOALLOC_SCRATCH_BYTES (about 2 (restart + 1) n_dofs doubles; 270k DoFs
 * at restart 30), else SBM_EINVAL with a message (sbm_last_error) and nothing
 * runs.  Every problem on one GPU shares that GPU's array, which keeps the
 * last call's contents (none of it needs to start at zero): calls that overlap
 * on one GPU -- two streams, two threads -- race and must be serialised by the
 * caller.  Synchronous, like sbm_solve. */
int sbm_solve_noalloc(struct sbm_problem *pb, const double *b_dev, double *x_dev, double tol, int restart,
                      int max_iter, sbm_stats *st);
/* Doubles of scratch the allocation-free solve needs for pb at this restart
 * length (-1 for an invalid problem or restart).  Host only. */
long long sbm_solve_noalloc_doubles(const struct sbm_problem *pb, int restart);

/* Switch the precision of the V-cycle used by later sbm_solve calls
 * (0 = FP64, 1 = FP32 with FP32 blocks; the outer Arnoldi, the operator in
 * the Krylov space, the true residual and x stay FP64).  Host only. */
int sbm_set_vcycle_fp32(struct sbm_problem *pb, int fp32);

/* Level-resolved building blocks (for parity tests and training-data
 * generation).  level in [0, n_levels); -1 = finest.  All asynchronous.
 *  sbm_level_apply:   y = A_l x
 *  sbm_colour_update: z_K += omega B_K (b - A_l z)_K for the active cells of
 *                     the given colour (Sec. 3.1, successive correction; cells
 *                     of one colour do not couple)
 *  sbm_restrict:      b_c = I^T r   from level l to l-1 (Sec. 3.2)
 *  sbm_prolong_add:   z_f += I z_c  from level l-1 to level l            */
int sbm_level_apply(struct sbm_problem *pb, int level, const void *x_dev, void *y_dev, int fp32);
int sbm_colour_update(struct sbm_problem *pb, int level, int colour, const void *b_dev, void *z_dev,
                      int fp32);
int sbm_restrict(struct sbm_problem *pb, int level, const void *r_dev, void *bc_dev, int fp32);
int sbm_prolong_add(struct sbm_problem *pb, int level, const void *zc_dev, void *zf_dev, int fp32);

/* Host copies of the assembled cell block D_K = A_K (inverse = 0) or of its
 * FP64 LU inverse B_K (inverse = 1) of active cell `cell` on a level
 * ((p_l+1)^d x (p_l+1)^d doubles, row-major, row = test function), and of the
 * dense coarsest-level matrix (n0 x n0, n0 = active DoFs of level 0; cap =
 * capacity in doubles).  For tests; available also on host-only problems. */
int sbm_cell_block(const struct sbm_problem *pb, int level, int cell, int inverse, double *out);
int sbm_coarse_matrix(const struct sbm_problem *pb, double *out, long long cap);

/* ---------------------------------------------------------------------------
 * Learned boundary-cell correction of the smoother (not part of the paper;
 * the paper finds the cell-wise smoother weak for p = 3 in 3D, Sec. 5.3, and
 * leaves better smoothers to future work, Sec. 6).  On surrogate-boundary
 * cells of the finest level the colour update becomes
 *     z_K += omega * w_K * (B_K + U_K V_K^T) r_K,   w_K = 2 sigmoid(o_0),
 * with (o_0, U_K, V_K) (U_K, V_K: (p+1)^d x 4, row-major) the output of a
 * 3-layer tanh MLP on per-cell features.  Parameters are one flat FP32/FP64
 * array: W1 (width x n_in, row-major), b1, W2 (width x width), b2,
 * W3 (n_out x width), b3; n_out = 1 + 8 (p+1)^d.
 *
 * sbm_feature_dim:       n_in for a dimension (2d faces x (4 + 2d)).
 * sbm_boundary_cells:    number (and, if cells != NULL, the active indices)
 *                        of the finest level's boundary cells (host).
 * sbm_boundary_features: n_boundary x n_in doubles (host): per face (k, s):
 *                        surrogate mask, mean/min/max of d.n~/h, mean d/h,
 *                        mean unit normal of Gamma at the projections.
 * sbm_boundary_samples:  training rows of the boundary cells (device, FP64,
 *                        n_boundary x (p+1)^d each): R = r_K, BR = B_K r_K,
 *                        E = e_K for finest-level vectors r, e.  Async.
 * sbm_set_learned:       BF16 inference (matrix cores, FP32 accumulation) on
 *                        the features with device FP32 parameters of the
 *                        given width (64), installs w_K, U_K, V_K and enables
 *                        the correction; params = NULL disables it.  Sync.
 * sbm_set_learned_arrays:install given w_K (n_boundary), U_K and V_K
 *                        (n_boundary x (p+1)^d x 4) from host memory.  Sync.
 * sbm_use_learned:       switch an installed correction on (1) or off (0).
 *
 * Training kernels (no problem needed; fp64 selects double buffers, else
 * float; all device pointers, asynchronous on `stream`):
 * sbm_mlp_forward:   H1, H2: batch x width, O: batch x n_out.
 * sbm_mlp_loss_grad: L = mean_s |omega w (BR + U V^T R) - E|^2 / |E|^2 and
 *                    dL/dO (batch x n_out); loss_s: batch, loss: 1 value.
 *                    n_cell <= 64 (rank 4); a sample with E = 0 contributes
 *                    zero; train_uv = 0 zeroes the U, V part of dL/dO (the
 *                    relaxation weight alone is trained).
 * sbm_mlp_backward:  grads (flat, as the parameters); dH: 2 x batch x width;
 *                    work: sbm_mlp_work_elems(...) elements.
 * sbm_adam:          one Adam step (t = 1-based), FP32.
 * sbm_mlp_infer_bf16:O = MLP(X) in BF16 on the matrix cores (width 64,
 *                    n_in <= 64); wbuf: sbm_mlp_infer_wbuf_elems(n_out) shorts. */
int sbm_feature_dim(int dim);
int sbm_boundary_cells(const struct sbm_problem *pb, int *n_boundary, int *cells, long long cap);
int sbm_boundary_features(const struct sbm_problem *pb, double *host_out, long long cap);
int sbm_boundary_samples(struct sbm_problem *pb, const double *r_dev, const double *e_dev, double *R_dev,
                         double *BR_dev, double *E_dev);
/* Training pairs of the boundary cells from the method's own iterates (device,
 * FP64, asynchronous): for a known discrete solution x* (b = A x*) and an
 * iterate z, r = b - A z on the finest level, then per boundary cell K (in
 * sbm_boundary_cells order) R = r_K, BR = B_K r_K, E = x*_K - z_K, each row
 * triple scaled by 1 / |E| (the loss is invariant to a per-sample scale);
 * valid[b] = 0 and zero rows where |E| = 0 or an entry is not finite.
 * R, BR, E: n_boundary x (p+1)^d; valid: n_boundary ints.  Uses two
 * finest-level work vectors the problem allocates on first use. */
int sbm_collect_pairs(struct sbm_problem *pb, const double *x_star_dev, const double *b_dev, const double *z_dev,
                      double *R_dev, double *BR_dev, double *E_dev, int *valid_dev);
/* steps preconditioned Richardson iterations z <- z + M^{-1}(b - A z) with the
 * FP64 V-cycle (Sec. 3 smoother and cycle; the learned correction when it is
 * switched on), finest level, in place (device, asynchronous). */
int sbm_richardson(struct sbm_problem *pb, const double *b_dev, double *z_dev, int steps);
int sbm_set_learned(struct sbm_problem *pb, const float *params_dev, int width);
int sbm_set_learned_arrays(struct sbm_problem *pb, const double *w, const double *U, const double *V);
int sbm_use_learned(struct sbm_problem *pb, int on);
int sbm_mlp_forward(int fp64, int n_in, int width, int n_out, int batch, const void *params, const void *X, void *H1,
                    void *H2, void *O, void *stream);
int sbm_mlp_loss_grad(int fp64, int batch, int n_cell, int train_uv, double omega, const void *O, const void *R,
                      const void *BR, const void *E, void *dO, void *loss_s, void *loss, void *stream);
long long sbm_mlp_work_elems(int n_in, int width, int n_out, int batch);
int sbm_mlp_backward(int fp64, int n_in, int width, int n_out, int batch, const void *params, const void *X,
                     const void *H1, const void *H2, const void *dO, void *grads, void *dH, void *work, void *stream);
int sbm_adam(int n, float *params, const float *grads, float *m, float *v, int t, float lr, float b1, float b2,
             float eps, void *stream);
long long sbm_mlp_infer_wbuf_elems(int n_out);
int sbm_mlp_infer_bf16(int n_in, int width, int n_out, int batch, const float *params, const float *X, float *O,
                       short *wbuf, void *stream);

/* Synchronise the problem's stream.  Returns SBM_EDEVICE on a HIP error. */
int sbm_sync(struct sbm_problem *pb);

/* Free everything the problem owns (device and host).  NULL is accepted.
 * sbm_setup may hand back a problem together with an error status (so that
 * sbm_last_error can be read); it must still be destroyed. */
int sbm_destroy(struct sbm_problem *pb);
const char *sbm_strerror(int status);
/* Text of the last error recorded on pb (empty if none); owned by pb. */
const char *sbm_last_error(const struct sbm_problem *pb);

#ifdef __cplusplus
}
#endif
#endif /* SBM_H */
