/*
 * axs.h -- C ABI of the multibody acoustic scattering solver for bodies of
 * revolution (Hao, Martinsson, Young, arXiv 1406.0236), built for AMD MI355X.
 *
 * Problem (Sec. 2, eq. "basic"): sound-soft exterior Helmholtz problem
 *     -Lap u - kappa^2 u = 0 outside Gamma,  u = -v on Gamma,  radiating,
 * written as the combined-field BIE (eq. "intHelm2")
 *     1/2 sigma(x) + int_Gamma G(x, x') sigma(x') dA(x') = -v(x),
 *     G = d phi / d n(x') + i eta phi,   phi = exp(i kappa R) / (4 pi R)
 * (the paper fixes eta = kappa; eta is a parameter here).
 * Discretisation (Sec. 3): per body, a composite Gauss-Legendre rule on the
 * generating curve times the trapezoidal rule in the azimuth; Nystrom
 * matrix A = D + B with D = blockdiag(F* A~ F) (modal matrices, eq. "FAF")
 * and B the naive-rule inter-body blocks (Sec. 3.3).
 * Solver (Sec. 4, eq. "precond"): GMRES on  sigma + D^{-1} B sigma = -D^{-1} v.
 *
 * Global conventions
 *  - Node order: body (in build order), contour node i (panel-major), azimuth
 *    l (theta_l = 2 pi l / N_F, N_F = 2M + 1).  N = sum of N_G N_F over bodies.
 *  - Device vectors are complex128 interleaved (re, im), laid out [nrhs][N]
 *    row-major, in memory the caller owns (e.g. torch tensors).  The library
 *    never frees, retains or resizes caller memory.
 *  - Host arrays are copied during the call; the caller keeps ownership.
 *  - All device work is ordered on the stream given to axs_create; calls
 *    return once the work is enqueued unless stated otherwise.  axs_solve and
 *    axs_precompute_scattering synchronise that stream.
 *  - Every entry point returns an axs_status; a failed call leaves a message
 *    readable through axs_last_error.  Nothing crosses the ABI as an
 *    exception.  A context is not thread-safe; distinct contexts are
 *    independent.
 */
#ifndef AXS_H
#define AXS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct axs_ctx axs_ctx;
typedef int32_t axs_status;

enum {
    AXS_OK = 0,
    AXS_NOT_CONVERGED = 1,   /* soft: solve stopped at max_iters above tol */
    AXS_EINVAL = -1,         /* invalid argument (message says which) */
    AXS_EHIP = -2,           /* a HIP runtime call failed */
    AXS_ENOMEM = -3,         /* device allocation failed */
    AXS_ESTATE = -4,         /* call out of order (e.g. matvec before precompute) */
    AXS_ENONFINITE = -5      /* NaN/Inf in an input or in a residual */
};

enum {
    AXS_FP64 = 0,            /* every step of the operator in FP64 */
    AXS_FP32 = 1             /* inter-body sum, DFTs and modal applies in FP32,
                                input/output vectors still complex128 */
};

/* Optional device allocator supplied by the caller (e.g. a framework's
 * caching allocator).  alloc returns NULL on failure.  If both are NULL the
 * library uses hipMalloc/hipFree. */
typedef void *(*axs_alloc_fn)(size_t bytes, void *user);
typedef void (*axs_free_fn)(void *ptr, void *user);

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
axs_status axs_create(axs_ctx **out, int device, void *hip_stream, axs_alloc_fn alloc,
                      axs_free_fn free_fn, void *user);
/* Release every device buffer the context owns, then the context. */
axs_status axs_destroy(axs_ctx *ctx);
/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char *axs_last_error(const axs_ctx *ctx);

/* Add one body of revolution (Sec. 3.2 discretisation).
 *  rz[2*NG], drz[2*NG] : (r, z) and d(r, z)/ds at the NG = n_panels * p contour
 *      nodes, panel-major; s in [-1, 1] is the panel parameter and the nodes
 *      sit at the p-point Gauss-Legendre nodes of each panel.  The curve runs
 *      from an axis point at the top to one at the bottom, so the outward
 *      normal is (-z', r') / |gamma'|.  r must be > 0 at every node.
 *  gw[NG] : the Gauss-Legendre weight of each node on [-1, 1]; checked against
 *      the library's own p-point rule (AXS_EINVAL if they differ).
 *  kappa >= 0, eta : wavenumber and coupling; all bodies of a context must
 *      share them (AXS_EINVAL otherwise).
 *  M >= 0 : Fourier cutoff; the body has N_F = 2M + 1 azimuthal nodes.
 *  centre[3], rot[9] (row-major, orthonormal) : x = centre + rot (r cos th, r sin th, z).
 *  Bodies with identical (rz, drz, gw, p, M) share their scattering matrices.
 *  Bodies whose bounding balls (about `centre`) overlap are rejected
 *  (AXS_EINVAL): Sec. 3.3 leaves touching or overlapping scatterers out.
 *  On success *body_id is the body's index (build order). */
axs_status axs_build_body(axs_ctx *ctx, const double *rz, const double *drz, const double *gw,
                          int n_panels, int p, double kappa, double eta, int M,
                          const double centre[3], const double rot[9], int *body_id);

/* Build the modal matrices A~_m (m = 0..M) of every distinct shape on the
 * device in FP64 -- modal kernels, near-panel product integration, 1/2 I --
 * and store S_m = A~_m^{-1} (Sec. 3.2, eqs. "FAF", "singleinverse";
 * A~_{-m} = A~_m).  Also lays out the global node arrays.  Synchronous.
 * After it, axs_build_body returns AXS_ESTATE. */
axs_status axs_precompute_scattering(axs_ctx *ctx);

/* Number of unknowns N (valid after the first axs_build_body). */
axs_status axs_num_unknowns(const axs_ctx *ctx, int64_t *N);

/* Host copy of the node geometry, [N][7] = (x, y, z, nx, ny, nz, w) with w the
 * surface quadrature weight (2 pi / N_F) r |gamma'| w_gauss.  After precompute. */
axs_status axs_node_geometry(axs_ctx *ctx, double *xyz_n_w);

/* Device copy of the modal matrices of body `body_id`'s shape, complex128
 * [M+1][NG][NG] row-major: which = 0 gives A~_m, which = 1 gives S_m. */
axs_status axs_modal_matrices(axs_ctx *ctx, int body_id, int which, void *out);

/* y = sigma + D^{-1} B sigma  (eq. "precond") for nrhs vectors.
 * sigma, y : device complex128 [nrhs][N]; they must not overlap.
 * precision : AXS_FP64 or AXS_FP32 (see above).
 * The input is scanned for NaN/Inf first (AXS_ENONFINITE, nothing computed);
 * that scan synchronises the stream before the operator is queued.  The same
 * holds for axs_apply_interbody and axs_apply_precond below. */
axs_status axs_apply_matvec(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision);

/* axs_apply_matvec without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and result as axs_apply_matvec (the same
 * kernels); the library's scratch for the call -- staged densities, inter-body
 * partial sums, DFT workspaces, and the work table where the launch shape's
 * table is not cached yet -- is a file-scope device array of 256 MiB on each
 * device (taken at axs_create, held until the process ends), so:
 *  - sizes whose scratch exceeds 256 MiB are refused (AXS_EINVAL, the message
 *    gives the bytes needed): nrhs x N x (splits + 3) x 16 bytes in FP64, half
 *    that in FP32 (the 27-sphere workload: one rhs in either precision);
 *  - only the point and ring orders of the inter-body sum run here (the
 *    defaults below 16 right-hand sides); a context configured for the MFMA
 *    orders gets AXS_EINVAL;
 *  - every call on a device shares that device's array: calls that overlap
 *    on one device (other streams, other contexts, other threads) race;
 *  - no scan for NaN/Inf and no synchronisation, except on the first call
 *    with a launch shape whose work table is not cached (one synchronous
 *    host-to-device copy of the table into the array). */
axs_status axs_apply_matvec_noalloc(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision);

/* Building blocks of the operator, same layouts as axs_apply_matvec:
 *   axs_apply_interbody : y = B sigma        (inter-body sum alone)
 *   axs_apply_precond   : y = D^{-1} x       (per-body DFT, S_m applies, inverse DFT) */
axs_status axs_apply_interbody(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision);
axs_status axs_apply_precond(axs_ctx *ctx, const void *x, void *y, int nrhs, int precision);

typedef struct {
    int32_t iterations;       /* outer iterations (FP64 operator applications) */
    int32_t inner_iterations; /* inner (FP32 operator) iterations, mixed mode */
    double rel_residual;      /* final FP64 || b - (I + D^-1 B) sigma || / || b ||, b = -D^-1 v:
                                 the GMRES least-squares residual of the FP64 Arnoldi
                                 relation, or with AXS_SOLVE_CERTIFY recomputed from sigma */
    double seconds;           /* wall time of the solve on the host clock */
    int32_t used_warm_start;  /* 1 if sigma0 was kept (see axs_solve) */
    int32_t converged;
} axs_solve_info;

enum {
    AXS_SOLVE_FP64 = 0,       /* GMRES, FP64 operator */
    AXS_SOLVE_MIXED = 1,      /* flexible GMRES with FP64 operator and residual, whose
                                 preconditioner is an inner GMRES on the FP32 operator */
    AXS_SOLVE_CERTIFY = 16,   /* flag, OR-ed into the mode: after the iteration, apply
                                 the FP64 operator once more to the returned sigma and
                                 report (and test convergence on) that explicit residual */
    AXS_SOLVE_UNPRECONDITIONED = 32, /* flag, FP64 mode only: GMRES on (D + B) sigma = -v,
                                 the system of Sec. 3.3 without the block-diagonal
                                 preconditioner of Sec. 4 (residual relative to ||v||);
                                 for the comparison the paper makes at zero frequency
                                 (Sec. 6.1), where it finds the preconditioner superfluous */
    AXS_SOLVE_RESTART_INNER = 64 /* flag, mixed mode only: every inner GMRES starts from
                                 scratch.  By default the first inner run keeps its Krylov
                                 basis (up to 61 vectors of nrhs x N complex128) and every
                                 later inner run is augmented with it (it orthogonalises
                                 against A U = C as well and adds U's part to its result),
                                 which saves inner iterations; the flag saves that memory.
                                 The answer is certified by the FP64 outer residual either way. */
};

/* Solve (eq. "precond")  sigma + D^{-1} B sigma = -D^{-1} v  for nrhs incident fields
 * (with AXS_SOLVE_UNPRECONDITIONED: (D + B) sigma = -v).
 *  incident : device complex128 [nrhs][N], v at the nodes.
 *  sigma0   : device complex128 [nrhs][N] initial guess, or NULL for zero.
 *             AXS_SOLVE_FP64: GMRES starts from the guess if its FP64 residual is
 *             below || b || (one FP64 application), else from zero.
 *             AXS_SOLVE_MIXED: the guess g enters the first application of the
 *             flexible preconditioner, z_1 = (g + inner(b - A32 g)) / || b ||, if
 *             its residual in the FP32 operator is below || b || (one FP32
 *             application), else that application is the plain one; the FP64
 *             outer residual decides convergence either way.
 *  sigma    : device complex128 [nrhs][N], the result.
 *  mode     : AXS_SOLVE_FP64 or AXS_SOLVE_MIXED, optionally | AXS_SOLVE_CERTIFY
 *             (and, mixed only, | AXS_SOLVE_RESTART_INNER).
 *             Without the flag the residual is the one GMRES minimises in its FP64
 *             Arnoldi basis (classical Gram-Schmidt twice), equal to the explicit
 *             one up to FP64 rounding; the flag costs one more FP64 application.
 *  tol      : stop when every right-hand side has relative FP64 residual <= tol.
 *  max_iters: cap on outer iterations (Krylov dimension; no restart).
 *  info     : host array [nrhs].  Returns AXS_NOT_CONVERGED if any rhs missed tol. */
axs_status axs_solve(axs_ctx *ctx, const void *incident, const void *sigma0, void *sigma,
                     int nrhs, int mode, double tol, int max_iters, axs_solve_info *info);

/* v[c][i] = exp(i kappa d_c . x_i) for nrhs unit directions dirs[nrhs][3] (host). */
axs_status axs_incident_plane_waves(axs_ctx *ctx, const double *dirs, int nrhs, void *v);

/* v[i] = sum_s amp_s exp(i kappa |x_i - y_s|) / (4 pi |x_i - y_s|): the field of
 * ns point sources y_s (host [ns][3]) with complex amplitudes amp (host [ns][2]);
 * one right-hand side. */
axs_status axs_incident_point_sources(axs_ctx *ctx, const double *src, const double *amp,
                                      int ns, void *v);

/* u[c][t] = sum_j G(x_t, x_j) w_j sigma[c][j] at nt targets tgt (host [nt][3]),
 * every body included (eq. "intHelm1" with the surface rule); FP64.
 * sigma : device [nrhs][N]; u : device complex128 [nrhs][nt]. */
axs_status axs_eval_field(axs_ctx *ctx, const void *sigma, int nrhs, const double *tgt, int nt,
                          void *u);

/* Far-field pattern u_inf(xh) with u ~ e^{i kappa |x|}/|x| u_inf:
 * u_inf = (1/4pi) sum_j (-i kappa xh.n_j + i eta) e^{-i kappa xh.x_j} w_j sigma_j.
 * xhat host [nd][3]; out device complex128 [nrhs][nd]. */
axs_status axs_far_field(axs_ctx *ctx, const void *sigma, int nrhs, const double *xhat, int nd,
                         void *out);

/* Kernel timing of the last axs_apply_* call on the context's stream (HIP events
 * around each stage), milliseconds: [0] inter-body sum, [1] forward DFT,
 * [2] modal applies, [3] inverse DFT (+ identity), [4] total.
 * Only filled when timing was enabled with axs_set_timing(ctx, 1). */
axs_status axs_set_timing(axs_ctx *ctx, int enable);
axs_status axs_last_timing(axs_ctx *ctx, double ms[5]);

/* Inter-body sum launch shape, per precision; 0 = library default for each field.
 *  variant: 1 = sources streamed as points, 2 = sources streamed as azimuthal rings
 *           in mirror pairs (azimuths l and N_F - l): per target and ring, R^2
 *           of a pair costs 3 FMAs and n.d one each (needs N_F/2 + 1 <= block),
 *           3 = MFMA order, kappa > 0: R^2 and n.d of 16 x 16 (source,
 *           target) blocks from matrix-core products of 4-vectors in the source
 *           body's frame; with 16 right-hand sides per group the complex
 *           multiply-accumulate is a matrix-core product too,
 *           4 = the MFMA order with the complex multiply-accumulate of each
 *           group of 16 right-hand sides on the FP16 matrix cores: kernel
 *           values and densities split into high and low FP16 parts (three
 *           of the four part products kept), scaled by powers of two into
 *           FP16 range, results in FP32 (FP32 only; needs kappa > 0 and
 *           bodies whose bounding balls are disjoint, from which the scale of
 *           the kernel values is bounded)
 *  targets_per_thread: 1, 2, 4 or 8 (variants 3 and 4: 1, 2 or 4 groups of 16
 *           targets per wavefront);  block: 128 or 256 threads (variants 3 and 4: 256);
 *  splits: number of source chunks per target tile (partial sums reduced in order).
 * Every shape computes the same sum; used by the launch-shape autotuner.
 * Shapes that do not fit the context are rejected (AXS_EINVAL) at the next
 * inter-body application, not here. */
axs_status axs_set_interbody_config(axs_ctx *ctx, int precision, int variant,
                                    int targets_per_thread, int block, int splits);

/* The launch shape an inter-body application in `precision` on nrhs right-hand
 * sides will use, defaults resolved: out[0..3] = variant, targets per thread
 * (variants 3 and 4: groups of 16 targets per wavefront), block, splits.  out:
 * host int[4].  The FP32 default is the ring order below 16 right-hand sides and
 * from 16 on the MFMA order with the FP16 multiply-accumulate (the FP32 MFMA
 * order where bounding balls overlap); the FP64 default is the ring order below
 * 16 and the MFMA order from 16 on.  AXS_ESTATE before axs_precompute_scattering;
 * AXS_EINVAL if the configured shape does not fit the context. */
axs_status axs_interbody_launch_shape(axs_ctx *ctx, int precision, int nrhs, int *out);

/* One GPU's share of the block rows (Sec. 3.3: the rows of A_pq for the bodies
 * p a GPU owns, against the sources of every other body q).  After
 * axs_set_target_bodies(ctx, first, count), axs_apply_interbody computes the
 * inter-body sum only for the targets of bodies [first, first + count), with
 * all sources as before (every other body, own body excluded); the rows of the
 * other bodies in its output are set to zero.  The default number of source
 * splits is chosen for the share's own tiles (so a share fills the GPU as the
 * full sum does); with the same launch shape set explicitly
 * (axs_set_interbody_config) its rows equal the full sum's bit for bit.  While
 * a range is set, the operators and solves that need every
 * row (axs_apply_matvec, axs_solve, axs_solve_skeleton) return AXS_ESTATE.
 * (0, 0) restores every body.  AXS_EINVAL for an empty or out-of-range range. */
axs_status axs_set_target_bodies(axs_ctx *ctx, int first_body, int count);

/* ------------------------------------------------------------------------
 * Skeletonization (Sec. 5, eqs. ip0-ip6): each off-diagonal block is factored
 * as U_p A_pq(I_p, I_q) V_q^* by interpolative decompositions, and GMRES runs on
 * the smaller system  s~ + S B~ s~ = -v~  with S_p = V_p^* A_pp^{-1} U_p,
 * v~_p = V_p^* A_pp^{-1} v_p, B~ the inter-body sum over the skeleton nodes;
 * the full density is s_p = -A_pp^{-1} (v_p + U_p (B~ s~)_p).  Skeletons are
 * whole rings (contour nodes with all their azimuthal nodes): U_p = X (x) I,
 * V_p^* = X^T (x) I with one X (NG x k) per shape from the row ID, over the
 * contour index, of the fields of combined-field sources on a proxy sphere at
 * the contour nodes and of the contour nodes' fields at two proxy spheres,
 * all Fourier modes stacked; so S_p is k x k per mode and B~ a ring-order sum.
 * ------------------------------------------------------------------------ */

/* Build the skeleton system after axs_precompute_scattering.
 *  eps          : relative tolerance of the IDs (pivoted Gram-Schmidt stops when
 *                 the pivot norm falls below eps x the first one), e.g. 1e-8.
 *  proxy_factor : proxy radius = min(proxy_factor x bounding radius, distance to
 *                 the nearest other body's bounding ball) over the bodies of a
 *                 shape; a shape whose proxy radius is below 1.05 x its bounding
 *                 radius keeps all its rings.  2.0 is typical.
 *  out_nskel    : host int64, number of skeleton nodes (may be NULL).
 * FP64 on the device; replaces an earlier skeleton system of the context. */
axs_status axs_skeletonize(axs_ctx *ctx, double eps, double proxy_factor, int64_t *out_nskel);

/* Point skeletons (Sec. 5 with index sets of single nodes; the remark of
 * Sec. 5 on randomized sampling): the row ID runs over the N_G N_F nodes of a
 * shape against the proxy matrix H[(i, l), (m, c)] = Hm[i, c] e^{i m theta_l},
 * m = -M..M, Hm = [IN_|m| | OUT_|m|^T] (the proxy fields of the ring version,
 * n_proxy polar points per proxy sphere), taken of the Gaussian sketch
 * Psi H^* (Psi: ell x (2M+1) 3 n_proxy, complex Gaussian, entry (s, r) the
 * conjugate of draw s (2M+1) 3 n_proxy + r of the generator below).  Nodes are
 * chosen by QR with randomized column pivoting of the sketch (blocks of 64
 * pivots, each block orthonormalised by CholeskyQR2 and projected out of the
 * rest twice); the rank k is the first pivot with |R_kk| < eps
 * |R_00|; ell starts at 256 for the first shape and at 1.25 k + 64 of the
 * shape before for each later one, and grows, by the decay of |R_jj| seen,
 * until k <= ell - 16.  Then U_p = V_p = X
 * (N_G N_F x k), S_p = X^T A_pp^{-1} X is dense k x k (FP64 and FP32 copies),
 * B~ is the inter-body sum over the skeleton nodes (the point order, or the
 * MFMA orders from 16 rhs), S_p and X^T are applied per body in one launch
 * over all bodies, and axs_solve_skeleton solves through it.
 *  eps, proxy_factor : as for axs_skeletonize; every shape needs a proxy
 *                 radius of at least 1.05 x its bounding radius (AXS_EINVAL).
 *  n_proxy      : polar proxy points per sphere, 0 for 40 + ceil(1.25 kappa R_p).
 *  seed         : the sketch's stream: uniform draw k is (splitmix64(seed *
 *                 0x632BE59BD9B4E019 + k) >> 11 + 0.5) 2^-53, complex Gaussian
 *                 draw e is sqrt(-2 ln u_2e) e^{2 pi i u_(2e+1)} (Box-Muller).
 *  out_nskel    : host int64, number of skeleton nodes (may be NULL).
 * FP64 on the device (rocBLAS for the dense products); replaces an earlier
 * skeleton system of the context. */
axs_status axs_skeletonize_points(axs_ctx *ctx, double eps, double proxy_factor, int n_proxy, uint64_t seed,
                                  int64_t *out_nskel);

/* Skeleton rings k and contour nodes NG of a body's shape (host ints); for
 * point skeletons the skeleton nodes k and the nodes N_G N_F of the shape. */
axs_status axs_skeleton_rank(axs_ctx *ctx, int body_id, int *rings, int *contour_nodes);

/* The skeleton nodes of a body as local node indices i N_F + l, ascending
 * (ring skeletons: every azimuthal node of each skeleton ring).  count (host
 * int) returns their number; nodes (host int array of *count entries on input,
 * or NULL to query the number) receives them.  AXS_EINVAL if *count is too small. */
axs_status axs_skeleton_nodes(axs_ctx *ctx, int body_id, int *count, int *nodes);

/* Point skeletons only (AXS_ESTATE otherwise): copies X^T of the body's shape,
 * k x N_G N_F column-major complex128 (column j = row j of X, rows in the order
 * of axs_skeleton_nodes), into xt (device, caller-allocated). */
axs_status axs_skeleton_interp(axs_ctx *ctx, int body_id, void *xt);

/* Solve through the skeleton system; incident and sigma as for axs_solve
 * (device complex128 [nrhs][N], full-size).  mode: AXS_SOLVE_FP64 or
 * AXS_SOLVE_MIXED for the GMRES on the compressed system, whose residual info
 * reports; with | AXS_SOLVE_CERTIFY, info reports instead the residual of the
 * lifted sigma in the full system (one FP64 application of I + D^{-1} B), which
 * also includes the skeletonization error. */
axs_status axs_solve_skeleton(axs_ctx *ctx, const void *incident, void *sigma, int nrhs, int mode,
                              double tol, int max_iters, axs_solve_info *info);

/* ------------------------------------------------------------------------ *
 * Learned warm start.  A multilayer perceptron maps (incident direction,
 * wavenumber) to an initial guess for axs_solve.  The guess is exact in its
 * single-body part and learned in the rest: by eq. "precond" the solution
 * satisfies sigma* = b~ - D^{-1} B sigma* with b~ = -D^{-1} v (the response of
 * each body alone to the incident wave, one preconditioner application), and
 * the network predicts the multiple-scattering part split by source body,
 *     sigma*_b - b~_b = sum_{b' != b} u^{b'}_b,   u^{b'}_b = -D_b^{-1} B_{bb'} sigma*_{b'},
 * each term with its leading phase phi_{bb'} = kappa (d.c_{b'} + |c_b - c_{b'}|)
 * (the incident wave at the centre of b' carried to the centre of b) taken
 * out and only its azimuthal modes |m| <= m_max kept.  It is trained on
 * solves of the method itself.  axs_solve keeps a guess only if its FP64
 * residual is below || b || (the zero guess otherwise).
 *
 * Warm-start layout, floats per right-hand side (axs_warm_start_size):
 *   for target body b (build order), source slot s = 0..B-2 (the other bodies
 *   b' in build order), contour node i, m = -m_max..m_max: (re, im) of
 *     Y = e^{-i phi_{bb'}} (1/N_F) sum_l u^{b'}_b(i, l) e^{-i m theta_l};
 *   P = 2 (B - 1) (2 m_max + 1) sum_b N_G(b).
 * ------------------------------------------------------------------------ */
typedef struct axs_mlp axs_mlp;

/* Network n_in -> width (x depth hidden layers, GELU) -> n_out (linear), FP32,
 * on ctx's device and stream, parameters zero until axs_mlp_set_params or
 * axs_mlp_train.  The network must be destroyed before its context.  Parameters
 * are packed layer by layer as [W_1 (n_in x width, row-major, input index
 * first), b_1, W_2, b_2, ...].  For the warm start n_in = 4 and n_out = P. */
axs_status axs_mlp_create(axs_ctx *ctx, int n_in, int width, int depth, int n_out, axs_mlp **out);
axs_status axs_mlp_destroy(axs_mlp *mlp);
axs_status axs_mlp_num_params(const axs_mlp *mlp, int64_t *count);
/* host float arrays of axs_mlp_num_params entries; set also resets the Adam state */
axs_status axs_mlp_set_params(axs_mlp *mlp, const float *host_params);
axs_status axs_mlp_get_params(axs_mlp *mlp, float *host_params);
/* Y = network(X); X device float [batch][n_in], Y device float [batch][n_out] */
axs_status axs_mlp_forward(axs_mlp *mlp, const float *X, float *Y, int batch);
/* mean squared error L = sum (Y - T)^2 / (batch n_out) and dL/dparams (device
 * float [num_params], may be NULL); loss may be NULL (else synchronises) */
axs_status axs_mlp_gradient(axs_mlp *mlp, const float *X, const float *T, int batch, double *loss,
                            float *grad);
/* one Adam step on the batch (bias-corrected moments) */
axs_status axs_mlp_adam_step(axs_mlp *mlp, const float *X, const float *T, int batch, double lr,
                             double beta1, double beta2, double eps, double *loss);
/* `steps` Adam steps over sample rows held on the device: step s gathers rows
 * order[s batch .. (s+1) batch - 1] of X (device float [rows][n_in]) and of T
 * (device float [rows][n_out]) into the network's own batch buffers and takes
 * the step of axs_mlp_adam_step with learning rate lr[s].  order (host int32
 * [steps x batch], each in [0, rows)) and lr (host double [steps], each > 0)
 * are checked and copied before the first step is queued, so the caller may
 * reuse them on return; a bad entry gives AXS_EINVAL with nothing queued.
 * Synchronises ctx's stream before and after the copy; loss (may be NULL, else
 * synchronises again) receives the last step's loss.  The result equals the
 * same steps taken one by one through axs_mlp_adam_step on gathered batches. */
axs_status axs_mlp_train_epoch(axs_mlp *mlp, const float *X, const float *T, int64_t rows, const int32_t *order,
                               int batch, int steps, const double *lr, double beta1, double beta2, double eps,
                               double *loss);

/* Train the warm-start network (n_in = 4) on S samples: X device float [S][4]
 * = (d_x, d_y, d_z, k) per sample, Y device float [S][n_out] its targets
 * (axs_warm_start_encode of the solution).  The library maps k to
 * (2k - (k_min + k_max)) / (k_max - k_min), divides Y by its root mean
 * square, initialises the parameters (He: W ~ N(0, 2 / fan_in), biases 0,
 * from a counter-based generator seeded by init_seed; init_seed < 0 keeps the
 * current network), and runs `epochs` epochs of Adam: each epoch a seeded
 * permutation (Fisher-Yates) of the samples in floor(S / batch) batches, the
 * learning rate decaying from lr to lr_final along a cosine over all steps;
 * at the end the target scale is folded into the last layer, so that
 * axs_mlp_forward returns Y-scaled outputs, and the Adam state is reset.
 * hparams: a JSON object of numbers with keys k_min, k_max (required),
 * epochs (200), batch (256), lr (1e-3), lr_final (1e-5), beta1 (0.9),
 * beta2 (0.999), eps (1e-8), seed (5), init_seed (4); anything else is
 * AXS_EINVAL.  loss_per_epoch: host double [epochs] receiving each epoch's
 * last-step loss on the scaled targets, or NULL.  Synchronous. */
axs_status axs_mlp_train(axs_mlp *mlp, const float *X, const float *Y, int64_t S, const char *hparams,
                         double *loss_per_epoch);

/* Initial guess sigma0 (device complex128 [nrhs][N]) for the plane waves dirs
 * (host [nrhs][3]) on ctx: sigma0 = b~ + decode(network(features)), with the
 * features (d, k mapped through k_range as in axs_mlp_train) at ctx's
 * wavenumber, b~ = -D^{-1} v computed by the library, and the decoding of the
 * warm-start layout above; m_max follows from the network's n_out (AXS_EINVAL
 * if n_out is not a warm-start size of ctx).  kappas (host [nrhs]) may be
 * NULL; if given, every entry must equal ctx's wavenumber (AXS_EINVAL).
 * k_range: host double[2], the training range.  mlp and ctx must be on one
 * device (they may use different streams).  Synchronous. */
axs_status axs_mlp_predict(axs_mlp *mlp, axs_ctx *ctx, const double *dirs, const double *kappas, int nrhs,
                           const double k_range[2], void *sigma0);

/* Floats per right-hand side of the warm-start layout, P (above).  AXS_EINVAL
 * for fewer than two bodies or m_max beyond a body's mode cutoff. */
axs_status axs_warm_start_size(axs_ctx *ctx, int mmax, int64_t *P);
/* Training targets: Y (device float [nrhs][P]) of the densities sigma (device
 * complex128 [nrhs][N], normally solutions of axs_solve for the plane waves
 * dirs, host [nrhs][3]): per source body b', the FP64 inter-body sum of sigma
 * restricted to b', -D^{-1} of it, then the layout's modes and phases.
 * Synchronous. */
axs_status axs_warm_start_encode(axs_ctx *ctx, const void *sigma, const double *dirs, int nrhs, int mmax,
                                 float *Y);
/* sigma (device complex128 [nrhs][N]) = the decoding of Y (device float
 * [nrhs][P]): sum over source slots and |m| <= m_max of e^{i phi_{bb'}} Y
 * e^{i m theta_l}.  With m_max = every body's M, decode(encode(x)) =
 * -D^{-1} B x for any x (the sum over sources is exact).  Synchronous. */
axs_status axs_warm_start_decode(axs_ctx *ctx, const float *Y, const double *dirs, int nrhs, int mmax,
                                 void *sigma);

#ifdef __cplusplus
}
#endif
#endif /* AXS_H */
