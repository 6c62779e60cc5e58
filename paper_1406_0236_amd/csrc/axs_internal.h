// Internal declarations of the axs library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <memory>
#include <vector>

#include "../../include/axs.h"
#include "worktable.h"

namespace axs {

// ---------------------------------------------------------------------------
// error handling: every HIP call is checked; failures become axs_status codes
// ---------------------------------------------------------------------------
struct Error {
    axs_status code;
    std::string msg;
};

#define AXS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::axs::Error{AXS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define AXS_REQUIRE(cond, code, text)                          \
    do {                                                       \
        if (!(cond)) throw ::axs::Error{(code), (text)};       \
    } while (0)

// ---------------------------------------------------------------------------
// device memory owned by a context
// ---------------------------------------------------------------------------
struct Ctx;

struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// ---------------------------------------------------------------------------
// geometry / shape tables
// ---------------------------------------------------------------------------
struct Shape {
    int n_panels = 0, p = 0, NG = 0, M = 0, NF = 0, Nt = 0;
    double kappa = 0, eta = 0;
    std::vector<double> r, z, dr, dz, gw;   // host, per contour node
    std::vector<int> bodies;                // body ids using this shape (build order)
    // device (owned by ctx buffers)
    double *A64 = nullptr;    // complex128 interleaved [M+1][NG][NG], A~_m row-major
    double *S64 = nullptr;    // complex128 interleaved [M+1][NG][NG], S_m row-major
    double *S64r = nullptr, *S64i = nullptr;   // planar, column-major [M+1][NG(k)][NG(i)]
    float *S32r = nullptr, *S32i = nullptr;    // same in FP32
    double *A64r = nullptr, *A64i = nullptr;   // planar A~_m (FP64), for the unpreconditioned operator
    int64_t xoff = 0;         // offset (in complex elements per rhs) of this shape's
                              // mode-major block in the DFT workspace
};

// per-body frame record on the device: centre[3], rotation[9] (row-major,
// global = centre + rot * local), bounding radius, 3 pad
constexpr int FRAME = 16;

struct Body {
    int shape = 0;
    int local = 0;            // index among the bodies of its shape
    double centre[3] = {0, 0, 0};
    double rot[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double bound_radius = 0;  // max |node - centre|
    int64_t offset = 0;       // first global node index
    int64_t n = 0;            // NG * NF
};

// Inter-body work item: one body-aligned target tile against up to two
// contiguous source ranges (everything outside the target's body, cut into
// `splits` chunks).  slot = chunk index; partial sums go to part[slot].

// Body descriptor used by the DFT kernels.  The DFT workspace holds, per
// shape, a mode-major block of columns (column-major, leading dimension NG):
// mode |m| owns nb*nrhs columns for m = 0 and 2*nb*nrhs otherwise; column
// (sgn*nb + local)*nrhs + c holds body `local`, rhs c, sign sgn (1 for -m).
// `xoff` is the shape block's element offset for nrhs = 1 (scale by nrhs).
struct BodyDev {
    int64_t offset;      // first global node
    int64_t xoff;
    int64_t twoff;       // offset of this body's N_F twiddle table
    int32_t NG, NF, M, nb;   // nb = bodies of this shape
    int32_t local, shape;
};

// Batched GEMM descriptor: Y = S_|m| X for one shape and mode, for nrhs = 1
// (column counts and offsets scale with nrhs).
struct GemmBatch {
    int64_t a_off;       // element offset of S_|m| (planar, column-major NG x NG)
    int64_t x_off;       // element offset of the column block for nrhs = 1
    int32_t NG, ncols;   // ncols for nrhs = 1
};

// skeleton descriptor of one body: its full and skeleton node offsets, contour
// nodes, skeleton rings, azimuthal nodes, offset of its shape's X (NG x k)
struct SkelBody {
    int64_t o0, s0, xoff;
    int32_t NG, k, NF, pad;
};
struct Skeleton;
struct PointSkel;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    axs_alloc_fn alloc = nullptr;
    axs_free_fn free_fn = nullptr;
    void *user = nullptr;
    std::string err;

    bool have_k = false;
    double kappa = 0, eta = 0;
    // single-layer coupling gamma of G = d phi/dn' + gamma phi: i eta for kappa > 0
    // (Sec. 2), eta at kappa = 0 (the Laplace equation of Sec. 6.1)
    double gam_re = 0, gam_im = 0;
    std::vector<Shape> shapes;
    std::vector<Body> bodies;
    int64_t N = 0;
    bool precomputed = false;

    // global node arrays (device); FP64 and FP32 SoA
    double *g64 = nullptr;    // [7][N]: x y z nx ny nz w
    float *g32 = nullptr;     // [6][N]: x y z nx ny nz
    std::vector<BodyDev> body_dev_host;
    BodyDev *body_dev = nullptr;
    double *tw64 = nullptr;   // per distinct NF: twiddles; indexed via twoff
    float *tw32 = nullptr;
    GemmBatch *gemm = nullptr;     // batched GEMM table (built at precompute)
    int ngemm = 0, gemm_max_cols = 0, max_NG = 0;

    // cached inter-body work tables, per precision (0 = fp64, 1 = fp32)
    // [precision][0: point / ring orders, 1: MFMA order (node units),
    // 2: MFMA order with the FP16 multiply-accumulate (32-node block units)],
    // so that alternating single and batched calls do not rebuild them
    IBWork *ib_work[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int ib_nwork[2][3] = {{0, 0, 0}, {0, 0, 0}};
    int ib_key[2][3][6] = {};   // launch shape and target range of the cached table

    // launch configuration of the inter-body sum (0 = library default)
    int ib_variant[2] = {0, 0};   // 1 = point sources, 2 = azimuthal rings, 3 = MFMA, 4 = MFMA + FP16 MAC (FP32)
    int ib_tpt[2] = {0, 0};       // targets per thread [fp64, fp32]
    int ib_block[2] = {0, 0};
    int ib_splits[2] = {0, 0};
    // target rows of the inter-body sum: bodies [tgt_first, tgt_first +
    // tgt_count), tgt_count < 0 = every body (axs_set_target_bodies)
    int tgt_first = 0, tgt_count = -1;

    // ring tables (one ring = one contour node of one body = its N_F azimuthal nodes)
    int nrings = 0;
    std::vector<int64_t> ring_base;      // first ring id of each body
    int32_t *ring_i = nullptr;           // [3][nrings]: node offset, N_F, body; [nrings + 1]: first mirror-pair entry
    int2 *ring_pair = nullptr;           // [entries]: node of azimuth e, node of N_F - e (-1: none)
    double *ring_g64 = nullptr;          // [5][nrings]: r, z, n_r, n_z, -n_r / (2 r)
    float *ring_g32 = nullptr;
    double *frame64 = nullptr;           // [B][FRAME]: centre, rotation (row-major), bound radius
    float *frame32 = nullptr;
    double *cs64 = nullptr;              // [2][N]: cos, sin of each node's azimuth
    float *cs32 = nullptr;
    int max_nf = 0;
    // MFMA source order (FP32, kappa > 0): per node, in its body's frame,
    // [0, N): (k/2pi)^2 (-2y, |y|^2); [N, 2N): (k/2pi)^3 (n, -n.y)
    float *mf_src = nullptr;
    double *mf_src64 = nullptr;          // the same in FP64
    int64_t *body_off = nullptr;         // [B + 1]: first node of each body, then N
    // 32-node source blocks of the FP16 multiply-accumulate: first block of each
    // body (the last block of a body padded), and the power of two that scales
    // the kernel values into FP16 range (mf16_gexp; mf16_ok is false where no
    // bound applies, i.e. where bounding balls of two bodies overlap)
    int32_t *blk_off = nullptr;          // [B + 1]
    int64_t nblk = 0;
    int mf16_gexp = 0;
    bool mf16_ok = false;
    double2 *sctab = nullptr;            // [1024]: (cos, sin)(2 pi k / 1024) for the FP64 sin/cos
    // every body's diameter is under 127 wavelengths, so the phase less the
    // per-(wavefront, source body) whole revolutions floor(min (|p| - r_b) k/2pi)
    // stays inside the hardware sin/cos input range (ring and MFMA orders rely on it)
    bool near_phase_ok = false;
    // no ring tables (the child context of point skeletons): the ring order
    // is never chosen
    bool no_rings = false;
    // every node pair is under 255 wavelengths apart (the point order then
    // passes FP32 phases to the hardware sin/cos without a fraction step)
    bool scene_phase_ok = false;

    // skeletonization (Sec. 5): the compressed system and its factors
    std::unique_ptr<Skeleton> skel;
    // set in the child context of point skeletons: its operator is
    // s~ + S B~ s~ with dense S_p (the parent's skeleton owns the factors)
    const PointSkel *pop = nullptr;
    // rocBLAS handle bound to the stream (dense products of the point skeletons)
    void *blas = nullptr;

    // timing
    bool timing = false;
    hipEvent_t ev[6] = {};
    double last_ms[5] = {0, 0, 0, 0, 0};

    // device allocations owned by the context
    std::vector<void *> owned;
    // named scratch buffers (grow-only)
    Buffer ws[19];
    // while `arena` is set, scratch() hands out slices of that caller-supplied
    // region instead (one slice per slot, bump order) and allocates nothing
    char *arena = nullptr;
    size_t arena_cap = 0, arena_top = 0;
    void *arena_slot[19] = {};
    size_t arena_slot_bytes[19] = {};

    void *dalloc(size_t bytes);
    void dfree(void *p);
    void *scratch(int slot, size_t bytes);
    ~Ctx();
};

enum ScratchSlot {
    WS_Q = 0,        // staged densities q (R2 [nrhs][N])
    WS_PART = 1,     // inter-body partial sums (R2 [splits][nrhs][N])
    WS_XR = 2,       // DFT workspace (planar re)
    WS_XI = 3,       // DFT workspace (planar im)
    WS_YR = 4,
    WS_YI = 5,
    WS_WORK = 6,     // inter-body work table
    WS_TMP = 7,      // complex128 temporaries [nrhs][N]
    WS_TMP2 = 8,
    WS_KRYLOV = 9,   // Krylov bases
    WS_RED = 10,     // reduction partials
    WS_GEMM = 11,    // gemm batch table
    WS_MISC = 12,
    WS_TMP3 = 13,
    WS_KRYLOV2 = 14,
    WS_EVAL = 15,
    WS_Q16 = 16,     // FP16 density planes of the FP16 multiply-accumulate
    WS_QMAX = 17,    // per-rhs max |q| (float bits), then the per-slice partial maxima
    WS_FLAG = 18,    // one int: set when an input vector holds NaN or Inf
};

// Point skeletons: per shape k skeleton nodes of its n = NG NF nodes, the
// interpolation matrix as X^T (k x n, column-major: column j holds row j of X,
// columns of X in ascending skeleton node order) and S_p = X^T A_pp^{-1} X
// (k x k, column-major) in FP64 and FP32; bodies grouped in runs of
// consecutive bodies of one shape (one batched product per run)
struct PointRun {
    int shape, first, nb, k, n;
    int64_t o0, s0;                      // first full node and first skeleton node of the run
};
// 256 rows of one body's dense m x K block (column-major, ld m) times the
// body's K-vector of every rhs: the work item of the per-body products of
// point skeletons (S_p in the skeleton system, X^T in the restriction)
struct BodyMatItem {
    const float2 *A32;                   // complex64 copy of the block, or null
    const double2 *A64;                  // complex128
    int64_t in0, out0;                   // the body's first entry in the input and output vectors
    int m, K, row0, pad;
};

struct PointSkel {
    std::vector<int> k, n, ell;          // per shape: skeleton nodes, nodes, sketch width used
    std::vector<double> R_p;             // per shape: proxy radius
    std::vector<std::vector<int>> nodes; // per shape: ascending local node indices
    std::vector<double2 *> XT;           // per shape (device)
    std::vector<double2 *> S64;
    std::vector<float2 *> S32;
    std::vector<PointRun> runs;
    BodyMatItem *sp_items = nullptr;     // device: S_p per skeleton body
    BodyMatItem *rs_items = nullptr;     // device: X^T per body (full -> skeleton)
    int n_sp = 0, n_rs = 0;
};

struct Skeleton {
    int kind = 0;                        // 0: whole rings, 1: single nodes
    std::unique_ptr<Ctx> child;          // skeleton of every body: rings with S~_m = X^T S_m X, or nodes
    double2 *X = nullptr;                // rings: per shape NG x k (row-major, columns by ascending ring)
    SkelBody *desc = nullptr;            // rings: [bodies]
    std::vector<int> rank;               // skeleton rings (nodes) per shape
    std::vector<std::vector<int>> rings; // rings: ascending skeleton rings per shape
    int64_t Ns = 0;                      // skeleton nodes
    double eps = 0;
    std::unique_ptr<PointSkel> pts;      // nodes: the factors
};

// ---------------------------------------------------------------------------
// launches (defined in the .hip files)
// ---------------------------------------------------------------------------
// setup.hip
void precompute_shape(Ctx &c, Shape &s);   // A~_m of one shape
void invert_shapes(Ctx &c);                 // S_m = A~_m^{-1} of every shape
void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w);
// k^G_m w (m = 0..M) for arbitrary (target ring, source ring) pairs: host arrays
// pts[7][P] = (r_t, r_s, r_s - r_t, z_s - z_t, n_r, n_z of the source, weight);
// result on the device, [P][M+1]
void modal_values(Ctx &c, double kappa, double gam_re, double gam_im, int M, int Nt,
                  const std::vector<double> &pts, int64_t P, double2 *kout);
// api.hip
void finish_precompute(Ctx &c);
// interbody.hip
void interbody_partials(Ctx &c, const void *sigma, int nrhs, int prec);   // -> WS_PART
// bytes of scratch the inter-body sum takes in `prec` with nrhs rhs (staged
// densities, partial sums, and the work table where it is not cached), each
// rounded up to 256; -1 for the MFMA orders (variants 3 and 4)
int64_t interbody_scratch_bytes(Ctx &c, int prec, int nrhs);
void interbody_reduce_to_c128(Ctx &c, void *y, int nrhs, int prec, bool add = false);  // WS_PART -> (+)y
int interbody_splits(Ctx &c, int prec, int nrhs);
void eval_field_launch(Ctx &c, const void *sigma, int nrhs, const double *tgt_dev, int nt,
                       void *u);
void far_field_launch(Ctx &c, const void *sigma, int nrhs, const double *xh_dev, int nd,
                      void *u);
void incident_plane_launch(Ctx &c, const double *dirs_dev, int nrhs, void *v);
void incident_point_launch(Ctx &c, const double *src_dev, const double *amp_dev, int ns, void *v);
// modal.hip
// forward DFT from partial sums (src = 0) or from a complex128 vector (src = 1)
void dft_forward(Ctx &c, int prec, int from_vec, const void *vec, int nrhs, int splits);
// per-mode products with S_m = A~_m^{-1}, or with A~_m itself (forward = true, FP64)
void modal_gemm(Ctx &c, int prec, int nrhs, bool forward = false);
// y = alpha * sigma + beta * inverse DFT
void dft_inverse(Ctx &c, int prec, const void *sigma, double alpha, double beta, void *y,
                 int nrhs);
// skeleton.hip
void skeletonize(Ctx &c, double eps, double proxy_factor);
// point skeletons: n_proxy polar proxy points per sphere (0: 40 + ceil(1.25 kappa R_p)),
// seed of the Gaussian sketch
void skeletonize_points(Ctx &c, double eps, double proxy_factor, int n_proxy, uint64_t seed);
void point_operator(Ctx &c, const void *sigma, void *y, int nrhs, int prec);   // child: y = s + S B~ s
void release_skeleton(Ctx &c);           // frees the parent-side factors of c.skel
void destroy_blas(Ctx &c);
void skel_restrict(Ctx &c, const void *y, void *out, int nrhs, double alpha);      // out = alpha (X^T (x) I) y
void skel_prolong(Ctx &c, const void *w, const void *add, void *out, int nrhs);   // out = add + (X (x) I) w
double skel_sumsq(Ctx &c, const double2 *a, int64_t n);
double skel_residual_sumsq(Ctx &c, const double2 *a, const double2 *b, int64_t n);   // sum |a + b|^2
// krylov.hip
// b_given: the right-hand side b itself (instead of b = -D^{-1} incident)
axs_status solve_impl(Ctx &c, const void *incident, const void *sigma0, void *sigma, int nrhs,
                      int mode, double tol, int max_iters, axs_solve_info *info,
                      const void *b_given = nullptr);
// api-level helpers
void apply_operator(Ctx &c, const void *sigma, void *y, int nrhs, int prec);  // y = sigma + D^-1 B sigma
void apply_precond(Ctx &c, const void *x, void *y, int nrhs, int prec, double beta);  // y = beta D^-1 x
void apply_unpreconditioned(Ctx &c, const void *x, void *y, int nrhs);  // y = (D + B) x, FP64

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// AXS_ENONFINITE if any of the n complex128 values at v (device) is NaN or Inf;
// synchronises the context's stream
void require_finite(Ctx &c, const void *v, int64_t n, const char *what);

}  // namespace axs
