// C ABI entry points (include/axs.h): argument checks, context state, memory
// ownership, and the composition of the operator from the kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "axs_internal.h"

namespace axs {

void gauss_legendre_public(int n, std::vector<double> &x, std::vector<double> &w);
void split_planar(Ctx &c, Shape &s, const double *src, double *r64, double *i64, float *r32, float *i32);
void build_ring_tables(Ctx &c);
void interbody_shape(Ctx &c, int prec, int nrhs, int out[4]);

void *Ctx::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (alloc) {
        p = alloc(bytes, user);
        AXS_REQUIRE(p != nullptr, AXS_ENOMEM, "device allocation failed (caller allocator)");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        AXS_REQUIRE(e == hipSuccess && p, AXS_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    owned.push_back(p);
    return p;
}

void Ctx::dfree(void *p) {
    if (!p) return;
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it != owned.end()) owned.erase(it);
    if (free_fn)
        free_fn(p, user);
    else
        (void)hipFree(p);
}

void *Ctx::scratch(int slot, size_t bytes) {
    if (arena) {
        if (arena_slot[slot] && bytes <= arena_slot_bytes[slot]) return arena_slot[slot];
        const size_t need = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        AXS_REQUIRE(arena_top + need <= arena_cap, AXS_EINVAL, "static scratch exhausted");
        arena_slot[slot] = arena + arena_top;
        arena_slot_bytes[slot] = need;
        arena_top += need;
        return arena_slot[slot];
    }
    Buffer &b = ws[slot];
    if (bytes > b.bytes) {
        if (b.ptr) {
            AXS_HIP(hipStreamSynchronize(stream));   // the old buffer may still be in use
            dfree(b.ptr);
        }
        b.ptr = dalloc(bytes);
        b.bytes = bytes;
    }
    return b.ptr;
}

Ctx::~Ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    skel.reset();   // the child context first (it borrows this context's tables)
    destroy_blas(*this);
    for (void *p : std::vector<void *>(owned)) dfree(p);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
}

// p[0..n) = value (a kernel, not a memset, so that graph-captured callers record no memset node)
__global__ void fill_int_kernel(int *__restrict__ p, int n, int value) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = value;
}

// flag = 1 if any component of v[0..n) is NaN or Inf (integer OR, order-free)
__global__ void nonfinite_kernel(const double2 *__restrict__ v, int64_t n, int *__restrict__ flag) {
    int bad = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = v[t];
        bad |= !(isfinite(a.x) && isfinite(a.y));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

void require_finite(Ctx &c, const void *v, int64_t n, const char *what) {
    int *flag = (int *)c.scratch(WS_FLAG, sizeof(int));
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, c.stream, flag, 1, 0);
    AXS_HIP(hipGetLastError());
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(n, 256)));
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nblk), dim3(256), 0, c.stream, (const double2 *)v, n, flag);
    AXS_HIP(hipGetLastError());
    int host = 0;
    AXS_HIP(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));
    AXS_REQUIRE(host == 0, AXS_ENONFINITE, std::string("non-finite value (NaN or Inf) in ") + what);
}

// ---------------------------------------------------------------------------
// operator composition
// ---------------------------------------------------------------------------
static void rec(Ctx &c, int k) {
    if (c.timing) AXS_HIP(hipEventRecord(c.ev[k], c.stream));
}

static void finish_timing(Ctx &c, bool with_ib) {
    if (!c.timing) return;
    AXS_HIP(hipEventSynchronize(c.ev[4]));
    float ms = 0;
    for (int k = 0; k < 4; ++k) {
        if (k == 0 && !with_ib) {
            c.last_ms[0] = 0;
            continue;
        }
        AXS_HIP(hipEventElapsedTime(&ms, c.ev[k], c.ev[k + 1]));
        c.last_ms[k] = ms;
    }
    AXS_HIP(hipEventElapsedTime(&ms, c.ev[with_ib ? 0 : 1], c.ev[4]));
    c.last_ms[4] = ms;
}

void apply_operator(Ctx &c, const void *sigma, void *y, int nrhs, int prec) {
    if (c.pop) {   // the compressed system of point skeletons
        point_operator(c, sigma, y, nrhs, prec);
        return;
    }
    rec(c, 0);
    interbody_partials(c, sigma, nrhs, prec);
    rec(c, 1);
    dft_forward(c, prec, 0, nullptr, nrhs, interbody_splits(c, prec, nrhs));
    rec(c, 2);
    modal_gemm(c, prec, nrhs);
    rec(c, 3);
    dft_inverse(c, prec, sigma, 1.0, 1.0, y, nrhs);
    rec(c, 4);
    finish_timing(c, true);
}

// y = (D + B) x in FP64: per-body DFT, A~_m products, inverse DFT, plus the
// inter-body sum (the system matrix A of Sec. 3.3 without the preconditioner)
void apply_unpreconditioned(Ctx &c, const void *x, void *y, int nrhs) {
    rec(c, 0);
    interbody_partials(c, x, nrhs, AXS_FP64);
    rec(c, 1);
    dft_forward(c, AXS_FP64, 1, x, nrhs, 0);
    rec(c, 2);
    modal_gemm(c, AXS_FP64, nrhs, true);
    rec(c, 3);
    dft_inverse(c, AXS_FP64, nullptr, 0.0, 1.0, y, nrhs);
    interbody_reduce_to_c128(c, y, nrhs, AXS_FP64, true);
    rec(c, 4);
    finish_timing(c, true);
}

void apply_precond(Ctx &c, const void *x, void *y, int nrhs, int prec, double beta) {
    rec(c, 1);
    dft_forward(c, prec, 1, x, nrhs, 0);
    rec(c, 2);
    modal_gemm(c, prec, nrhs);
    rec(c, 3);
    dft_inverse(c, prec, nullptr, 0.0, beta, y, nrhs);
    rec(c, 4);
    finish_timing(c, false);
}

// ---------------------------------------------------------------------------
// precompute: shapes, global node arrays, tables
// ---------------------------------------------------------------------------
static void precompute_all(Ctx &c) {
    AXS_REQUIRE(!c.bodies.empty(), AXS_ESTATE, "no bodies");
    for (auto &s : c.shapes) precompute_shape(c, s);
    invert_shapes(c);
    finish_precompute(c);
}

// everything after the per-shape matrices: GEMM operands, DFT layout, node
// arrays, ring tables (also used for the skeleton context, whose S_m are given)
void finish_precompute(Ctx &c) {
    // planar copies of all S_m in one allocation per precision (GEMM operands)
    int64_t total = 0;
    std::vector<int64_t> soff(c.shapes.size());
    for (size_t k = 0; k < c.shapes.size(); ++k) {
        soff[k] = total;
        total += (int64_t)(c.shapes[k].M + 1) * c.shapes[k].NG * c.shapes[k].NG;
    }
    double *r64 = (double *)c.dalloc(total * sizeof(double));
    double *i64 = (double *)c.dalloc(total * sizeof(double));
    float *r32 = (float *)c.dalloc(total * sizeof(float));
    float *i32 = (float *)c.dalloc(total * sizeof(float));
    // the same layout for A~_m itself (FP64), used only by the unpreconditioned operator
    bool have_A = true;
    for (auto &s : c.shapes) have_A = have_A && s.A64 != nullptr;
    double *ar64 = have_A ? (double *)c.dalloc(total * sizeof(double)) : nullptr;
    double *ai64 = have_A ? (double *)c.dalloc(total * sizeof(double)) : nullptr;
    for (size_t k = 0; k < c.shapes.size(); ++k) {
        Shape &s = c.shapes[k];
        s.S64r = r64 + soff[k];
        s.S64i = i64 + soff[k];
        s.S32r = r32 + soff[k];
        s.S32i = i32 + soff[k];
        split_planar(c, s, s.S64, s.S64r, s.S64i, s.S32r, s.S32i);
        if (have_A) {
            s.A64r = ar64 + soff[k];
            s.A64i = ai64 + soff[k];
            split_planar(c, s, s.A64, s.A64r, s.A64i, nullptr, nullptr);
        }
    }
    // DFT workspace layout per shape and the batched GEMM table
    std::vector<GemmBatch> gb;
    int64_t xo = 0;
    c.max_NG = 0;
    c.gemm_max_cols = 0;
    for (size_t k = 0; k < c.shapes.size(); ++k) {
        Shape &s = c.shapes[k];
        s.xoff = xo;
        const int nb = (int)s.bodies.size();
        for (int m = 0; m <= s.M; ++m) {
            GemmBatch g;
            g.a_off = soff[k] + (int64_t)m * s.NG * s.NG;
            g.x_off = xo + (int64_t)nb * (m == 0 ? 0 : 2 * m - 1) * s.NG;
            g.NG = s.NG;
            g.ncols = nb * (m == 0 ? 1 : 2);
            gb.push_back(g);
            c.gemm_max_cols = std::max(c.gemm_max_cols, g.ncols);
        }
        xo += (int64_t)nb * s.NF * s.NG;
        c.max_NG = std::max(c.max_NG, s.NG);
    }
    c.gemm = (GemmBatch *)c.dalloc(gb.size() * sizeof(GemmBatch));
    AXS_HIP(hipMemcpy(c.gemm, gb.data(), gb.size() * sizeof(GemmBatch), hipMemcpyHostToDevice));
    c.ngemm = (int)gb.size();
    // twiddles per distinct N_F
    std::map<int, int64_t> twoff;
    std::vector<double> tw;
    for (auto &s : c.shapes) {
        if (twoff.count(s.NF)) continue;
        twoff[s.NF] = (int64_t)tw.size() / 2;
        for (int j = 0; j < s.NF; ++j) {
            // cos, sin of 2 pi j / NF, reduced to the first octant-free form j/NF in [0, 1)
            const double a = 2.0 * M_PI * j / s.NF;
            tw.push_back(std::cos(a));
            tw.push_back(std::sin(a));
        }
    }
    c.tw64 = (double *)c.dalloc(tw.size() * sizeof(double));
    c.tw32 = (float *)c.dalloc(tw.size() * sizeof(float));
    std::vector<float> tw32(tw.begin(), tw.end());
    AXS_HIP(hipMemcpy(c.tw64, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(c.tw32, tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice));
    // body descriptors
    c.body_dev_host.clear();
    for (auto &b : c.bodies) {
        const Shape &s = c.shapes[b.shape];
        BodyDev d{};
        d.offset = b.offset;
        d.xoff = s.xoff;
        d.twoff = twoff[s.NF];
        d.NG = s.NG;
        d.NF = s.NF;
        d.M = s.M;
        d.nb = (int)s.bodies.size();
        d.local = b.local;
        d.shape = b.shape;
        c.body_dev_host.push_back(d);
    }
    c.body_dev = (BodyDev *)c.dalloc(c.body_dev_host.size() * sizeof(BodyDev));
    AXS_HIP(hipMemcpy(c.body_dev, c.body_dev_host.data(), c.body_dev_host.size() * sizeof(BodyDev),
                      hipMemcpyHostToDevice));
    // global node arrays, FP64 (7 x N) and FP32 (6 x N)
    const int64_t N = c.N;
    std::vector<double> g(7 * N);
    for (auto &b : c.bodies) {
        const Shape &s = c.shapes[b.shape];
        for (int i = 0; i < s.NG; ++i) {
            const double sp = std::hypot(s.dr[i], s.dz[i]);
            const double nr = -s.dz[i] / sp, nz = s.dr[i] / sp;
            const double w = (2.0 * M_PI / s.NF) * s.r[i] * sp * s.gw[i];
            for (int l = 0; l < s.NF; ++l) {
                const double th = 2.0 * M_PI * l / s.NF;
                const double ct = std::cos(th), st = std::sin(th);
                const double loc[3] = {s.r[i] * ct, s.r[i] * st, s.z[i]};
                const double nl[3] = {nr * ct, nr * st, nz};
                const int64_t j = b.offset + (int64_t)i * s.NF + l;
                for (int a = 0; a < 3; ++a) {
                    double xv = b.centre[a], nv = 0;
                    for (int q = 0; q < 3; ++q) {
                        xv += b.rot[3 * a + q] * loc[q];
                        nv += b.rot[3 * a + q] * nl[q];
                    }
                    g[a * N + j] = xv;
                    g[(3 + a) * N + j] = nv;
                }
                g[6 * N + j] = w;
            }
        }
    }
    std::vector<float> g32(g.begin(), g.begin() + 6 * N);
    c.g64 = (double *)c.dalloc(7 * N * sizeof(double));
    c.g32 = (float *)c.dalloc(6 * N * sizeof(float));
    AXS_HIP(hipMemcpy(c.g64, g.data(), 7 * N * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(c.g32, g32.data(), 6 * N * sizeof(float), hipMemcpyHostToDevice));
    build_ring_tables(c);
    AXS_HIP(hipStreamSynchronize(c.stream));
    c.precomputed = true;
}

// ---------------------------------------------------------------------------
// Scratch of the no-allocation operator (axs_apply_matvec_noalloc): a
// file-scope device array, NOALLOC_BYTES on every device the library runs on,
// held until the process ends.  Host code never uses the array's name as an
// address: at set-up (axs_create, once per device, with that device current)
// its device address is taken with hipGetSymbolAddress and kept per device.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = (size_t)256 << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on the current device `device`; hipSuccess or the error
static hipError_t setup_static_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = p;
    return e;
}

static void *static_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < MAX_DEVICES ? g_scratch_ptr[device] : nullptr;
}

// scratch() draws from the static array for the lifetime of this object
struct ArenaScope {
    Ctx &c;
    ArenaScope(Ctx &c_, void *base, size_t cap) : c(c_) {
        c.arena = (char *)base;
        c.arena_cap = cap;
        c.arena_top = 0;
        for (int k = 0; k < 19; ++k) {
            c.arena_slot[k] = nullptr;
            c.arena_slot_bytes[k] = 0;
        }
    }
    ~ArenaScope() { c.arena = nullptr; }
};

}  // namespace axs

using axs::Ctx;
using axs::Error;

struct axs_ctx {
    Ctx c;
};

template <class F>
static axs_status guarded(axs_ctx *ctx, F &&f) {
    if (!ctx) return AXS_EINVAL;
    ctx->c.err.clear();
    try {
        {
            int cur = -1;
            if (hipGetDevice(&cur) == hipSuccess && cur != ctx->c.device) (void)hipSetDevice(ctx->c.device);
        }
        return f(ctx->c);
    } catch (const Error &e) {
        ctx->c.err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->c.err = "host allocation failed";
        return AXS_ENOMEM;
    } catch (const std::exception &e) {
        ctx->c.err = e.what();
        return AXS_EINVAL;
    }
}

extern "C" {

axs_status axs_create(axs_ctx **out, int device, void *hip_stream, axs_alloc_fn alloc, axs_free_fn free_fn,
                      void *user) {
    if (!out) return AXS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return AXS_EINVAL;
    if ((alloc == nullptr) != (free_fn == nullptr)) return AXS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return AXS_EHIP;
    axs_ctx *ctx = new (std::nothrow) axs_ctx();
    if (!ctx) return AXS_ENOMEM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    ctx->c.alloc = alloc;
    ctx->c.free_fn = free_fn;
    ctx->c.user = user;
    for (auto &e : ctx->c.ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            delete ctx;
            return AXS_EHIP;
        }
    }
    if (axs::setup_static_scratch(device) != hipSuccess) {
        delete ctx;
        return AXS_EHIP;
    }
    *out = ctx;
    return AXS_OK;
}

axs_status axs_destroy(axs_ctx *ctx) {
    if (!ctx) return AXS_EINVAL;
    (void)hipSetDevice(ctx->c.device);
    delete ctx;
    return AXS_OK;
}

const char *axs_last_error(const axs_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

axs_status axs_build_body(axs_ctx *ctx, const double *rz, const double *drz, const double *gw, int n_panels, int p,
                          double kappa, double eta, int M, const double centre[3], const double rot[9],
                          int *body_id) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(!c.precomputed, AXS_ESTATE, "bodies cannot be added after axs_precompute_scattering");
        AXS_REQUIRE(rz && drz && gw && centre && rot && body_id, AXS_EINVAL, "null pointer argument");
        AXS_REQUIRE(n_panels >= 1 && p >= 2 && p <= 16, AXS_EINVAL, "need n_panels >= 1 and 2 <= p <= 16");
        AXS_REQUIRE(M >= 0 && M <= 255, AXS_EINVAL, "mode cutoff M must be in [0, 255]");
        AXS_REQUIRE(std::isfinite(kappa) && kappa >= 0 && std::isfinite(eta), AXS_EINVAL,
                    "kappa must be finite and >= 0, eta finite");
        if (c.have_k)
            AXS_REQUIRE(kappa == c.kappa && eta == c.eta, AXS_EINVAL,
                        "all bodies of a context must share kappa and eta");
        const int NG = n_panels * p;
        for (int i = 0; i < 2 * NG; ++i)
            AXS_REQUIRE(std::isfinite(rz[i]) && std::isfinite(drz[i]), AXS_ENONFINITE, "non-finite contour data");
        for (int i = 0; i < 9; ++i) AXS_REQUIRE(std::isfinite(rot[i]), AXS_ENONFINITE, "non-finite rotation");
        for (int i = 0; i < 3; ++i) AXS_REQUIRE(std::isfinite(centre[i]), AXS_ENONFINITE, "non-finite centre");
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = 0;
                for (int k = 0; k < 3; ++k) d += rot[3 * a + k] * rot[3 * b + k];
                AXS_REQUIRE(std::fabs(d - (a == b ? 1.0 : 0.0)) < 1e-10, AXS_EINVAL, "rot is not orthonormal");
            }
        std::vector<double> sx, sw;
        axs::gauss_legendre_public(p, sx, sw);
        for (int i = 0; i < NG; ++i) {
            AXS_REQUIRE(rz[2 * i] > 0, AXS_EINVAL, "contour nodes must have r > 0");
            AXS_REQUIRE(std::hypot(drz[2 * i], drz[2 * i + 1]) > 0, AXS_EINVAL, "degenerate contour derivative");
            AXS_REQUIRE(std::fabs(gw[i] - sw[i % p]) < 1e-12, AXS_EINVAL,
                        "gw does not match the p-point Gauss-Legendre weights");
        }
        // shape dedupe
        int sid = -1;
        for (size_t k = 0; k < c.shapes.size(); ++k) {
            const auto &s = c.shapes[k];
            if (s.NG != NG || s.p != p || s.M != M) continue;
            bool same = true;
            for (int i = 0; i < NG && same; ++i)
                same = s.r[i] == rz[2 * i] && s.z[i] == rz[2 * i + 1] && s.dr[i] == drz[2 * i] &&
                       s.dz[i] == drz[2 * i + 1] && s.gw[i] == gw[i];
            if (same) {
                sid = (int)k;
                break;
            }
        }
        if (sid < 0) {
            axs::Shape s;
            s.n_panels = n_panels;
            s.p = p;
            s.NG = NG;
            s.M = M;
            s.NF = 2 * M + 1;
            s.kappa = kappa;
            s.eta = eta;
            for (int i = 0; i < NG; ++i) {
                s.r.push_back(rz[2 * i]);
                s.z.push_back(rz[2 * i + 1]);
                s.dr.push_back(drz[2 * i]);
                s.dz.push_back(drz[2 * i + 1]);
                s.gw.push_back(gw[i]);
            }
            c.shapes.push_back(s);
            sid = (int)c.shapes.size() - 1;
        }
        axs::Body b;
        b.shape = sid;
        std::copy(centre, centre + 3, b.centre);
        std::copy(rot, rot + 9, b.rot);
        double rad = 0;
        for (int i = 0; i < NG; ++i) rad = std::max(rad, std::hypot(rz[2 * i], rz[2 * i + 1]));
        b.bound_radius = rad;
        for (const auto &o : c.bodies) {
            const double d = std::sqrt((o.centre[0] - centre[0]) * (o.centre[0] - centre[0]) +
                                       (o.centre[1] - centre[1]) * (o.centre[1] - centre[1]) +
                                       (o.centre[2] - centre[2]) * (o.centre[2] - centre[2]));
            AXS_REQUIRE(d > o.bound_radius + rad, AXS_EINVAL, "bodies overlap (bounding balls intersect)");
        }
        b.offset = c.N;
        b.n = (int64_t)NG * (2 * M + 1);
        AXS_REQUIRE(c.N + b.n < (int64_t)1 << 31, AXS_EINVAL, "more than 2^31 unknowns");
        b.local = (int)c.shapes[sid].bodies.size();
        c.shapes[sid].bodies.push_back((int)c.bodies.size());
        c.bodies.push_back(b);
        c.N += b.n;
        c.have_k = true;
        c.kappa = kappa;
        c.eta = eta;
        c.gam_re = kappa > 0 ? 0.0 : eta;
        c.gam_im = kappa > 0 ? eta : 0.0;
        *body_id = (int)c.bodies.size() - 1;
        return AXS_OK;
    });
}

axs_status axs_precompute_scattering(axs_ctx *ctx) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(!c.precomputed, AXS_ESTATE, "already precomputed");
        AXS_REQUIRE(!c.bodies.empty(), AXS_ESTATE, "no bodies");
        axs::precompute_all(c);
        return AXS_OK;
    });
}

axs_status axs_num_unknowns(const axs_ctx *ctx, int64_t *N) {
    if (!ctx || !N) return AXS_EINVAL;
    *N = ctx->c.N;
    return AXS_OK;
}

axs_status axs_node_geometry(axs_ctx *ctx, double *out) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(out, AXS_EINVAL, "null output");
        std::vector<double> g(7 * c.N);
        AXS_HIP(hipMemcpy(g.data(), c.g64, g.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < c.N; ++j)
            for (int a = 0; a < 7; ++a) out[7 * j + a] = g[a * c.N + j];
        return AXS_OK;
    });
}

axs_status axs_modal_matrices(axs_ctx *ctx, int body_id, int which, void *out) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(body_id >= 0 && body_id < (int)c.bodies.size(), AXS_EINVAL, "bad body id");
        AXS_REQUIRE(which == 0 || which == 1, AXS_EINVAL, "which must be 0 (A~) or 1 (S)");
        AXS_REQUIRE(out, AXS_EINVAL, "null output");
        const auto &s = c.shapes[c.bodies[body_id].shape];
        const size_t bytes = (size_t)(s.M + 1) * s.NG * s.NG * 2 * sizeof(double);
        AXS_HIP(hipMemcpyAsync(out, which == 0 ? s.A64 : s.S64, bytes, hipMemcpyDeviceToDevice, c.stream));
        return AXS_OK;
    });
}

static axs_status check_apply(Ctx &c, const void *a, const void *b, int nrhs, int prec) {
    AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
    AXS_REQUIRE(a && b, AXS_EINVAL, "null vector");
    AXS_REQUIRE(nrhs >= 1 && nrhs <= 4096, AXS_EINVAL, "nrhs must be in [1, 4096]");
    AXS_REQUIRE(prec == AXS_FP64 || prec == AXS_FP32, AXS_EINVAL, "precision must be AXS_FP64 or AXS_FP32");
    const char *pa = (const char *)a, *pb = (const char *)b;
    const size_t bytes = (size_t)nrhs * c.N * 16;
    AXS_REQUIRE(pa + bytes <= pb || pb + bytes <= pa, AXS_EINVAL, "input and output vectors overlap");
    return AXS_OK;
}

// the preconditioned operator and the solves need every row of the sum
static void require_all_targets(const Ctx &c) {
    AXS_REQUIRE(c.tgt_count < 0, AXS_ESTATE,
                "a target-body range is set (axs_set_target_bodies): only axs_apply_interbody runs");
}

axs_status axs_apply_matvec(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        check_apply(c, sigma, y, nrhs, precision);
        require_all_targets(c);
        axs::require_finite(c, sigma, (int64_t)nrhs * c.N, "sigma");
        axs::apply_operator(c, sigma, y, nrhs, precision);
        return AXS_OK;
    });
}

axs_status axs_apply_matvec_noalloc(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        check_apply(c, sigma, y, nrhs, precision);
        require_all_targets(c);
        const int64_t ib = axs::interbody_scratch_bytes(c, precision, nrhs);
        AXS_REQUIRE(ib >= 0, AXS_EINVAL,
                    "the no-allocation operator runs the point and ring orders of the inter-body sum only "
                    "(the defaults below 16 right-hand sides)");
        const int64_t e = precision == AXS_FP32 ? 4 : 8, x = ((int64_t)nrhs * c.N * e + 255) / 256 * 256;
        const int64_t need = ib + 4 * x;   // + the DFT workspaces (planar re and im, forward and back)
        AXS_REQUIRE(need <= (int64_t)axs::NOALLOC_BYTES, AXS_EINVAL,
                    "the operator needs " + std::to_string(need) + " bytes of scratch, beyond the static " +
                        std::to_string(axs::NOALLOC_BYTES) + ": fewer right-hand sides per call");
        void *base = axs::static_scratch(c.device);
        AXS_REQUIRE(base, AXS_ESTATE, "static scratch not set up on this device");
        axs::ArenaScope arena(c, base, axs::NOALLOC_BYTES);
        axs::apply_operator(c, sigma, y, nrhs, precision);
        return AXS_OK;
    });
}

axs_status axs_apply_interbody(axs_ctx *ctx, const void *sigma, void *y, int nrhs, int precision) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        check_apply(c, sigma, y, nrhs, precision);
        axs::require_finite(c, sigma, (int64_t)nrhs * c.N, "sigma");
        axs::rec(c, 0);
        axs::interbody_partials(c, sigma, nrhs, precision);
        axs::interbody_reduce_to_c128(c, y, nrhs, precision);
        axs::rec(c, 1);
        if (c.timing) {
            AXS_HIP(hipEventSynchronize(c.ev[1]));
            float ms = 0;
            AXS_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
            c.last_ms[0] = c.last_ms[4] = ms;
            c.last_ms[1] = c.last_ms[2] = c.last_ms[3] = 0;
        }
        return AXS_OK;
    });
}

axs_status axs_apply_precond(axs_ctx *ctx, const void *x, void *y, int nrhs, int precision) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        check_apply(c, x, y, nrhs, precision);
        axs::require_finite(c, x, (int64_t)nrhs * c.N, "x");
        axs::apply_precond(c, x, y, nrhs, precision, 1.0);
        return AXS_OK;
    });
}

axs_status axs_solve(axs_ctx *ctx, const void *incident, const void *sigma0, void *sigma, int nrhs, int mode,
                     double tol, int max_iters, axs_solve_info *info) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        check_apply(c, incident, sigma, nrhs, AXS_FP64);
        if (sigma0) check_apply(c, sigma0, sigma, nrhs, AXS_FP64);
        require_all_targets(c);
        const int base = mode & ~(AXS_SOLVE_CERTIFY | AXS_SOLVE_UNPRECONDITIONED | AXS_SOLVE_RESTART_INNER);
        AXS_REQUIRE(base == AXS_SOLVE_FP64 || base == AXS_SOLVE_MIXED, AXS_EINVAL, "bad solve mode");
        AXS_REQUIRE(!(mode & AXS_SOLVE_UNPRECONDITIONED) || base == AXS_SOLVE_FP64, AXS_EINVAL,
                    "the unpreconditioned solve is FP64 GMRES only");
        AXS_REQUIRE(!(mode & AXS_SOLVE_RESTART_INNER) || base == AXS_SOLVE_MIXED, AXS_EINVAL,
                    "inner restarts exist in the mixed solve only");
        AXS_REQUIRE(tol > 0 && tol < 1 && std::isfinite(tol), AXS_EINVAL, "tol must be in (0, 1)");
        AXS_REQUIRE(max_iters >= 1 && max_iters <= 2000, AXS_EINVAL, "max_iters must be in [1, 2000]");
        const bool t = c.timing;
        c.timing = false;
        axs_status st = axs::solve_impl(c, incident, sigma0, sigma, nrhs, mode, tol, max_iters, info);
        c.timing = t;
        return st;
    });
}

axs_status axs_incident_plane_waves(axs_ctx *ctx, const double *dirs, int nrhs, void *v) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(dirs && v && nrhs >= 1, AXS_EINVAL, "bad arguments");
        for (int i = 0; i < 3 * nrhs; ++i) AXS_REQUIRE(std::isfinite(dirs[i]), AXS_ENONFINITE, "non-finite direction");
        double *d = (double *)c.scratch(axs::WS_EVAL, 3 * nrhs * sizeof(double));
        AXS_HIP(hipMemcpy(d, dirs, 3 * nrhs * sizeof(double), hipMemcpyHostToDevice));
        axs::incident_plane_launch(c, d, nrhs, v);
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    });
}

axs_status axs_incident_point_sources(axs_ctx *ctx, const double *src, const double *amp, int ns, void *v) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(src && amp && v && ns >= 1, AXS_EINVAL, "bad arguments");
        std::vector<double> buf(src, src + 3 * ns);
        buf.insert(buf.end(), amp, amp + 2 * ns);
        for (double x : buf) AXS_REQUIRE(std::isfinite(x), AXS_ENONFINITE, "non-finite source data");
        double *d = (double *)c.scratch(axs::WS_EVAL, buf.size() * sizeof(double));
        AXS_HIP(hipMemcpy(d, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
        axs::incident_point_launch(c, d, d + 3 * ns, ns, v);
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    });
}

axs_status axs_eval_field(axs_ctx *ctx, const void *sigma, int nrhs, const double *tgt, int nt, void *u) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(sigma && tgt && u && nt >= 1 && nrhs >= 1 && nt <= 65535 && nrhs <= 4096, AXS_EINVAL,
                    "bad arguments");
        double *d = (double *)c.scratch(axs::WS_EVAL, 3 * nt * sizeof(double));
        AXS_HIP(hipMemcpy(d, tgt, 3 * nt * sizeof(double), hipMemcpyHostToDevice));
        axs::eval_field_launch(c, sigma, nrhs, d, nt, u);
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    });
}

axs_status axs_far_field(axs_ctx *ctx, const void *sigma, int nrhs, const double *xhat, int nd, void *out) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(sigma && xhat && out && nd >= 1 && nrhs >= 1 && nd <= 65535 && nrhs <= 4096, AXS_EINVAL,
                    "bad arguments");
        AXS_REQUIRE(c.kappa > 0, AXS_EINVAL, "no far field at kappa = 0");
        double *d = (double *)c.scratch(axs::WS_EVAL, 3 * nd * sizeof(double));
        AXS_HIP(hipMemcpy(d, xhat, 3 * nd * sizeof(double), hipMemcpyHostToDevice));
        axs::far_field_launch(c, sigma, nrhs, d, nd, out);
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    });
}

axs_status axs_set_timing(axs_ctx *ctx, int enable) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        c.timing = enable != 0;
        return AXS_OK;
    });
}

axs_status axs_last_timing(axs_ctx *ctx, double ms[5]) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(ms, AXS_EINVAL, "null output");
        for (int k = 0; k < 5; ++k) ms[k] = c.last_ms[k];
        return AXS_OK;
    });
}

axs_status axs_set_interbody_config(axs_ctx *ctx, int precision, int variant, int tpt, int block, int splits) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(precision == AXS_FP64 || precision == AXS_FP32, AXS_EINVAL, "bad precision");
        AXS_REQUIRE(variant >= 0 && variant <= 4, AXS_EINVAL,
                    "variant must be 0, 1 (points), 2 (rings), 3 (MFMA) or 4 (MFMA, FP16 multiply-accumulate)");
        AXS_REQUIRE(tpt == 0 || tpt == 1 || tpt == 2 || tpt == 4 || tpt == 8, AXS_EINVAL,
                    "targets per thread must be 0, 1, 2, 4 or 8");
        AXS_REQUIRE(block == 0 || block == 128 || block == 256, AXS_EINVAL, "block must be 0, 128 or 256");
        AXS_REQUIRE(splits >= 0 && splits <= 256, AXS_EINVAL, "splits must be in [0, 256]");
        AXS_REQUIRE(!(tpt == 8 && block == 128), AXS_EINVAL, "unsupported combination");
        const int pi = precision == AXS_FP32 ? 1 : 0;
        c.ib_variant[pi] = variant;
        c.ib_tpt[pi] = tpt;
        c.ib_block[pi] = block;
        c.ib_splits[pi] = splits;
        return AXS_OK;
    });
}

axs_status axs_set_target_bodies(axs_ctx *ctx, int first_body, int count) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        const int nb = (int)c.bodies.size();
        if (first_body == 0 && count == 0) {
            c.tgt_first = 0;
            c.tgt_count = -1;
            return AXS_OK;
        }
        AXS_REQUIRE(first_body >= 0 && count >= 1 && (int64_t)first_body + count <= nb, AXS_EINVAL,
                    "target bodies must be a non-empty range of built bodies, or (0, 0) for all");
        c.tgt_first = first_body;
        c.tgt_count = count;
        return AXS_OK;
    });
}

axs_status axs_skeletonize(axs_ctx *ctx, double eps, double proxy_factor, int64_t *out_nskel) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        skeletonize(c, eps, proxy_factor);
        if (out_nskel) *out_nskel = c.skel->Ns;
        return AXS_OK;
    });
}

axs_status axs_skeletonize_points(axs_ctx *ctx, double eps, double proxy_factor, int n_proxy, uint64_t seed,
                                  int64_t *out_nskel) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        skeletonize_points(c, eps, proxy_factor, n_proxy, seed);
        if (out_nskel) *out_nskel = c.skel->Ns;
        return AXS_OK;
    });
}

axs_status axs_skeleton_rank(axs_ctx *ctx, int body_id, int *rings, int *contour_nodes) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.skel, AXS_ESTATE, "call axs_skeletonize first");
        require_all_targets(c);
        AXS_REQUIRE(rings && contour_nodes, AXS_EINVAL, "null output");
        AXS_REQUIRE(body_id >= 0 && body_id < (int)c.bodies.size(), AXS_EINVAL, "bad body id");
        const int sh = c.bodies[body_id].shape;
        *rings = c.skel->rank[sh];
        *contour_nodes = c.skel->kind == 1 ? c.skel->pts->n[sh] : c.shapes[sh].NG;
        return AXS_OK;
    });
}

axs_status axs_skeleton_nodes(axs_ctx *ctx, int body_id, int *count, int *nodes) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.skel, AXS_ESTATE, "call axs_skeletonize first");
        AXS_REQUIRE(count, AXS_EINVAL, "null output");
        AXS_REQUIRE(body_id >= 0 && body_id < (int)c.bodies.size(), AXS_EINVAL, "bad body id");
        const int sh = c.bodies[body_id].shape;
        std::vector<int> out;
        if (c.skel->kind == 1) {
            out = c.skel->pts->nodes[sh];
        } else {
            // whole rings: the ascending skeleton rings times every azimuthal node
            const int NF = c.shapes[sh].NF;
            for (int i : c.skel->rings[sh])
                for (int l = 0; l < NF; ++l) out.push_back(i * NF + l);
        }
        if (nodes) {
            AXS_REQUIRE(*count >= (int)out.size(), AXS_EINVAL, "node array too small");
            std::copy(out.begin(), out.end(), nodes);
        }
        *count = (int)out.size();
        return AXS_OK;
    });
}

axs_status axs_skeleton_interp(axs_ctx *ctx, int body_id, void *xt) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.skel, AXS_ESTATE, "call axs_skeletonize first");
        AXS_REQUIRE(c.skel->kind == 1, AXS_ESTATE, "interpolation matrices are returned for point skeletons only");
        AXS_REQUIRE(xt, AXS_EINVAL, "null output");
        AXS_REQUIRE(body_id >= 0 && body_id < (int)c.bodies.size(), AXS_EINVAL, "bad body id");
        const axs::PointSkel &P = *c.skel->pts;
        const int sh = c.bodies[body_id].shape;
        AXS_HIP(hipMemcpyAsync(xt, P.XT[sh], (size_t)P.k[sh] * P.n[sh] * sizeof(double2), hipMemcpyDeviceToDevice,
                               c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    });
}

axs_status axs_solve_skeleton(axs_ctx *ctx, const void *incident, void *sigma, int nrhs, int mode, double tol,
                              int max_iters, axs_solve_info *info) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(c.skel, AXS_ESTATE, "call axs_skeletonize first");
        require_all_targets(c);
        AXS_REQUIRE(incident && sigma && nrhs >= 1 && nrhs <= 4096 && max_iters >= 1 && max_iters <= 2000,
                    AXS_EINVAL, "bad arguments");
        AXS_REQUIRE(incident != sigma, AXS_EINVAL, "sigma must not alias the incident field");
        const bool certify = (mode & AXS_SOLVE_CERTIFY) != 0;
        const int restart = mode & AXS_SOLVE_RESTART_INNER;
        const int base = mode & ~(AXS_SOLVE_CERTIFY | AXS_SOLVE_RESTART_INNER);
        AXS_REQUIRE(base == AXS_SOLVE_FP64 || base == AXS_SOLVE_MIXED, AXS_EINVAL, "bad solve mode");
        AXS_REQUIRE(!restart || base == AXS_SOLVE_MIXED, AXS_EINVAL, "inner restarts exist in the mixed solve only");
        AXS_REQUIRE(tol > 0 && tol < 1, AXS_EINVAL, "tol must be in (0, 1)");
        Ctx &ch = *c.skel->child;
        const int64_t N = c.N, Ns = c.skel->Ns;
        double2 *y = (double2 *)c.dalloc((size_t)N * nrhs * sizeof(double2));
        double2 *u = (double2 *)c.dalloc((size_t)N * nrhs * sizeof(double2));
        double2 *bs = (double2 *)c.dalloc((size_t)Ns * nrhs * sizeof(double2));
        double2 *xs = (double2 *)c.dalloc((size_t)Ns * nrhs * sizeof(double2));
        double2 *ws = (double2 *)c.dalloc((size_t)Ns * nrhs * sizeof(double2));
        const auto t0 = std::chrono::steady_clock::now();
        apply_precond(c, incident, y, nrhs, AXS_FP64, 1.0);           // D^{-1} v
        skel_restrict(c, y, bs, nrhs, -1.0);                           // -v~ = -V^* D^{-1} v
        axs_status st = solve_impl(ch, nullptr, nullptr, xs, nrhs, base | restart, tol, max_iters, info, bs);
        interbody_partials(ch, xs, nrhs, AXS_FP64);                    // B~ s~
        interbody_reduce_to_c128(ch, ws, nrhs, AXS_FP64);
        skel_prolong(c, ws, incident, u, nrhs);                         // v + U B~ s~
        apply_precond(c, u, sigma, nrhs, AXS_FP64, -1.0);              // s = -D^{-1} (...)
        AXS_HIP(hipStreamSynchronize(c.stream));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info)
            for (int cc = 0; cc < nrhs; ++cc) info[cc].seconds = secs;
        if (certify) {
            // residual of the lifted sigma in the full system: b - (I + D^{-1} B) sigma, b = -D^{-1} v
            apply_operator(c, sigma, u, nrhs, AXS_FP64);
            bool ok = true;
            for (int cc = 0; cc < nrhs; ++cc) {
                const double2 *uc = u + (int64_t)cc * N, *yc = y + (int64_t)cc * N;
                const double num = skel_residual_sumsq(c, uc, yc, N), den = skel_sumsq(c, yc, N);
                const double rel = std::sqrt(num / (den > 0 ? den : 1.0));
                if (info) {
                    info[cc].rel_residual = rel;
                    info[cc].converged = rel <= tol ? 1 : 0;
                }
                ok = ok && rel <= tol;
            }
            if (st == AXS_OK && !ok) st = AXS_NOT_CONVERGED;
        }
        for (void *q : {(void *)y, (void *)u, (void *)bs, (void *)xs, (void *)ws}) c.dfree(q);
        return st;
    });
}

axs_status axs_interbody_launch_shape(axs_ctx *ctx, int precision, int nrhs, int *out) {
    return guarded(ctx, [&](Ctx &c) -> axs_status {
        AXS_REQUIRE(out, AXS_EINVAL, "null output");
        AXS_REQUIRE(precision == AXS_FP64 || precision == AXS_FP32, AXS_EINVAL, "bad precision");
        AXS_REQUIRE(nrhs >= 1, AXS_EINVAL, "nrhs must be positive");
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        interbody_shape(c, precision, nrhs, out);
        return AXS_OK;
    });
}

}  // extern "C"
