// Learned warm start: a multilayer perceptron (GELU hidden layers, linear
// output) trained on solves of the method itself, with hand-written FP32
// kernels for inference and training, and the maps between densities and the
// low Fourier modes the network predicts.
//
// Network: y = L_D(... GELU(L_1(x))), L_k(h) = h W_k + b_k, W_k row-major with
// the input index first; parameters packed as [W_1, b_1, W_2, b_2, ...].
// Loss: mean squared error over the batch and outputs; optimiser: Adam.
// GEMMs run on the matrix cores (16x16x4 FP32 MFMA) with 64x64 block tiles
// staged through LDS; the bias and GELU are fused into the GEMM epilogue.
//
// Warm-start encoding (the network's output): for body b, contour node i and
// |m| <= m_max, c_{b,i,m} = e^{-i kappa d.c_b} (1/N_F) sum_l sigma e^{-i m th_l},
// i.e. the low azimuthal modes of the density with the incident plane wave's
// phase at the body centre taken out; decoding puts the phase back and sums
// the modes.  Modes above m_max are zero in the decoded guess.
#include <cmath>

#include "axs_internal.h"

namespace axs {

struct Mlp {
    Ctx *ctx = nullptr;
    std::vector<int> sizes;          // n_in, width x depth, n_out
    int64_t nparams = 0;
    std::vector<int64_t> woff, boff; // per layer offsets into the packed vector
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;   // params, Adam moments, gradient
    int64_t step = 0;
    // activations for a batch (grown on demand)
    int cap_batch = 0;
    std::vector<float *> H, Z;       // H[k]: input to layer k (B x sizes[k]); Z[k]: pre-activation (B x sizes[k+1])
    float *G0 = nullptr, *G1 = nullptr, *loss_part = nullptr;
    float *Tb = nullptr;             // gathered targets of one batch (B x n_out)
    double *loss_dev = nullptr;
    int32_t *order = nullptr;        // row order of one epoch (device copy)
    int64_t cap_order = 0;
};

// ---------------------------------------------------------------------------
// GEMM: C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) with optional GELU.
// TA: A stored as K x M (transposed); TB: B stored as N x K.  All row-major.
// out_z (if set) receives the pre-activation, out_h the activation.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int GBM = 64, GBN = 64, GKT = 16;

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        const float *__restrict__ B, int ldb,
                                                        const float *__restrict__ bias, int act, float beta,
                                                        float *__restrict__ out_z, float *__restrict__ out_h, int ldc) {
    __shared__ float As[GBM][GKT + 1];
    __shared__ float Bs[GKT][GBN + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GKT) {
        // stage A tile (GBM x GKT) and B tile (GKT x GBN), 4 elements per thread each
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * 256;
            int mm, kk;
            if (TA) {            // stored K x M: consecutive threads walk m
                mm = idx % GBM;
                kk = idx / GBM;
            } else {             // stored M x K: consecutive threads walk k
                kk = idx % GKT;
                mm = idx / GKT;
            }
            const int gm = m0 + mm, gk = k0 + kk;
            float val = 0.f;
            if (gm < M && gk < K) val = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[mm][kk] = val;
            int nn, kb;
            if (TB) {            // stored N x K: consecutive threads walk k
                kb = idx % GKT;
                nn = idx / GKT;
            } else {             // stored K x N: consecutive threads walk n
                nn = idx % GBN;
                kb = idx / GBN;
            }
            const int gn = n0 + nn, gkb = k0 + kb;
            float vb = 0.f;
            if (gn < N && gkb < K) vb = TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn];
            Bs[kb][nn] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GKT; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    float z = acc[i][j][r];
                    if (bias) z += bias[gn];
                    const int64_t o = (int64_t)gm * ldc + gn;
                    if (beta != 0.f) z += beta * out_z[o];
                    if (out_z) out_z[o] = z;
                    if (out_h) out_h[o] = act ? gelu_f(z) : z;
                }
            }
}

template <bool TA, bool TB>
static void gemm(Ctx &c, int M, int N, int K, const float *A, int lda, const float *B, int ldb, const float *bias,
                 int act, float *out_z, float *out_h, int ldc) {
    dim3 grid((unsigned)ceil_div(N, GBN), (unsigned)ceil_div(M, GBM));
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB>), grid, dim3(256), 0, c.stream, M, N, K, A, lda, B, ldb, bias, act,
                       0.f, out_z, out_h, ldc);
    AXS_HIP(hipGetLastError());
}

// G <- G * GELU'(Z)
__global__ void gelu_backward_kernel(float *__restrict__ G, const float *__restrict__ Z, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) G[t] *= gelu_grad_f(Z[t]);
}

// db[j] = sum_b G[b][j]   (fixed order over the batch)
__global__ void colsum_kernel(const float *__restrict__ G, int B, int n, float *__restrict__ db) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += G[(int64_t)b * n + j];
    db[j] = s;
}

// G = 2 (Y - T) / (B n); per-block partial sums of (Y - T)^2 in double
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ Y, const float *__restrict__ T, int64_t n,
                                                  float scale, float *__restrict__ G, float *__restrict__ part) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const float d = Y[t] - T[t];
        G[t] = 2.f * d * scale;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts_kernel(const float *__restrict__ part, int n, double scale, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// dst[r][:] = src[idx[r]][:] for r < batch; idx already checked against the source rows
__global__ __launch_bounds__(256) void gather_rows_kernel(const float *__restrict__ src, int ncol,
                                                          const int32_t *__restrict__ idx, int batch,
                                                          float *__restrict__ dst) {
    const int64_t n = (int64_t)batch * ncol;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int64_t r = t / ncol, col = t - r * ncol;
        dst[t] = src[(int64_t)idx[r] * ncol + col];
    }
}

__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gg = g[t];
    const float mm = b1 * m[t] + (1.f - b1) * gg;
    const float vv = b2 * v[t] + (1.f - b2) * gg * gg;
    m[t] = mm;
    v[t] = vv;
    p[t] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

// ---------------------------------------------------------------------------
// density <-> low modes (with the plane-wave phase at each body centre removed)
// ---------------------------------------------------------------------------
// coeff layout per rhs: bodies in order, contour node i, m = -mmax..mmax, (re, im)
__global__ void modes_from_density_kernel(const BodyDev *__restrict__ bodies, const int64_t *__restrict__ coff,
                                          const double *__restrict__ frame, const double2 *__restrict__ sigma,
                                          const double *__restrict__ dirs, int64_t N, int64_t P, int mmax,
                                          double kappa, int nb, float *__restrict__ coeff) {
    const int b = blockIdx.y, c = blockIdx.z;
    const BodyDev bd = bodies[b];
    const int nm = 2 * mmax + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bd.NG * nm) return;
    const int i = t / nm, mi = t % nm, m = mi - mmax;
    const double *d = dirs + 3 * c;
    const double ph = kappa * (d[0] * frame[FRAME * b] + d[1] * frame[FRAME * b + 1] + d[2] * frame[FRAME * b + 2]);
    double sr = 0, si = 0;
    const double2 *row = sigma + (int64_t)c * N + bd.offset + (int64_t)i * bd.NF;
    for (int l = 0; l < bd.NF; ++l) {
        double sn, cs;
        sincospi(-2.0 * (double)(((int64_t)m * l) % bd.NF) / bd.NF, &sn, &cs);
        sr += row[l].x * cs - row[l].y * sn;
        si += row[l].x * sn + row[l].y * cs;
    }
    double pn, pc;
    sincos(-ph, &pn, &pc);
    const double re = (sr * pc - si * pn) / bd.NF, im = (sr * pn + si * pc) / bd.NF;
    float *o = coeff + (int64_t)c * P + coff[b] + 2 * (int64_t)t;
    o[0] = (float)re;
    o[1] = (float)im;
}

__global__ void density_from_modes_kernel(const BodyDev *__restrict__ bodies, const int64_t *__restrict__ coff,
                                          const double *__restrict__ frame, const float *__restrict__ coeff,
                                          const double *__restrict__ dirs, int64_t N, int64_t P, int mmax,
                                          double kappa, double2 *__restrict__ sigma) {
    const int b = blockIdx.y, c = blockIdx.z;
    const BodyDev bd = bodies[b];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bd.NG * bd.NF) return;
    const int i = t / bd.NF, l = t % bd.NF;
    const int nm = 2 * mmax + 1;
    const double *d = dirs + 3 * c;
    const double ph = kappa * (d[0] * frame[FRAME * b] + d[1] * frame[FRAME * b + 1] + d[2] * frame[FRAME * b + 2]);
    const float *cf = coeff + (int64_t)c * P + coff[b] + 2 * (int64_t)i * nm;
    double sr = 0, si = 0;
    for (int mi = 0; mi < nm; ++mi) {
        const int m = mi - mmax;
        int64_t ml = ((int64_t)m * l) % bd.NF;
        double sn, cs;
        sincospi(2.0 * (double)ml / bd.NF, &sn, &cs);
        const double ar = cf[2 * mi], ai = cf[2 * mi + 1];
        sr += ar * cs - ai * sn;
        si += ar * sn + ai * cs;
    }
    double pn, pc;
    sincos(ph, &pn, &pc);
    sigma[(int64_t)c * N + bd.offset + t] = make_double2(sr * pc - si * pn, sr * pn + si * pc);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
static void ensure_batch(Mlp &n, int B) {
    if (B <= n.cap_batch) return;
    Ctx &c = *n.ctx;
    for (auto *p : n.H) c.dfree(p);
    for (auto *p : n.Z) c.dfree(p);
    c.dfree(n.G0);
    c.dfree(n.G1);
    c.dfree(n.Tb);
    const int L = (int)n.sizes.size() - 1;
    n.H.assign(L + 1, nullptr);
    n.Z.assign(L, nullptr);
    int wmax = 0;
    for (int s : n.sizes) wmax = std::max(wmax, s);
    for (int k = 0; k <= L; ++k) n.H[k] = (float *)c.dalloc((size_t)B * n.sizes[k] * sizeof(float));
    for (int k = 0; k < L; ++k) n.Z[k] = (float *)c.dalloc((size_t)B * n.sizes[k + 1] * sizeof(float));
    n.G0 = (float *)c.dalloc((size_t)B * wmax * sizeof(float));
    n.G1 = (float *)c.dalloc((size_t)B * wmax * sizeof(float));
    n.Tb = (float *)c.dalloc((size_t)B * n.sizes[L] * sizeof(float));
    n.cap_batch = B;
}

// forward pass from the input already in H[0]; H[L] = output
static void mlp_forward_h0(Mlp &n, int B) {
    Ctx &c = *n.ctx;
    const int L = (int)n.sizes.size() - 1;
    for (int k = 0; k < L; ++k) {
        const int a = n.sizes[k], b = n.sizes[k + 1];
        gemm<false, false>(c, B, b, a, n.H[k], a, n.p + n.woff[k], b, n.p + n.boff[k], k < L - 1 ? 1 : 0, n.Z[k],
                           n.H[k + 1], b);
    }
}

// forward pass: H[0] = X (copied), H[L] = output
static void mlp_forward(Mlp &n, const float *X, int B) {
    Ctx &c = *n.ctx;
    ensure_batch(n, B);
    AXS_HIP(hipMemcpyAsync(n.H[0], X, (size_t)B * n.sizes[0] * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
    mlp_forward_h0(n, B);
}

// bias-corrected Adam update of the packed parameters from the gradient in n.g
static void adam_update(Mlp &n, double lr, double b1, double b2, double eps) {
    Ctx &c = *n.ctx;
    n.step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)n.step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)n.step)));
    hipLaunchKernelGGL(adam_kernel, dim3(ceil_div(n.nparams, 256)), dim3(256), 0, c.stream, n.p, n.m, n.v, n.g,
                       n.nparams, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    AXS_HIP(hipGetLastError());
}

static void gather_rows(Ctx &c, const float *src, int ncol, const int32_t *idx, int batch, float *dst) {
    const int nblk = (int)std::min<int64_t>(4096, ceil_div((int64_t)batch * ncol, 256));
    hipLaunchKernelGGL(gather_rows_kernel, dim3(nblk), dim3(256), 0, c.stream, src, ncol, idx, batch, dst);
    AXS_HIP(hipGetLastError());
}

// loss and gradient of the packed parameters into n.g
static void mlp_backward(Mlp &n, const float *T, int B) {
    Ctx &c = *n.ctx;
    const int L = (int)n.sizes.size() - 1;
    const int nout = n.sizes[L];
    const int64_t ny = (int64_t)B * nout;
    const int nblk = (int)std::min<int64_t>(1024, ceil_div(ny, 256));
    if (!n.loss_part) {
        n.loss_part = (float *)c.dalloc(1024 * sizeof(float));
        n.loss_dev = (double *)c.dalloc(sizeof(double));
    }
    hipLaunchKernelGGL(mse_kernel, dim3(nblk), dim3(256), 0, c.stream, n.H[L], T, ny, 1.f / (float)ny, n.G0,
                       n.loss_part);
    AXS_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, c.stream, n.loss_part, nblk, 1.0 / (double)ny,
                       n.loss_dev);
    AXS_HIP(hipGetLastError());
    float *G = n.G0, *Gn = n.G1;
    for (int k = L - 1; k >= 0; --k) {
        const int a = n.sizes[k], b = n.sizes[k + 1];
        if (k < L - 1) {
            hipLaunchKernelGGL(gelu_backward_kernel, dim3(ceil_div((int64_t)B * b, 256)), dim3(256), 0, c.stream, G,
                               n.Z[k], (int64_t)B * b);
            AXS_HIP(hipGetLastError());
        }
        // dW = H^T G  (a x b),  db = colsum(G),  dH = G W^T (B x a)
        gemm<true, false>(c, a, b, B, n.H[k], a, G, b, nullptr, 0, nullptr, n.g + n.woff[k], b);
        hipLaunchKernelGGL(colsum_kernel, dim3(ceil_div(b, 256)), dim3(256), 0, c.stream, G, B, b, n.g + n.boff[k]);
        AXS_HIP(hipGetLastError());
        if (k > 0) {
            gemm<false, true>(c, B, a, b, G, b, n.p + n.woff[k], b, nullptr, 0, nullptr, Gn, a);
            std::swap(G, Gn);
        }
    }
}

}  // namespace axs

using axs::Ctx;
using axs::Error;
using axs::Mlp;

struct axs_ctx {
    Ctx c;
};
struct axs_mlp {
    Mlp n;
};

template <class F>
static axs_status mlp_guarded(axs_mlp *h, F &&f) {
    if (!h || !h->n.ctx) return AXS_EINVAL;
    Ctx &c = *h->n.ctx;
    c.err.clear();
    try {
        return f(h->n, c);
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        c.err = e.what();
        return AXS_EINVAL;
    }
}

extern "C" {

axs_status axs_mlp_create(axs_ctx *ctx, int n_in, int width, int depth, int n_out, axs_mlp **out) {
    if (!ctx || !out || n_in < 1 || width < 1 || depth < 1 || n_out < 1) return AXS_EINVAL;
    *out = nullptr;
    try {
        axs_mlp *h = new axs_mlp();
        Mlp &n = h->n;
        n.ctx = &ctx->c;
        n.sizes.push_back(n_in);
        for (int k = 0; k < depth; ++k) n.sizes.push_back(width);
        n.sizes.push_back(n_out);
        int64_t o = 0;
        for (size_t k = 0; k + 1 < n.sizes.size(); ++k) {
            n.woff.push_back(o);
            o += (int64_t)n.sizes[k] * n.sizes[k + 1];
            n.boff.push_back(o);
            o += n.sizes[k + 1];
        }
        n.nparams = o;
        n.p = (float *)n.ctx->dalloc(o * sizeof(float));
        n.m = (float *)n.ctx->dalloc(o * sizeof(float));
        n.v = (float *)n.ctx->dalloc(o * sizeof(float));
        n.g = (float *)n.ctx->dalloc(o * sizeof(float));
        AXS_HIP(hipMemsetAsync(n.p, 0, o * sizeof(float), n.ctx->stream));
        AXS_HIP(hipMemsetAsync(n.m, 0, o * sizeof(float), n.ctx->stream));
        AXS_HIP(hipMemsetAsync(n.v, 0, o * sizeof(float), n.ctx->stream));
        *out = h;
        return AXS_OK;
    } catch (const Error &e) {
        ctx->c.err = e.msg;
        return e.code;
    }
}

axs_status axs_mlp_destroy(axs_mlp *h) {
    if (!h) return AXS_EINVAL;
    Mlp &n = h->n;
    if (n.ctx) {
        (void)hipStreamSynchronize(n.ctx->stream);
        for (auto *p : n.H) n.ctx->dfree(p);
        for (auto *p : n.Z) n.ctx->dfree(p);
        for (void *p : {(void *)n.p, (void *)n.m, (void *)n.v, (void *)n.g, (void *)n.G0, (void *)n.G1,
                        (void *)n.Tb, (void *)n.loss_part, (void *)n.loss_dev, (void *)n.order})
            n.ctx->dfree(p);
    }
    delete h;
    return AXS_OK;
}

axs_status axs_mlp_num_params(const axs_mlp *h, int64_t *count) {
    if (!h || !count) return AXS_EINVAL;
    *count = h->n.nparams;
    return AXS_OK;
}

axs_status axs_mlp_set_params(axs_mlp *h, const float *host) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(host, AXS_EINVAL, "null parameters");
        for (int64_t i = 0; i < n.nparams; ++i) AXS_REQUIRE(std::isfinite(host[i]), AXS_ENONFINITE, "non-finite parameter");
        AXS_HIP(hipMemcpy(n.p, host, n.nparams * sizeof(float), hipMemcpyHostToDevice));
        AXS_HIP(hipMemset(n.m, 0, n.nparams * sizeof(float)));
        AXS_HIP(hipMemset(n.v, 0, n.nparams * sizeof(float)));
        n.step = 0;
        return AXS_OK;
    });
}

axs_status axs_mlp_get_params(axs_mlp *h, float *host) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(host, AXS_EINVAL, "null output");
        AXS_HIP(hipStreamSynchronize(c.stream));
        AXS_HIP(hipMemcpy(host, n.p, n.nparams * sizeof(float), hipMemcpyDeviceToHost));
        return AXS_OK;
    });
}

axs_status axs_mlp_forward(axs_mlp *h, const float *X, float *Y, int batch) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(X && Y && batch >= 1, AXS_EINVAL, "bad arguments");
        axs::mlp_forward(n, X, batch);
        const int L = (int)n.sizes.size() - 1;
        AXS_HIP(hipMemcpyAsync(Y, n.H[L], (size_t)batch * n.sizes[L] * sizeof(float), hipMemcpyDeviceToDevice,
                               c.stream));
        return AXS_OK;
    });
}

axs_status axs_mlp_gradient(axs_mlp *h, const float *X, const float *T, int batch, double *loss, float *grad) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(X && T && batch >= 1, AXS_EINVAL, "bad arguments");
        axs::mlp_forward(n, X, batch);
        axs::mlp_backward(n, T, batch);
        if (grad)
            AXS_HIP(hipMemcpyAsync(grad, n.g, n.nparams * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
        if (loss) {
            AXS_HIP(hipMemcpyAsync(loss, n.loss_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
        }
        return AXS_OK;
    });
}

axs_status axs_mlp_adam_step(axs_mlp *h, const float *X, const float *T, int batch, double lr, double b1, double b2,
                             double eps, double *loss) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(X && T && batch >= 1 && lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0,
                    AXS_EINVAL, "bad arguments");
        axs::mlp_forward(n, X, batch);
        axs::mlp_backward(n, T, batch);
        axs::adam_update(n, lr, b1, b2, eps);
        if (loss) {
            AXS_HIP(hipMemcpyAsync(loss, n.loss_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
        }
        return AXS_OK;
    });
}

axs_status axs_mlp_train_epoch(axs_mlp *h, const float *X, const float *T, int64_t rows, const int32_t *order,
                               int batch, int steps, const double *lr, double b1, double b2, double eps,
                               double *loss) {
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(X && T && order && lr && rows >= 1 && batch >= 1 && steps >= 1 && b1 >= 0 && b1 < 1 &&
                        b2 >= 0 && b2 < 1 && eps > 0,
                    AXS_EINVAL, "bad arguments");
        AXS_REQUIRE(rows <= INT32_MAX, AXS_EINVAL, "more than 2^31 - 1 sample rows");
        const int64_t total = (int64_t)batch * steps;
        AXS_REQUIRE(total <= INT32_MAX, AXS_EINVAL, "batch x steps exceeds 2^31 - 1");
        for (int s = 0; s < steps; ++s) AXS_REQUIRE(lr[s] > 0, AXS_EINVAL, "learning rates must be positive");
        for (int64_t i = 0; i < total; ++i)
            AXS_REQUIRE(order[i] >= 0 && order[i] < rows, AXS_EINVAL, "row index out of range");
        if (total > n.cap_order) {
            AXS_HIP(hipStreamSynchronize(c.stream));
            c.dfree(n.order);
            n.order = nullptr;
            n.order = (int32_t *)c.dalloc((size_t)total * sizeof(int32_t));
            n.cap_order = total;
        }
        // after the previous epoch's steps (readers of n.order), and complete before the
        // first step is queued, so the caller may reuse the host array on return
        AXS_HIP(hipStreamSynchronize(c.stream));
        AXS_HIP(hipMemcpyAsync(n.order, order, (size_t)total * sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        axs::ensure_batch(n, batch);
        const int L = (int)n.sizes.size() - 1;
        for (int s = 0; s < steps; ++s) {
            const int32_t *idx = n.order + (int64_t)s * batch;
            axs::gather_rows(c, X, n.sizes[0], idx, batch, n.H[0]);
            axs::gather_rows(c, T, n.sizes[L], idx, batch, n.Tb);
            axs::mlp_forward_h0(n, batch);
            axs::mlp_backward(n, n.Tb, batch);
            axs::adam_update(n, lr[s], b1, b2, eps);
        }
        if (loss) {
            AXS_HIP(hipMemcpyAsync(loss, n.loss_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
        }
        return AXS_OK;
    });
}

}  // extern "C"

namespace axs {
// shared by the two mode maps: per-body coefficient offsets (per rhs) and checks
static int64_t mode_layout(Ctx &c, int mmax, std::vector<int64_t> &coff) {
    coff.clear();
    int64_t P = 0;
    for (auto &b : c.bodies) {
        coff.push_back(P);
        P += 2LL * c.shapes[b.shape].NG * (2 * mmax + 1);
    }
    return P;
}
}  // namespace axs

extern "C" {

axs_status axs_warm_start_size(axs_ctx *ctx, int mmax, int64_t *P) {
    if (!ctx || !P || mmax < 0) return AXS_EINVAL;
    std::vector<int64_t> coff;
    *P = axs::mode_layout(ctx->c, mmax, coff);
    return AXS_OK;
}

static axs_status mode_map(axs_ctx *ctx, bool to_modes, const void *sigma, const float *coeff_in, float *coeff_out,
                           const double *dirs, int nrhs, int mmax, void *sigma_out) {
    if (!ctx) return AXS_EINVAL;
    Ctx &c = ctx->c;
    c.err.clear();
    try {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(dirs && nrhs >= 1 && nrhs <= 4096 && mmax >= 0, AXS_EINVAL, "bad arguments");
        for (auto &s : c.shapes) AXS_REQUIRE(mmax <= s.M, AXS_EINVAL, "m_max exceeds a body's mode cutoff");
        std::vector<int64_t> coff;
        const int64_t P = axs::mode_layout(c, mmax, coff);
        const size_t extra = coff.size() * sizeof(int64_t) + 3 * nrhs * sizeof(double);
        char *d = (char *)c.scratch(axs::WS_EVAL, extra);
        AXS_HIP(hipMemcpy(d, coff.data(), coff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        AXS_HIP(hipMemcpy(d + coff.size() * sizeof(int64_t), dirs, 3 * nrhs * sizeof(double), hipMemcpyHostToDevice));
        const int64_t *dcoff = (const int64_t *)d;
        const double *ddirs = (const double *)(d + coff.size() * sizeof(int64_t));
        int maxng = 0, maxn = 0;
        for (auto &s : c.shapes) {
            maxng = std::max(maxng, s.NG);
            maxn = std::max(maxn, s.NG * s.NF);
        }
        const int nb = (int)c.bodies.size();
        if (to_modes) {
            AXS_REQUIRE(sigma && coeff_out, AXS_EINVAL, "null vector");
            dim3 grid((unsigned)axs::ceil_div((int64_t)maxng * (2 * mmax + 1), 128), nb, nrhs);
            hipLaunchKernelGGL(axs::modes_from_density_kernel, grid, dim3(128), 0, c.stream, c.body_dev, dcoff,
                               c.frame64, (const double2 *)sigma, ddirs, c.N, P, mmax, c.kappa, nb, coeff_out);
        } else {
            AXS_REQUIRE(coeff_in && sigma_out, AXS_EINVAL, "null vector");
            dim3 grid((unsigned)axs::ceil_div(maxn, 128), nb, nrhs);
            hipLaunchKernelGGL(axs::density_from_modes_kernel, grid, dim3(128), 0, c.stream, c.body_dev, dcoff,
                               c.frame64, coeff_in, ddirs, c.N, P, mmax, c.kappa, (double2 *)sigma_out);
        }
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    }
}

axs_status axs_modes_from_density(axs_ctx *ctx, const void *sigma, const double *dirs, int nrhs, int mmax,
                                  float *coeff) {
    return mode_map(ctx, true, sigma, nullptr, coeff, dirs, nrhs, mmax, nullptr);
}

axs_status axs_density_from_modes(axs_ctx *ctx, const float *coeff, const double *dirs, int nrhs, int mmax,
                                  void *sigma) {
    return mode_map(ctx, false, nullptr, coeff, nullptr, dirs, nrhs, mmax, sigma);
}

}  // extern "C"
