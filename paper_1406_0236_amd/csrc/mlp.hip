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
// Warm-start encoding (the network's output).  From eq. "precond" the solution
// satisfies sigma* = b~ - D^{-1} B sigma*, b~ = -D^{-1} v, and b~ (the
// single-body responses) costs one preconditioner application.  The network
// predicts only the rest, split by source body:
//   sigma*_b - b~_b = sum_{b' != b} u^{b'}_b,   u^{b'}_b = -D_b^{-1} B_{bb'} sigma*_{b'},
// the response of body b to the field radiated by body b'.  The leading phase
// of that term, the incident wave's phase at c_{b'} carried over the distance
// between the centres, phi_{bb'} = kappa (d.c_{b'} + |c_b - c_{b'}|), is taken
// out, and the low azimuthal modes of the rest are the outputs:
//   Y[b][s][i][m] = e^{-i phi_{bb'}} (1/N_F) sum_l u^{b'}_b(i, l) e^{-i m th_l},
// s the index of b' among the bodies other than b (build order), |m| <= m_max.
// Decoding puts the phases back, sums over the sources and the modes, and the
// guess is b~ plus that sum.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

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
    float *ws = nullptr;             // split-K partial products (grown on demand)
    int64_t cap_ws = 0;
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

// With gridDim.z > 1 (split K) block z sums k in [z kc, min(K, (z+1) kc)) and
// writes its partial product, without bias or activation, to out_h + z M ldc.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K, int kc, const float *__restrict__ A,
                                                        int lda, const float *__restrict__ B, int ldb,
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
    const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
    if (gridDim.z > 1) out_h += (int64_t)blockIdx.z * M * ldc;
    for (int k0 = kb; k0 < ke; k0 += GKT) {
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
            if (gm < M && gk < ke) val = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
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
            if (gn < N && gkb < ke) vb = TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn];
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

// out[m][n] = sum_s part[s][m][n] (fixed order) + bias[n], GELU with act
__global__ void splitk_reduce_kernel(const float *__restrict__ part, int S, int M, int N,
                                     const float *__restrict__ bias, int act, float *__restrict__ out_z,
                                     float *__restrict__ out_h) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, mn = (int64_t)M * N;
    if (t >= mn) return;
    float z = 0.f;
    for (int s = 0; s < S; ++s) z += part[s * mn + t];
    if (bias) z += bias[t % N];
    if (out_z) out_z[t] = z;
    if (out_h) out_h[t] = act ? gelu_f(z) : z;
}

// K splits for a GEMM whose output has too few 64 x 64 tiles to fill the
// GPU (at least 1024 k per split, up to about 1024 blocks in all); 1 = none
static int splitk_count(int M, int N, int K) {
    const int64_t tiles = ceil_div(M, GBM) * ceil_div(N, GBN);
    if (tiles >= 256 || K < 2048) return 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(K / 1024, 1024 / tiles));
}

// C = op(A) op(B) (+ bias, GELU); ws: workspace of splitk_count(M, N, K) M N
// floats when that count exceeds 1 (ldc must then be N)
template <bool TA, bool TB>
static void gemm(Ctx &c, int M, int N, int K, const float *A, int lda, const float *B, int ldb, const float *bias,
                 int act, float *out_z, float *out_h, int ldc, float *ws = nullptr) {
    const int S = ws && ldc == N ? splitk_count(M, N, K) : 1;
    const int kc = S > 1 ? (int)(ceil_div(ceil_div(K, S), GKT) * GKT) : K;
    const int Sg = S > 1 ? (int)ceil_div(K, kc) : 1;
    dim3 grid((unsigned)ceil_div(N, GBN), (unsigned)ceil_div(M, GBM), (unsigned)Sg);
    if (Sg > 1) {
        hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB>), grid, dim3(256), 0, c.stream, M, N, K, kc, A, lda, B, ldb,
                           nullptr, 0, 0.f, nullptr, ws, N);
        AXS_HIP(hipGetLastError());
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)ceil_div((int64_t)M * N, 256)), dim3(256), 0,
                           c.stream, ws, Sg, M, N, bias, act, out_z, out_h);
    } else {
        hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB>), grid, dim3(256), 0, c.stream, M, N, K, K, A, lda, B, ldb, bias,
                           act, 0.f, out_z, out_h, ldc);
    }
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
            // dH has few output tiles and, for the output layer, a long k range: split K
            const int64_t need = (int64_t)splitk_count(B, a, b) * B * a;
            if (need > (int64_t)B * a && need > n.cap_ws) {
                AXS_HIP(hipStreamSynchronize(c.stream));
                c.dfree(n.ws);
                n.ws = nullptr;
                n.ws = (float *)c.dalloc((size_t)need * sizeof(float));
                n.cap_ws = need;
            }
            gemm<false, true>(c, B, a, b, G, b, n.p + n.woff[k], b, nullptr, 0, nullptr, Gn, a, n.ws);
            std::swap(G, Gn);
        }
    }
}


// copy one epoch's row order (host, already checked) to the device; the copy is
// complete on return, so the caller may reuse the host array
static void load_order(Mlp &n, const int32_t *order, int64_t total) {
    Ctx &c = *n.ctx;
    if (total > n.cap_order) {
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(n.order);
        n.order = nullptr;
        n.order = (int32_t *)c.dalloc((size_t)total * sizeof(int32_t));
        n.cap_order = total;
    }
    // after the previous epoch's steps (readers of n.order)
    AXS_HIP(hipStreamSynchronize(c.stream));
    AXS_HIP(hipMemcpyAsync(n.order, order, (size_t)total * sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));
}

// `steps` Adam steps on the rows n.order[s batch .. (s+1) batch) of X and T,
// queued without synchronisation
static void queue_steps(Mlp &n, const float *X, const float *T, int batch, int steps, const double *lr, double b1,
                        double b2, double eps) {
    Ctx &c = *n.ctx;
    ensure_batch(n, batch);
    const int L = (int)n.sizes.size() - 1;
    for (int s = 0; s < steps; ++s) {
        const int32_t *idx = n.order + (int64_t)s * batch;
        gather_rows(c, X, n.sizes[0], idx, batch, n.H[0]);
        gather_rows(c, T, n.sizes[L], idx, batch, n.Tb);
        mlp_forward_h0(n, batch);
        mlp_backward(n, n.Tb, batch);
        adam_update(n, lr[s], b1, b2, eps);
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
                        (void *)n.Tb, (void *)n.loss_part, (void *)n.loss_dev, (void *)n.order, (void *)n.ws})
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
        axs::load_order(n, order, total);
        axs::queue_steps(n, X, T, batch, steps, lr, b1, b2, eps);
        if (loss) {
            AXS_HIP(hipMemcpyAsync(loss, n.loss_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
        }
        return AXS_OK;
    });
}

}  // extern "C"


// ===========================================================================
// Training, encoding, decoding and prediction of the warm start
// ===========================================================================
namespace axs {

// per-target-body offsets of the warm-start layout (per rhs); returns the
// floats per rhs, 2 (B - 1) (2 m_max + 1) sum_b N_G(b)
static int64_t ws_layout(const Ctx &c, int mmax, std::vector<int64_t> &toff) {
    toff.clear();
    const int64_t B = (int64_t)c.bodies.size();
    int64_t P = 0;
    for (auto &b : c.bodies) {
        toff.push_back(P);
        P += 2 * (B - 1) * c.shapes[b.shape].NG * (2 * mmax + 1);
    }
    return P;
}

// e^{i phi}, phi = kappa (d_c . c_{b'} + |c_b - c_{b'}|), for rhs c, target b,
// source slot s (b' = s for s < b, s + 1 otherwise): ph[(c nb + b) (nb - 1) + s]
__global__ void ws_phase_kernel(const double *__restrict__ frame, const double *__restrict__ dirs, int nb, int nrhs,
                                double kappa, double2 *__restrict__ ph) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nb * (nb - 1);
    if (t >= per * nrhs) return;
    const int c = (int)(t / per), r = (int)(t % per), b = r / (nb - 1), s = r % (nb - 1);
    const int bs = s < b ? s : s + 1;
    const double *d = dirs + 3 * c, *cb = frame + FRAME * b, *cs = frame + FRAME * bs;
    const double dx = cb[0] - cs[0], dy = cb[1] - cs[1], dz = cb[2] - cs[2];
    const double phi = kappa * (d[0] * cs[0] + d[1] * cs[1] + d[2] * cs[2] + sqrt(dx * dx + dy * dy + dz * dz));
    double sn, cn;
    sincos(phi, &sn, &cn);
    ph[t] = make_double2(cn, sn);
}

// out[(b' nch + c)][n] = sigma[c][n] on the nodes of body b', 0 elsewhere
__global__ void mask_by_body_kernel(const double2 *__restrict__ sigma, const int64_t *__restrict__ body_off, int nb,
                                    int nch, int64_t N, double2 *__restrict__ out) {
    const int64_t total = (int64_t)nb * nch * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = t % N, z = t / N;
        const int bp = (int)(z / nch), c = (int)(z % nch);
        const bool in = n >= body_off[bp] && n < body_off[bp + 1];
        out[t] = in ? sigma[(int64_t)c * N + n] : make_double2(0.0, 0.0);
    }
}

// targets of one rhs chunk: u[(b' nch + c)][N] = -D^{-1} B (sigma_c masked to
// body b'); Y[c][toff[b] + 2 ((s N_G + i) nm + mi)] for every target b and slot s
__global__ void ws_encode_kernel(const BodyDev *__restrict__ bodies, const int64_t *__restrict__ toff,
                                 const double2 *__restrict__ ph, const double2 *__restrict__ u, int64_t N, int64_t P,
                                 int mmax, int nb, int nch, float *__restrict__ Y) {
    const int b = blockIdx.y, z = blockIdx.z;
    const int c = z / (nb - 1), s = z % (nb - 1);
    const int bs = s < b ? s : s + 1;
    const BodyDev bd = bodies[b];
    const int nm = 2 * mmax + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bd.NG * nm) return;
    const int i = t / nm, mi = t % nm, m = mi - mmax;
    const double2 *row = u + ((int64_t)bs * nch + c) * N + bd.offset + (int64_t)i * bd.NF;
    double sr = 0, si = 0;
    for (int l = 0; l < bd.NF; ++l) {
        double sn, cs;
        sincospi(-2.0 * (double)(((int64_t)m * l) % bd.NF) / bd.NF, &sn, &cs);
        sr += row[l].x * cs - row[l].y * sn;
        si += row[l].x * sn + row[l].y * cs;
    }
    const double2 e = ph[((int64_t)c * nb + b) * (nb - 1) + s];   // multiply by conj(e) / N_F
    const double re = (sr * e.x + si * e.y) / bd.NF, im = (si * e.x - sr * e.y) / bd.NF;
    float *o = Y + (int64_t)c * P + toff[b] + 2 * (((int64_t)s * bd.NG + i) * nm + mi);
    o[0] = (float)re;
    o[1] = (float)im;
}

// sigma[c](b, i, l) (+)= sum_m e^{i m th_l} sum_s e^{i phi_{b b'_s}} Y[c][b][s][i][m]
__global__ void ws_decode_kernel(const BodyDev *__restrict__ bodies, const int64_t *__restrict__ toff,
                                 const double2 *__restrict__ ph, const float *__restrict__ Y, int64_t N, int64_t P,
                                 int mmax, int nb, int add, double2 *__restrict__ sigma) {
    const int b = blockIdx.y, c = blockIdx.z;
    const BodyDev bd = bodies[b];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bd.NG * bd.NF) return;
    const int i = t / bd.NF, l = t % bd.NF;
    const int nm = 2 * mmax + 1;
    const double2 *e = ph + ((int64_t)c * nb + b) * (nb - 1);
    const float *cf = Y + (int64_t)c * P + toff[b];
    double sr = 0, si = 0;
    for (int mi = 0; mi < nm; ++mi) {
        double ar = 0, ai = 0;
        for (int s = 0; s < nb - 1; ++s) {
            const float *y = cf + 2 * (((int64_t)s * bd.NG + i) * nm + mi);
            const double yr = y[0], yi = y[1];
            ar += e[s].x * yr - e[s].y * yi;
            ai += e[s].x * yi + e[s].y * yr;
        }
        const int64_t ml = ((int64_t)(mi - mmax) * l) % bd.NF;
        double sn, cs;
        sincospi(2.0 * (double)ml / bd.NF, &sn, &cs);
        sr += ar * cs - ai * sn;
        si += ar * sn + ai * cs;
    }
    double2 *o = sigma + (int64_t)c * N + bd.offset + t;
    if (add) {
        const double2 v = *o;
        *o = make_double2(v.x + sr, v.y + si);
    } else {
        *o = make_double2(sr, si);
    }
}

// network input: (d_x, d_y, d_z, (2 k - (k_min + k_max)) / (k_max - k_min)) from (d, k)
__global__ void ws_features_kernel(const float *__restrict__ X, int64_t S, double kmin, double kmax,
                                   float *__restrict__ Xs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    const float *x = X + 4 * t;
    float *o = Xs + 4 * t;
    o[0] = x[0];
    o[1] = x[1];
    o[2] = x[2];
    o[3] = (float)((2.0 * (double)x[3] - (kmin + kmax)) / (kmax - kmin));
}

// per-block partial sums of squares (FP64), fixed order
__global__ __launch_bounds__(256) void sumsq_f32_kernel(const float *__restrict__ a, int64_t n,
                                                        double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const double v = a[t];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0..n) = f * in[0..n)
__global__ void scale_f32_kernel(const float *__restrict__ in, int64_t n, float f, float *__restrict__ out) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = f * in[t];
}

static void scale_f32(Ctx &c, const float *in, int64_t n, float f, float *out) {
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(8192, ceil_div(n, 256)));
    hipLaunchKernelGGL(scale_f32_kernel, dim3(nblk), dim3(256), 0, c.stream, in, n, f, out);
    AXS_HIP(hipGetLastError());
}

// the number m_max with n_out = 2 (B - 1) (2 m_max + 1) sum N_G, or -1
static int ws_mmax_for(const Ctx &c, int64_t nout) {
    const int64_t B = (int64_t)c.bodies.size();
    if (B < 2) return -1;
    int64_t ng = 0;
    for (auto &b : c.bodies) ng += c.shapes[b.shape].NG;
    const int64_t unit = 2 * (B - 1) * ng;
    if (nout % unit) return -1;
    const int64_t nm = nout / unit;
    if (nm % 2 == 0) return -1;
    return (int)((nm - 1) / 2);
}

static void ws_check_mmax(const Ctx &c, int mmax) {
    AXS_REQUIRE(c.bodies.size() >= 2, AXS_EINVAL, "the warm start needs at least two bodies");
    AXS_REQUIRE(mmax >= 0, AXS_EINVAL, "m_max must be >= 0");
    for (auto &s : c.shapes) AXS_REQUIRE(mmax <= s.M, AXS_EINVAL, "m_max exceeds a body's mode cutoff");
}

// device copies of the layout offsets and the phase table for nrhs directions
struct WsTables {
    Ctx &c;
    int64_t *toff = nullptr;
    double *dirs = nullptr;
    double2 *ph = nullptr;
    WsTables(Ctx &c_, const std::vector<int64_t> &off, const double *dirs_host, int nrhs) : c(c_) {
        const int nb = (int)c.bodies.size();
        toff = (int64_t *)c.dalloc(off.size() * sizeof(int64_t));
        dirs = (double *)c.dalloc((size_t)3 * nrhs * sizeof(double));
        ph = (double2 *)c.dalloc((size_t)nrhs * nb * (nb - 1) * sizeof(double2));
        AXS_HIP(hipMemcpy(toff, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        AXS_HIP(hipMemcpy(dirs, dirs_host, (size_t)3 * nrhs * sizeof(double), hipMemcpyHostToDevice));
        const int64_t n = (int64_t)nrhs * nb * (nb - 1);
        hipLaunchKernelGGL(ws_phase_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, c.frame64, dirs,
                           nb, nrhs, c.kappa, ph);
        AXS_HIP(hipGetLastError());
    }
    ~WsTables() {
        (void)hipStreamSynchronize(c.stream);
        c.dfree(toff);
        c.dfree(dirs);
        c.dfree(ph);
    }
};

static void ws_decode(Ctx &c, const WsTables &T, const float *Y, int64_t P, int mmax, int nrhs, bool add,
                      double2 *sigma) {
    int maxn = 0;
    for (auto &s : c.shapes) maxn = std::max(maxn, s.NG * s.NF);
    const int nb = (int)c.bodies.size();
    dim3 grid((unsigned)ceil_div(maxn, 128), nb, nrhs);
    hipLaunchKernelGGL(ws_decode_kernel, grid, dim3(128), 0, c.stream, c.body_dev, T.toff, T.ph, Y, c.N, P, mmax, nb,
                       add ? 1 : 0, sigma);
    AXS_HIP(hipGetLastError());
}

static void check_dirs(const double *dirs, int nrhs) {
    for (int i = 0; i < 3 * nrhs; ++i) AXS_REQUIRE(std::isfinite(dirs[i]), AXS_ENONFINITE, "non-finite direction");
}

// ---------------------------------------------------------------------------
// hyperparameters: a flat JSON object of numbers
// ---------------------------------------------------------------------------
struct TrainParams {
    double epochs = 200, batch = 256, lr = 1e-3, lr_final = 1e-5, beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
    double seed = 5, init_seed = 4, k_min = NAN, k_max = NAN;
};

static TrainParams parse_hparams(const char *txt) {
    TrainParams hp;
    struct Key {
        const char *name;
        double *dst;
    } keys[] = {{"epochs", &hp.epochs}, {"batch", &hp.batch},   {"lr", &hp.lr},
                {"lr_final", &hp.lr_final}, {"beta1", &hp.beta1}, {"beta2", &hp.beta2},
                {"eps", &hp.eps},           {"seed", &hp.seed},   {"init_seed", &hp.init_seed},
                {"k_min", &hp.k_min},       {"k_max", &hp.k_max}};
    const char *p = txt;
    auto ws = [&]() {
        while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
    };
    ws();
    AXS_REQUIRE(*p == '{', AXS_EINVAL, "hparams: expected a JSON object");
    ++p;
    ws();
    if (*p == '}') {
        ++p;
    } else {
        for (;;) {
            ws();
            AXS_REQUIRE(*p == '"', AXS_EINVAL, "hparams: expected a quoted key");
            const char *k0 = ++p;
            while (*p && *p != '"') ++p;
            AXS_REQUIRE(*p == '"', AXS_EINVAL, "hparams: unterminated key");
            const std::string key(k0, p - k0);
            ++p;
            ws();
            AXS_REQUIRE(*p == ':', AXS_EINVAL, "hparams: expected ':'");
            ++p;
            ws();
            char *end = nullptr;
            const double v = std::strtod(p, &end);
            AXS_REQUIRE(end != p, AXS_EINVAL, "hparams: value of \"" + key + "\" is not a number");
            p = end;
            bool known = false;
            for (auto &k : keys)
                if (key == k.name) {
                    *k.dst = v;
                    known = true;
                }
            AXS_REQUIRE(known, AXS_EINVAL, "hparams: unknown key \"" + key + "\"");
            ws();
            if (*p == ',') {
                ++p;
                continue;
            }
            AXS_REQUIRE(*p == '}', AXS_EINVAL, "hparams: expected ',' or '}'");
            ++p;
            break;
        }
    }
    ws();
    AXS_REQUIRE(*p == 0, AXS_EINVAL, "hparams: trailing characters");
    return hp;
}

// counter-based generator (splitmix64 of seed + counter), the same on host and device
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}
__host__ __device__ inline double uniform01(uint64_t seed, uint64_t k) {   // in (0, 1)
    return ((double)(splitmix64(seed * 0x632be59bd9b4e019ULL + k) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// p[e] = sd sqrt(-2 log u1) cos(2 pi u2), (u1, u2) = draws k0 + 2e and k0 + 2e + 1 (Box-Muller)
__global__ void he_init_kernel(float *__restrict__ p, int64_t n, uint64_t seed, uint64_t k0, double sd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double u1 = uniform01(seed, k0 + 2 * (uint64_t)e), u2 = uniform01(seed, k0 + 2 * (uint64_t)e + 1);
    p[e] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
}

// He initialisation: W_k ~ N(0, 2 / fan_in), biases zero; the draws are
// numbered through all weight matrices in order
static void he_init(Mlp &n, uint64_t seed) {
    Ctx &c = *n.ctx;
    AXS_HIP(hipMemsetAsync(n.p, 0, n.nparams * sizeof(float), c.stream));
    uint64_t k = 0;
    for (size_t l = 0; l + 1 < n.sizes.size(); ++l) {
        const int64_t a = n.sizes[l], b = n.sizes[l + 1], cnt = a * b;
        hipLaunchKernelGGL(he_init_kernel, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, c.stream,
                           n.p + n.woff[l], cnt, seed, k, std::sqrt(2.0 / (double)a));
        AXS_HIP(hipGetLastError());
        k += 2 * (uint64_t)cnt;
    }
}

static void reset_adam(Mlp &n) {
    AXS_HIP(hipMemsetAsync(n.m, 0, n.nparams * sizeof(float), n.ctx->stream));
    AXS_HIP(hipMemsetAsync(n.v, 0, n.nparams * sizeof(float), n.ctx->stream));
    n.step = 0;
}

// multiply the last layer (weights and bias) by f: the network's output scales by f
static void scale_last_layer(Mlp &n, float f) {
    const size_t L = n.sizes.size() - 1;
    const int64_t off = n.woff[L - 1], len = n.nparams - off;
    scale_f32(*n.ctx, n.p + off, len, f, n.p + off);
}

// root mean square of n floats on the device
static double rms_f32(Ctx &c, const float *a, int64_t n) {
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(n, 256)));
    double *part = (double *)c.dalloc((size_t)nblk * sizeof(double));
    hipLaunchKernelGGL(sumsq_f32_kernel, dim3(nblk), dim3(256), 0, c.stream, a, n, part);
    AXS_HIP(hipGetLastError());
    std::vector<double> h(nblk);
    AXS_HIP(hipMemcpyAsync(h.data(), part, (size_t)nblk * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));
    c.dfree(part);
    double s = 0;
    for (double v : h) s += v;
    return std::sqrt(s / (double)n);
}

}  // namespace axs

extern "C" {

axs_status axs_warm_start_size(axs_ctx *ctx, int mmax, int64_t *P) {
    if (!ctx || !P) return AXS_EINVAL;
    Ctx &c = ctx->c;
    c.err.clear();
    try {
        axs::ws_check_mmax(c, mmax);
        std::vector<int64_t> toff;
        *P = axs::ws_layout(c, mmax, toff);
        return AXS_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    }
}

axs_status axs_warm_start_encode(axs_ctx *ctx, const void *sigma, const double *dirs, int nrhs, int mmax, float *Y) {
    if (!ctx) return AXS_EINVAL;
    Ctx &c = ctx->c;
    c.err.clear();
    try {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(c.tgt_count < 0, AXS_ESTATE, "a target-body range is set (axs_set_target_bodies)");
        AXS_REQUIRE(sigma && dirs && Y && nrhs >= 1 && nrhs <= 4096, AXS_EINVAL, "bad arguments");
        axs::ws_check_mmax(c, mmax);
        axs::check_dirs(dirs, nrhs);
        axs::require_finite(c, sigma, (int64_t)nrhs * c.N, "sigma");
        std::vector<int64_t> toff;
        const int64_t P = axs::ws_layout(c, mmax, toff);
        axs::WsTables T(c, toff, dirs, nrhs);
        const int nb = (int)c.bodies.size();
        // rhs per chunk: the masked copies (nb per rhs) stay within one inter-body
        // application (4096 rhs) and about 512 MiB per buffer
        const int64_t per_rhs = (int64_t)nb * c.N * (int64_t)sizeof(double2);
        const int nch = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nrhs, 4096 / nb,
                                                                      ((int64_t)512 << 20) / per_rhs}));
        double2 *masked = (double2 *)c.dalloc((size_t)nch * per_rhs);
        double2 *bsum = (double2 *)c.dalloc((size_t)nch * per_rhs);
        double2 *u = (double2 *)c.dalloc((size_t)nch * per_rhs);
        int maxng = 0;
        for (auto &s : c.shapes) maxng = std::max(maxng, s.NG);
        for (int c0 = 0; c0 < nrhs; c0 += nch) {
            const int ch = std::min(nch, nrhs - c0);
            const int64_t tot = (int64_t)nb * ch * c.N;
            const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(8192, axs::ceil_div(tot, 256)));
            hipLaunchKernelGGL(axs::mask_by_body_kernel, dim3(nblk), dim3(256), 0, c.stream,
                               (const double2 *)sigma + (int64_t)c0 * c.N, c.body_off, nb, ch, c.N, masked);
            AXS_HIP(hipGetLastError());
            axs::interbody_partials(c, masked, nb * ch, AXS_FP64);
            axs::interbody_reduce_to_c128(c, bsum, nb * ch, AXS_FP64);
            axs::apply_precond(c, bsum, u, nb * ch, AXS_FP64, -1.0);
            dim3 grid((unsigned)axs::ceil_div((int64_t)maxng * (2 * mmax + 1), 128), nb, ch * (nb - 1));
            hipLaunchKernelGGL(axs::ws_encode_kernel, grid, dim3(128), 0, c.stream, c.body_dev, T.toff,
                               T.ph + (int64_t)c0 * nb * (nb - 1), u, c.N, P, mmax, nb, ch, Y + (int64_t)c0 * P);
            AXS_HIP(hipGetLastError());
        }
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(masked);
        c.dfree(bsum);
        c.dfree(u);
        return AXS_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    }
}

axs_status axs_warm_start_decode(axs_ctx *ctx, const float *Y, const double *dirs, int nrhs, int mmax,
                                 void *sigma) {
    if (!ctx) return AXS_EINVAL;
    Ctx &c = ctx->c;
    c.err.clear();
    try {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(sigma && dirs && Y && nrhs >= 1 && nrhs <= 4096, AXS_EINVAL, "bad arguments");
        axs::ws_check_mmax(c, mmax);
        axs::check_dirs(dirs, nrhs);
        std::vector<int64_t> toff;
        const int64_t P = axs::ws_layout(c, mmax, toff);
        axs::WsTables T(c, toff, dirs, nrhs);
        axs::ws_decode(c, T, Y, P, mmax, nrhs, false, (double2 *)sigma);
        AXS_HIP(hipStreamSynchronize(c.stream));
        return AXS_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    }
}

axs_status axs_mlp_train(axs_mlp *h, const float *X, const float *Y, int64_t S, const char *hparams,
                         double *loss_per_epoch) {
    if (!hparams) return AXS_EINVAL;
    return mlp_guarded(h, [&](Mlp &n, Ctx &c) -> axs_status {
        AXS_REQUIRE(X && Y && S >= 1, AXS_EINVAL, "bad arguments");
        AXS_REQUIRE(S <= INT32_MAX, AXS_EINVAL, "more than 2^31 - 1 samples");
        AXS_REQUIRE(n.sizes.front() == 4, AXS_EINVAL, "the network input must be (d_x, d_y, d_z, k)");
        const axs::TrainParams hp = axs::parse_hparams(hparams);
        AXS_REQUIRE(std::isfinite(hp.k_min) && std::isfinite(hp.k_max) && hp.k_max > hp.k_min, AXS_EINVAL,
                    "hparams: k_min < k_max are required");
        AXS_REQUIRE(hp.epochs >= 1 && hp.epochs <= 1e6 && hp.batch >= 1 && hp.batch <= 65536, AXS_EINVAL,
                    "hparams: epochs in [1, 1e6], batch in [1, 65536]");
        AXS_REQUIRE(hp.lr > 0 && hp.lr_final > 0 && hp.beta1 >= 0 && hp.beta1 < 1 && hp.beta2 >= 0 &&
                        hp.beta2 < 1 && hp.eps > 0,
                    AXS_EINVAL, "hparams: lr, lr_final, eps > 0 and beta1, beta2 in [0, 1)");
        const int epochs = (int)hp.epochs;
        const int batch = (int)std::min<int64_t>((int64_t)hp.batch, S);
        const int L = (int)n.sizes.size() - 1;
        const int64_t nout = n.sizes[L];
        // target scale: the root mean square of Y, folded into the last layer at the end
        double scale = axs::rms_f32(c, Y, S * nout);
        AXS_REQUIRE(std::isfinite(scale), AXS_ENONFINITE, "non-finite training targets");
        if (!(scale > 0)) scale = 1.0;
        float *Xs = (float *)c.dalloc((size_t)S * 4 * sizeof(float));
        float *Ys = (float *)c.dalloc((size_t)S * nout * sizeof(float));
        hipLaunchKernelGGL(axs::ws_features_kernel, dim3((unsigned)axs::ceil_div(S, 256)), dim3(256), 0, c.stream, X,
                           S, hp.k_min, hp.k_max, Xs);
        AXS_HIP(hipGetLastError());
        axs::scale_f32(c, Y, S * nout, (float)(1.0 / scale), Ys);
        if (hp.init_seed >= 0)
            axs::he_init(n, (uint64_t)hp.init_seed);
        else
            axs::scale_last_layer(n, (float)(1.0 / scale));   // continue from the current network
        axs::reset_adam(n);
        const int steps = (int)std::max<int64_t>(1, S / batch);
        const int64_t total = (int64_t)epochs * steps;
        std::vector<int32_t> perm((size_t)S), order((size_t)steps * batch);
        std::vector<double> lrs(steps);
        const uint64_t seed = (uint64_t)hp.seed;
        uint64_t draw = 0;
        for (int ep = 0; ep < epochs; ++ep) {
            // a fresh permutation per epoch (Fisher-Yates); its first steps x batch rows
            for (int64_t i = 0; i < S; ++i) perm[(size_t)i] = (int32_t)i;
            for (int64_t i = S - 1; i > 0; --i) {
                const int64_t j = (int64_t)(axs::uniform01(seed, draw++) * (double)(i + 1));
                std::swap(perm[(size_t)i], perm[(size_t)std::min(j, i)]);
            }
            std::copy(perm.begin(), perm.begin() + (int64_t)steps * batch, order.begin());
            // cosine decay from lr to lr_final over all steps
            for (int s = 0; s < steps; ++s) {
                const double t = (double)((int64_t)ep * steps + s) / (double)std::max<int64_t>(1, total - 1);
                lrs[s] = hp.lr_final + 0.5 * (hp.lr - hp.lr_final) * (1.0 + std::cos(M_PI * t));
            }
            axs::load_order(n, order.data(), (int64_t)steps * batch);
            axs::queue_steps(n, Xs, Ys, batch, steps, lrs.data(), hp.beta1, hp.beta2, hp.eps);
            if (loss_per_epoch) {
                AXS_HIP(hipMemcpyAsync(&loss_per_epoch[ep], n.loss_dev, sizeof(double), hipMemcpyDeviceToHost,
                                       c.stream));
                AXS_HIP(hipStreamSynchronize(c.stream));
            }
        }
        axs::scale_last_layer(n, (float)scale);
        axs::reset_adam(n);
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(Xs);
        c.dfree(Ys);
        return AXS_OK;
    });
}

axs_status axs_mlp_predict(axs_mlp *h, axs_ctx *ctx, const double *dirs, const double *kappas, int nrhs,
                           const double k_range[2], void *sigma0) {
    if (!h || !h->n.ctx || !ctx) return AXS_EINVAL;
    Ctx &c = ctx->c;
    Mlp &n = h->n;
    c.err.clear();
    try {
        AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
        AXS_REQUIRE(c.tgt_count < 0, AXS_ESTATE, "a target-body range is set (axs_set_target_bodies)");
        AXS_REQUIRE(n.ctx->device == c.device, AXS_EINVAL, "network and context on different devices");
        AXS_REQUIRE(dirs && k_range && sigma0 && nrhs >= 1 && nrhs <= 4096, AXS_EINVAL, "bad arguments");
        AXS_REQUIRE(std::isfinite(k_range[0]) && std::isfinite(k_range[1]) && k_range[1] > k_range[0], AXS_EINVAL,
                    "k_range must be finite with k_range[0] < k_range[1]");
        AXS_REQUIRE(n.sizes.front() == 4, AXS_EINVAL, "the network input must be (d_x, d_y, d_z, k)");
        const int L = (int)n.sizes.size() - 1;
        const int mmax = axs::ws_mmax_for(c, n.sizes[L]);
        AXS_REQUIRE(mmax >= 0, AXS_EINVAL, "the network's output size is not the warm-start layout of this context");
        axs::ws_check_mmax(c, mmax);
        axs::check_dirs(dirs, nrhs);
        if (kappas)
            for (int i = 0; i < nrhs; ++i)
                AXS_REQUIRE(std::fabs(kappas[i] - c.kappa) <= 1e-12 * std::max(1.0, c.kappa), AXS_EINVAL,
                            "kappas must equal the context's wavenumber (its discretisation and matrices are for it)");
        // features and the forward pass on the network's stream
        std::vector<float> xf((size_t)4 * nrhs);
        const double ks = (2.0 * c.kappa - (k_range[0] + k_range[1])) / (k_range[1] - k_range[0]);
        for (int i = 0; i < nrhs; ++i) {
            for (int a = 0; a < 3; ++a) xf[(size_t)4 * i + a] = (float)dirs[3 * i + a];
            xf[(size_t)4 * i + 3] = (float)ks;
        }
        float *xd = (float *)n.ctx->dalloc(xf.size() * sizeof(float));
        AXS_HIP(hipMemcpy(xd, xf.data(), xf.size() * sizeof(float), hipMemcpyHostToDevice));
        axs::mlp_forward(n, xd, nrhs);
        AXS_HIP(hipStreamSynchronize(n.ctx->stream));
        n.ctx->dfree(xd);
        // sigma0 = b~ = -D^{-1} v, then the decoded multiple-scattering part on top
        std::vector<int64_t> toff;
        const int64_t P = axs::ws_layout(c, mmax, toff);
        axs::WsTables T(c, toff, dirs, nrhs);
        double2 *v = (double2 *)c.dalloc((size_t)nrhs * c.N * sizeof(double2));
        axs::incident_plane_launch(c, T.dirs, nrhs, v);
        axs::apply_precond(c, v, sigma0, nrhs, AXS_FP64, -1.0);
        axs::ws_decode(c, T, n.H[L], P, mmax, nrhs, true, (double2 *)sigma0);
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(v);
        return AXS_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        c.err = e.what();
        return AXS_EINVAL;
    }
}

}  // extern "C"
