// Inter-body operator B (Sec. 3.3 naive-rule blocks, applied in Sec. 4), field
// evaluation (eq. "intHelm1") and incident fields, hand-written for gfx950.
//
// B sigma is a direct sum over every (target, source) pair on different bodies,
//   (B sigma)_i = sum_{j notin body(i)} G(x_i, x_j) q_j,   q_j = w_j sigma_j / (4 pi)
//   G * 4 pi = e^{i k R}/R [ (n_j . d)(1 - i k R)/R^2 + i eta ],  d = x_i - x_j.
// It replaces the paper's FMM by an exact O(N^2) sum that runs on the VALU:
//   - a block owns a tile of targets inside ONE body (so same-body exclusion is
//     two contiguous source ranges, no per-pair mask) and one chunk of the
//     remaining sources; partial sums per chunk are reduced later in a fixed
//     order, so results are bitwise reproducible (no float atomics);
//   - sources are streamed through LDS in tiles loaded with coalesced SoA reads
//     and read back as LDS broadcasts; each thread keeps TPT targets and their
//     complex accumulators in registers;
//   - FP32 path: phase reduced in revolutions (v_fract) and fed to the
//     hardware sin/cos (which take revolutions), 1/R from v_rsq;
//   - FP64 path: the same structure with libm sincospi / rsqrt.
#include "axs_internal.h"

namespace axs {

template <typename R> struct C2T;
template <> struct C2T<float> { using T = float2; };
template <> struct C2T<double> { using T = double2; };

__device__ __forceinline__ void sincos_rev(float ph, float &s, float &c) {
    float f = __builtin_amdgcn_fractf(ph);   // [0, 1)
    s = __builtin_amdgcn_sinf(f);            // sin(2 pi f)
    c = __builtin_amdgcn_cosf(f);
}
__device__ __forceinline__ void sincos_rev(double ph, double &s, double &c) {
    double f = ph - rint(ph);                // exact, in [-1/2, 1/2]
    sincospi(2.0 * f, &s, &c);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

// LDS stride (in elements) of one staged source: x y z nx ny nz + NR complex q,
// rounded up to 16 bytes so the compiler can use 128-bit LDS reads.
template <typename R, int NR> struct SrcStride {
    static constexpr int raw = 6 + 2 * NR;
    static constexpr int per16 = 16 / sizeof(R);
    static constexpr int value = (raw + per16 - 1) / per16 * per16;
};

template <typename R, int TPT, int NR, int BS>
__global__ __launch_bounds__(BS) void interbody_kernel(
    const IBWork *__restrict__ work, const R *__restrict__ geo, const typename C2T<R>::T *__restrict__ q,
    int64_t N, int nrhs, int c0, R kappa, R k2pi, R eta, typename C2T<R>::T *__restrict__ part) {
    using R2 = typename C2T<R>::T;
    constexpr int ST = SrcStride<R, NR>::value;
    __shared__ __align__(16) R tile[BS * ST];

    const IBWork w = work[blockIdx.x];
    const int tid = threadIdx.x;
    const R *gx = geo, *gy = geo + N, *gz = geo + 2 * N;
    const R *gnx = geo + 3 * N, *gny = geo + 4 * N, *gnz = geo + 5 * N;

    R tx[TPT], ty[TPT], tz[TPT];
    R ar[TPT][NR], ai[TPT][NR];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        int t = tid + k * BS;
        int64_t gi = w.t0 + (t < w.tn ? t : 0);
        tx[k] = gx[gi];
        ty[k] = gy[gi];
        tz[k] = gz[gi];
#pragma unroll
        for (int c = 0; c < NR; ++c) ar[k][c] = ai[k][c] = R(0);
    }

#pragma unroll 1
    for (int rng = 0; rng < 2; ++rng) {
        const int lo = rng == 0 ? w.s0 : w.s2;
        const int hi = rng == 0 ? w.s1 : w.s3;
#pragma unroll 1
        for (int base = lo; base < hi; base += BS) {
            const int cnt = min(BS, hi - base);
            __syncthreads();
            if (tid < cnt) {
                const int64_t j = base + tid;
                R *d = tile + tid * ST;
                d[0] = gx[j];
                d[1] = gy[j];
                d[2] = gz[j];
                d[3] = gnx[j];
                d[4] = gny[j];
                d[5] = gnz[j];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    R2 v = q[(int64_t)(c0 + c) * N + j];
                    d[6 + 2 * c] = v.x;
                    d[7 + 2 * c] = v.y;
                }
            }
            __syncthreads();
#pragma unroll 2
            for (int js = 0; js < cnt; ++js) {
                const R *s = tile + js * ST;
                const R sx = s[0], sy = s[1], sz = s[2], snx = s[3], sny = s[4], snz = s[5];
                R qr[NR], qi[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    qr[c] = s[6 + 2 * c];
                    qi[c] = s[7 + 2 * c];
                }
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    const R dx = tx[k] - sx, dy = ty[k] - sy, dz = tz[k] - sz;
                    const R r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    const R ri = rsq(r2);
                    const R rr = r2 * ri;
                    const R nd = fma(snx, dx, fma(sny, dy, snz * dz));
                    R sn, cs;
                    sincos_rev(rr * k2pi, sn, cs);
                    const R a = nd * ri * ri;                 // (n.d)/R^2
                    const R bim = fma(-a * kappa, rr, eta);   // eta - a k R
                    const R er = cs * ri, ei = sn * ri;       // e^{ikR}/R
                    const R gr = fma(er, a, -ei * bim);
                    const R gi = fma(er, bim, ei * a);
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        ar[k][c] = fma(gr, qr[c], fma(-gi, qi[c], ar[k][c]));
                        ai[k][c] = fma(gr, qi[c], fma(gi, qr[c], ai[k][c]));
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        int t = tid + k * BS;
        if (t < w.tn) {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                R2 v;
                v.x = ar[k][c];
                v.y = ai[k][c];
                part[((int64_t)w.slot * nrhs + c0 + c) * N + w.t0 + t] = v;
            }
        }
    }
}

// q[c][j] = w_j sigma[c][j] / (4 pi) in precision R
template <typename R>
__global__ void stage_density_kernel(const double2 *__restrict__ sigma, const double *__restrict__ w,
                                     int64_t N, int64_t total, typename C2T<R>::T *__restrict__ q) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double s = w[i % N] * (0.25 / M_PI);
    double2 v = sigma[i];
    typename C2T<R>::T o;
    o.x = (R)(v.x * s);
    o.y = (R)(v.y * s);
    q[i] = o;
}

template <typename R>
__global__ void reduce_parts_kernel(const typename C2T<R>::T *__restrict__ part, int splits,
                                    int64_t total, double2 *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double re = 0, im = 0;
    for (int s = 0; s < splits; ++s) {
        auto v = part[(int64_t)s * total + i];
        re += (double)v.x;
        im += (double)v.y;
    }
    y[i] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int default_tpt(int prec) { return prec == AXS_FP32 ? 4 : 2; }
static int default_block(int) { return 256; }

int interbody_splits(Ctx &c, int prec) {
    int pi = prec == AXS_FP32 ? 1 : 0;
    if (c.ib_splits[pi] > 0) return c.ib_splits[pi];
    // enough blocks to fill 256 CUs several times over
    int tpt = c.ib_tpt[pi] > 0 ? c.ib_tpt[pi] : default_tpt(prec);
    int bs = c.ib_block[pi] > 0 ? c.ib_block[pi] : default_block(prec);
    int64_t tiles = 0;
    for (auto &b : c.bodies) tiles += ceil_div(b.n, (int64_t)tpt * bs);
    int s = 1;
    while (tiles * s < 4096 && s < 64) s *= 2;
    return s;
}

static std::vector<IBWork> build_work(Ctx &c, int tile, int splits) {
    std::vector<IBWork> out;
    const int64_t N = c.N;
    for (auto &b : c.bodies) {
        const int64_t others = N - b.n;
        const int64_t chunk = ceil_div(std::max<int64_t>(others, 1), splits);
        for (int64_t t0 = 0; t0 < b.n; t0 += tile) {
            for (int s = 0; s < splits; ++s) {
                IBWork w{};
                w.t0 = (int32_t)(b.offset + t0);
                w.tn = (int32_t)std::min<int64_t>(tile, b.n - t0);
                int64_t v0 = std::min<int64_t>(others, (int64_t)s * chunk);
                int64_t v1 = std::min<int64_t>(others, v0 + chunk);
                // virtual index v < offset -> v ; v >= offset -> v + n
                int64_t a0 = v0, a1 = std::min<int64_t>(v1, b.offset);
                if (a1 < a0) a1 = a0;
                int64_t b0 = std::max<int64_t>(v0, b.offset), b1 = v1;
                if (b1 < b0) b1 = b0;
                w.s0 = (int32_t)a0;
                w.s1 = (int32_t)a1;
                w.s2 = (int32_t)(b0 + b.n);
                w.s3 = (int32_t)(b1 + b.n);
                w.slot = s;
                out.push_back(w);
            }
        }
    }
    return out;
}

template <typename R, int TPT, int BS>
static void launch_ib(Ctx &c, const IBWork *work, int nwork, const R *geo,
                      const typename C2T<R>::T *q, int nrhs, typename C2T<R>::T *part) {
    const R kappa = (R)c.kappa, k2pi = (R)(c.kappa / (2.0 * M_PI)), eta = (R)c.eta;
    int c0 = 0;
    while (c0 < nrhs) {
        int left = nrhs - c0;
        if (left >= 8) {
            hipLaunchKernelGGL((interbody_kernel<R, TPT, 8, BS>), dim3(nwork), dim3(BS), 0, c.stream,
                               work, geo, q, c.N, nrhs, c0, kappa, k2pi, eta, part);
            c0 += 8;
        } else if (left >= 4) {
            hipLaunchKernelGGL((interbody_kernel<R, TPT, 4, BS>), dim3(nwork), dim3(BS), 0, c.stream,
                               work, geo, q, c.N, nrhs, c0, kappa, k2pi, eta, part);
            c0 += 4;
        } else if (left >= 2) {
            hipLaunchKernelGGL((interbody_kernel<R, TPT, 2, BS>), dim3(nwork), dim3(BS), 0, c.stream,
                               work, geo, q, c.N, nrhs, c0, kappa, k2pi, eta, part);
            c0 += 2;
        } else {
            hipLaunchKernelGGL((interbody_kernel<R, TPT, 1, BS>), dim3(nwork), dim3(BS), 0, c.stream,
                               work, geo, q, c.N, nrhs, c0, kappa, k2pi, eta, part);
            c0 += 1;
        }
        AXS_HIP(hipGetLastError());
    }
}

template <typename R>
static void dispatch_ib(Ctx &c, int tpt, int bs, const IBWork *work, int nwork, const R *geo,
                        const typename C2T<R>::T *q, int nrhs, typename C2T<R>::T *part) {
#define AXS_IB_CASE(T_, B_)                                                 \
    if (tpt == T_ && bs == B_) {                                            \
        launch_ib<R, T_, B_>(c, work, nwork, geo, q, nrhs, part);           \
        return;                                                             \
    }
    AXS_IB_CASE(1, 256)
    AXS_IB_CASE(2, 256)
    AXS_IB_CASE(4, 256)
    AXS_IB_CASE(8, 256)
    AXS_IB_CASE(1, 128)
    AXS_IB_CASE(2, 128)
    AXS_IB_CASE(4, 128)
#undef AXS_IB_CASE
    throw Error{AXS_EINVAL, "unsupported inter-body launch shape (targets/thread, block)"};
}

void interbody_partials(Ctx &c, const void *sigma, int nrhs, int prec) {
    const int pi = prec == AXS_FP32 ? 1 : 0;
    const int tpt = c.ib_tpt[pi] > 0 ? c.ib_tpt[pi] : default_tpt(prec);
    const int bs = c.ib_block[pi] > 0 ? c.ib_block[pi] : default_block(prec);
    const int splits = interbody_splits(c, prec);
    if (!c.ib_work[pi] || c.ib_key[pi][0] != tpt || c.ib_key[pi][1] != bs || c.ib_key[pi][2] != splits) {
        // work tables are cached per launch shape; rebuilt only when it changes
        std::vector<IBWork> work = build_work(c, tpt * bs, splits);
        if (c.ib_work[pi]) {
            AXS_HIP(hipStreamSynchronize(c.stream));
            c.dfree(c.ib_work[pi]);
        }
        c.ib_work[pi] = (IBWork *)c.dalloc(work.size() * sizeof(IBWork));
        AXS_HIP(hipMemcpy(c.ib_work[pi], work.data(), work.size() * sizeof(IBWork), hipMemcpyHostToDevice));
        c.ib_nwork[pi] = (int)work.size();
        c.ib_key[pi][0] = tpt;
        c.ib_key[pi][1] = bs;
        c.ib_key[pi][2] = splits;
    }
    const IBWork *dwork = c.ib_work[pi];
    const int nwork = c.ib_nwork[pi];
    const int64_t total = (int64_t)nrhs * c.N;
    const int thr = 256;
    if (prec == AXS_FP32) {
        float2 *q = (float2 *)c.scratch(WS_Q, total * sizeof(float2));
        float2 *part = (float2 *)c.scratch(WS_PART, (size_t)splits * total * sizeof(float2));
        hipLaunchKernelGGL(stage_density_kernel<float>, dim3(ceil_div(total, thr)), dim3(thr), 0,
                           c.stream, (const double2 *)sigma, c.g64 + 6 * c.N, c.N, total, q);
        AXS_HIP(hipGetLastError());
        dispatch_ib<float>(c, tpt, bs, dwork, nwork, c.g32, q, nrhs, part);
    } else {
        double2 *q = (double2 *)c.scratch(WS_Q, total * sizeof(double2));
        double2 *part = (double2 *)c.scratch(WS_PART, (size_t)splits * total * sizeof(double2));
        hipLaunchKernelGGL(stage_density_kernel<double>, dim3(ceil_div(total, thr)), dim3(thr), 0,
                           c.stream, (const double2 *)sigma, c.g64 + 6 * c.N, c.N, total, q);
        AXS_HIP(hipGetLastError());
        dispatch_ib<double>(c, tpt, bs, dwork, nwork, c.g64, q, nrhs, part);
    }
}

void interbody_reduce_to_c128(Ctx &c, void *y, int nrhs, int prec) {
    const int splits = interbody_splits(c, prec);
    const int64_t total = (int64_t)nrhs * c.N;
    const int thr = 256;
    if (prec == AXS_FP32)
        hipLaunchKernelGGL(reduce_parts_kernel<float>, dim3(ceil_div(total, thr)), dim3(thr), 0, c.stream,
                           (const float2 *)c.scratch(WS_PART, 0), splits, total, (double2 *)y);
    else
        hipLaunchKernelGGL(reduce_parts_kernel<double>, dim3(ceil_div(total, thr)), dim3(thr), 0, c.stream,
                           (const double2 *)c.scratch(WS_PART, 0), splits, total, (double2 *)y);
    AXS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// field evaluation off the surface: few targets, all sources.  One block per
// (target, rhs); threads stride the sources and the complex sums are reduced
// with wavefront shuffles, then across the block's waves in LDS (fixed order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int BS>
__device__ __forceinline__ double2 block_sum2(double re, double im) {
    __shared__ double sr[BS / 64], si[BS / 64];
    re = wave_sum(re);
    im = wave_sum(im);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sr[wv] = re;
        si[wv] = im;
    }
    __syncthreads();
    double2 out = make_double2(0, 0);
    if (threadIdx.x == 0) {
        for (int k = 0; k < BS / 64; ++k) {
            out.x += sr[k];
            out.y += si[k];
        }
    }
    return out;
}

template <int BS>
__global__ __launch_bounds__(BS) void eval_field_kernel(const double *__restrict__ g, int64_t N,
                                                        const double2 *__restrict__ sigma,
                                                        const double *__restrict__ tgt, int nt,
                                                        double kappa, double eta,
                                                        double2 *__restrict__ u) {
    const int t = blockIdx.x, c = blockIdx.y;
    const double tx = tgt[3 * t], ty = tgt[3 * t + 1], tz = tgt[3 * t + 2];
    const double2 *sg = sigma + (int64_t)c * N;
    double re = 0, im = 0;
    for (int64_t j = threadIdx.x; j < N; j += BS) {
        const double dx = tx - g[j], dy = ty - g[N + j], dz = tz - g[2 * N + j];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double R = sqrt(r2);
        const double nd = g[3 * N + j] * dx + g[4 * N + j] * dy + g[5 * N + j] * dz;
        double s, cs;
        sincos(kappa * R, &s, &cs);
        const double a = nd / r2, bim = eta - a * kappa * R;
        const double er = cs / R, ei = s / R;
        const double gr = er * a - ei * bim, gi = er * bim + ei * a;
        const double w = g[6 * N + j] * (0.25 / M_PI);
        const double qr = sg[j].x * w, qi = sg[j].y * w;
        re += gr * qr - gi * qi;
        im += gr * qi + gi * qr;
    }
    double2 tot = block_sum2<BS>(re, im);
    if (threadIdx.x == 0) u[(int64_t)c * nt + t] = tot;
}

template <int BS>
__global__ __launch_bounds__(BS) void far_field_kernel(const double *__restrict__ g, int64_t N,
                                                       const double2 *__restrict__ sigma,
                                                       const double *__restrict__ xh, int nd,
                                                       double kappa, double eta,
                                                       double2 *__restrict__ u) {
    const int t = blockIdx.x, c = blockIdx.y;
    const double hx = xh[3 * t], hy = xh[3 * t + 1], hz = xh[3 * t + 2];
    const double2 *sg = sigma + (int64_t)c * N;
    double re = 0, im = 0;
    for (int64_t j = threadIdx.x; j < N; j += BS) {
        const double ph = -kappa * (hx * g[j] + hy * g[N + j] + hz * g[2 * N + j]);
        double s, cs;
        sincos(ph, &s, &cs);
        // (-i k xh.n + i eta) e^{i ph}
        const double fim = -kappa * (hx * g[3 * N + j] + hy * g[4 * N + j] + hz * g[5 * N + j]) + eta;
        const double gr = -fim * s, gi = fim * cs;
        const double w = g[6 * N + j] * (0.25 / M_PI);
        const double qr = sg[j].x * w, qi = sg[j].y * w;
        re += gr * qr - gi * qi;
        im += gr * qi + gi * qr;
    }
    double2 tot = block_sum2<BS>(re, im);
    if (threadIdx.x == 0) u[(int64_t)c * nd + t] = tot;
}

void eval_field_launch(Ctx &c, const void *sigma, int nrhs, const double *tgt_dev, int nt, void *u) {
    hipLaunchKernelGGL(eval_field_kernel<256>, dim3(nt, nrhs), dim3(256), 0, c.stream, c.g64, c.N,
                       (const double2 *)sigma, tgt_dev, nt, c.kappa, c.eta, (double2 *)u);
    AXS_HIP(hipGetLastError());
}

void far_field_launch(Ctx &c, const void *sigma, int nrhs, const double *xh_dev, int nd, void *u) {
    hipLaunchKernelGGL(far_field_kernel<256>, dim3(nd, nrhs), dim3(256), 0, c.stream, c.g64, c.N,
                       (const double2 *)sigma, xh_dev, nd, c.kappa, c.eta, (double2 *)u);
    AXS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// incident fields at the nodes
// ---------------------------------------------------------------------------
__global__ void plane_wave_kernel(const double *__restrict__ g, int64_t N, const double *__restrict__ dirs,
                                  int nrhs, double kappa, double2 *__restrict__ v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * nrhs) return;
    int c = (int)(i / N);
    int64_t j = i - (int64_t)c * N;
    double ph = kappa * (dirs[3 * c] * g[j] + dirs[3 * c + 1] * g[N + j] + dirs[3 * c + 2] * g[2 * N + j]);
    double s, cs;
    sincos(ph, &s, &cs);
    v[i] = make_double2(cs, s);
}

__global__ void point_source_kernel(const double *__restrict__ g, int64_t N, const double *__restrict__ src,
                                    const double *__restrict__ amp, int ns, double kappa,
                                    double2 *__restrict__ v) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double re = 0, im = 0;
    for (int s = 0; s < ns; ++s) {
        double dx = g[j] - src[3 * s], dy = g[N + j] - src[3 * s + 1], dz = g[2 * N + j] - src[3 * s + 2];
        double R = sqrt(dx * dx + dy * dy + dz * dz);
        double sn, cs;
        sincos(kappa * R, &sn, &cs);
        double f = 0.25 / (M_PI * R);
        double pr = cs * f, pi = sn * f;
        re += pr * amp[2 * s] - pi * amp[2 * s + 1];
        im += pr * amp[2 * s + 1] + pi * amp[2 * s];
    }
    v[j] = make_double2(re, im);
}

void incident_plane_launch(Ctx &c, const double *dirs_dev, int nrhs, void *v) {
    int64_t total = c.N * nrhs;
    hipLaunchKernelGGL(plane_wave_kernel, dim3(ceil_div(total, 256)), dim3(256), 0, c.stream, c.g64,
                       c.N, dirs_dev, nrhs, c.kappa, (double2 *)v);
    AXS_HIP(hipGetLastError());
}

void incident_point_launch(Ctx &c, const double *src_dev, const double *amp_dev, int ns, void *v) {
    hipLaunchKernelGGL(point_source_kernel, dim3(ceil_div(c.N, 256)), dim3(256), 0, c.stream, c.g64, c.N,
                       src_dev, amp_dev, ns, c.kappa, (double2 *)v);
    AXS_HIP(hipGetLastError());
}

}  // namespace axs
