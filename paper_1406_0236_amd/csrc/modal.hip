// The block-diagonal preconditioner D^{-1} = blockdiag(F* S F) (Sec. 3.2 eq.
// "singleinverse", Sec. 4 Remark on the cost of D^{-1} B sigma):
//   (1) forward DFT in the azimuth of every body,
//   (2) per Fourier mode, apply the stored S_|m| = A~_|m|^{-1} (A~_{-m} = A~_m),
//   (3) inverse DFT, optionally adding the identity term of eq. "precond".
// N_F = 2M + 1 is odd and small (41, 81), so the DFT is a direct sum with the
// twiddle table and the input rows staged in LDS (same result as an FFT).
// Step (2) is a batched complex GEMM on the matrix cores: for each shape and
// |m| the columns are (+m, -m) x (bodies of that shape) x (right-hand sides),
// and the complex product is four real MFMA products on planar operands.
#include "axs_internal.h"

namespace axs {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

constexpr int DFT_GI = 16;     // contour nodes per DFT block
constexpr int DFT_BS = 256;

__device__ __forceinline__ int64_t xelem(const BodyDev &b, int nrhs, int k, int c, int i) {
    const int m = k <= b.M ? k : k - b.NF;
    const int am = m < 0 ? -m : m;
    const int sgn = m < 0 ? 1 : 0;
    const int64_t colbase = (int64_t)b.nb * nrhs * (am == 0 ? 0 : 2 * am - 1);
    const int64_t col = (int64_t)(sgn * b.nb + b.local) * nrhs + c;
    return (int64_t)nrhs * b.xoff + (colbase + col) * b.NG + i;
}

// X[k][i] = sum_l w[i][l] e^{-2 pi i k l / N_F} for the body's contour nodes
// [i0, i0 + GI) and rhs c.  Input: sum over `splits` partial inter-body sums
// (from_vec = 0) or a complex128 vector (from_vec = 1).
template <typename R>
__global__ __launch_bounds__(DFT_BS) void dft_forward_kernel(
    const BodyDev *__restrict__ bodies, const typename CT<R>::T *__restrict__ part, int splits,
    const double2 *__restrict__ vec, int from_vec, int64_t N, int nrhs, const R *__restrict__ tw,
    R *__restrict__ Xr, R *__restrict__ Xi) {
    using R2 = typename CT<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    R2 *w = (R2 *)smem;                         // [GI][NF]
    const BodyDev b = bodies[blockIdx.z];
    const int c = blockIdx.y;
    const int i0 = blockIdx.x * DFT_GI;
    if (i0 >= b.NG) return;
    const int ni = min(DFT_GI, b.NG - i0);
    const int NF = b.NF;
    R2 *t = w + DFT_GI * NF;                    // [NF] twiddles (cos, sin)(2 pi j / NF)
    for (int j = threadIdx.x; j < NF; j += DFT_BS) {
        t[j].x = tw[2 * (b.twoff + j)];
        t[j].y = tw[2 * (b.twoff + j) + 1];
    }
    const int64_t base = b.offset + (int64_t)i0 * NF;
    for (int idx = threadIdx.x; idx < ni * NF; idx += DFT_BS) {
        R2 v;
        if (from_vec) {
            double2 d = vec[(int64_t)c * N + base + idx];
            v.x = (R)d.x;
            v.y = (R)d.y;
        } else {
            v.x = R(0);
            v.y = R(0);
            for (int s = 0; s < splits; ++s) {
                R2 p = part[((int64_t)s * nrhs + c) * N + base + idx];
                v.x += p.x;
                v.y += p.y;
            }
        }
        w[idx] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < ni * NF; idx += DFT_BS) {
        const int k = idx / ni, i = idx - k * ni;
        R re = 0, im = 0;
        int tj = 0;
        const R2 *row = w + i * NF;
        for (int l = 0; l < NF; ++l) {
            const R2 x = row[l], e = t[tj];
            // x * conj(e)
            re = fma(x.x, e.x, fma(x.y, e.y, re));
            im = fma(x.y, e.x, fma(-x.x, e.y, im));
            tj += k;
            if (tj >= NF) tj -= NF;
        }
        const int64_t o = xelem(b, nrhs, k, c, i0 + i);
        Xr[o] = re;
        Xi[o] = im;
    }
}

// y[c][node] = alpha sigma[c][node] + beta / N_F sum_k Y[k][i] e^{+2 pi i k l / N_F}
template <typename R>
__global__ __launch_bounds__(DFT_BS) void dft_inverse_kernel(
    const BodyDev *__restrict__ bodies, const R *__restrict__ Yr, const R *__restrict__ Yi, int64_t N,
    int nrhs, const R *__restrict__ tw, const double2 *__restrict__ sigma, double alpha, double beta,
    double2 *__restrict__ y) {
    using R2 = typename CT<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    R2 *yh = (R2 *)smem;                        // [GI][NF] (i-major)
    const BodyDev b = bodies[blockIdx.z];
    const int c = blockIdx.y;
    const int i0 = blockIdx.x * DFT_GI;
    if (i0 >= b.NG) return;
    const int ni = min(DFT_GI, b.NG - i0);
    const int NF = b.NF;
    R2 *t = yh + DFT_GI * NF;
    for (int j = threadIdx.x; j < NF; j += DFT_BS) {
        t[j].x = tw[2 * (b.twoff + j)];
        t[j].y = tw[2 * (b.twoff + j) + 1];
    }
    for (int idx = threadIdx.x; idx < ni * NF; idx += DFT_BS) {
        const int k = idx / ni, i = idx - k * ni;
        const int64_t o = xelem(b, nrhs, k, c, i0 + i);
        R2 v;
        v.x = Yr[o];
        v.y = Yi[o];
        yh[i * NF + k] = v;
    }
    __syncthreads();
    const double scale = beta / NF;
    const int64_t base = b.offset + (int64_t)i0 * NF;
    for (int idx = threadIdx.x; idx < ni * NF; idx += DFT_BS) {
        const int i = idx / NF, l = idx - i * NF;
        R re = 0, im = 0;
        int tj = 0;
        const R2 *row = yh + i * NF;
        for (int k = 0; k < NF; ++k) {
            const R2 x = row[k], e = t[tj];
            re = fma(x.x, e.x, fma(-x.y, e.y, re));
            im = fma(x.y, e.x, fma(x.x, e.y, im));
            tj += l;
            if (tj >= NF) tj -= NF;
        }
        const int64_t g = (int64_t)c * N + base + idx;
        double2 out = make_double2(scale * (double)re, scale * (double)im);
        if (alpha != 0.0) {
            const double2 s = sigma[g];
            out.x += alpha * s.x;
            out.y += alpha * s.y;
        }
        y[g] = out;
    }
}

// ---------------------------------------------------------------------------
// batched complex GEMM on MFMA:  Y = S X  per (shape, |m|)
// S planar column-major (element (i, k) at k*NG + i); X, Y planar column-major
// with leading dimension NG.  One 256-thread block computes a 32 x 32 tile,
// each wave a 16 x 16 tile with the 16x16x4 MFMA (k steps of 4).
// Operand layout of the 16x16x4 MFMA (one block of 16x16): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it receives column l % 16 of D in
// four registers v = 0..3, rows 4 (l / 16) + v for FP32 and (l / 16) + 4 v for
// FP64 (the FP64 result is not row-grouped).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename R> struct V4;
template <> struct V4<float> {
    using T = f32x4;
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct V4<double> {
    using T = f64x4;
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename R>
__global__ __launch_bounds__(256) void modal_gemm_kernel(const GemmBatch *__restrict__ batches, int nrhs,
                                                         const R *__restrict__ Sr, const R *__restrict__ Si,
                                                         const R *__restrict__ Xr, const R *__restrict__ Xi,
                                                         R *__restrict__ Yr, R *__restrict__ Yi) {
    using V = typename V4<R>::T;
    const GemmBatch bt = batches[blockIdx.z];
    const int NG = bt.NG;
    const int ncols = bt.ncols * nrhs;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = blockIdx.x * 32 + (wave >> 1) * 16;
    const int c0 = blockIdx.y * 32 + (wave & 1) * 16;
    if (r0 >= NG || c0 >= ncols) return;
    const R *Ar = Sr + bt.a_off, *Ai = Si + bt.a_off;
    const int64_t xo = bt.x_off * nrhs;
    const R *Br = Xr + xo, *Bi = Xi + xo;
    const int ar_row = r0 + (lane & 15);
    const int bcol = c0 + (lane & 15);
    const int kk = lane >> 4;
    const bool rok = ar_row < NG, cok = bcol < ncols;
    V accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    for (int k0 = 0; k0 < NG; k0 += 4) {
        const int k = k0 + kk;
        const bool kok = k < NG;
        const R ar = (rok && kok) ? Ar[(int64_t)k * NG + ar_row] : R(0);
        const R ai = (rok && kok) ? Ai[(int64_t)k * NG + ar_row] : R(0);
        const R br = (cok && kok) ? Br[(int64_t)bcol * NG + k] : R(0);
        const R bi = (cok && kok) ? Bi[(int64_t)bcol * NG + k] : R(0);
        accr = mfma16(ar, br, accr);
        accr = mfma16(ai, -bi, accr);
        acci = mfma16(ar, bi, acci);
        acci = mfma16(ai, br, acci);
    }
    const int ocol = c0 + (lane & 15);
    if (ocol < ncols) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int orow = r0 + V4<R>::row(lane, v);
            if (orow < NG) {
                Yr[xo + (int64_t)ocol * NG + orow] = accr[v];
                Yi[xo + (int64_t)ocol * NG + orow] = acci[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static size_t dft_smem(Ctx &c, size_t elem) {
    int maxnf = 0;
    for (auto &s : c.shapes) maxnf = std::max(maxnf, s.NF);
    return (size_t)(DFT_GI + 1) * maxnf * elem;
}

void dft_forward(Ctx &c, int prec, int from_vec, const void *vec, int nrhs, int splits) {
    const int64_t total = (int64_t)nrhs * c.N;
    dim3 grid((unsigned)ceil_div(c.max_NG, DFT_GI), nrhs, (unsigned)c.bodies.size());
    if (prec == AXS_FP32) {
        float *Xr = (float *)c.scratch(WS_XR, total * sizeof(float));
        float *Xi = (float *)c.scratch(WS_XI, total * sizeof(float));
        hipLaunchKernelGGL(dft_forward_kernel<float>, grid, dim3(DFT_BS), dft_smem(c, sizeof(float2)),
                           c.stream, c.body_dev, (const float2 *)c.scratch(WS_PART, 0), splits,
                           (const double2 *)vec, from_vec, c.N, nrhs, c.tw32, Xr, Xi);
    } else {
        double *Xr = (double *)c.scratch(WS_XR, total * sizeof(double));
        double *Xi = (double *)c.scratch(WS_XI, total * sizeof(double));
        hipLaunchKernelGGL(dft_forward_kernel<double>, grid, dim3(DFT_BS), dft_smem(c, sizeof(double2)),
                           c.stream, c.body_dev, (const double2 *)c.scratch(WS_PART, 0), splits,
                           (const double2 *)vec, from_vec, c.N, nrhs, c.tw64, Xr, Xi);
    }
    AXS_HIP(hipGetLastError());
}

void modal_gemm(Ctx &c, int prec, int nrhs, bool forward) {
    const int64_t total = (int64_t)nrhs * c.N;
    dim3 grid((unsigned)ceil_div(c.max_NG, 32), (unsigned)ceil_div((int64_t)c.gemm_max_cols * nrhs, 32),
              (unsigned)c.ngemm);
    // all shapes' matrices live in one planar allocation per precision (see precompute)
    const Shape &s0 = c.shapes[0];
    if (forward && prec != AXS_FP64) throw Error{AXS_EINVAL, "the A~_m products exist in FP64 only"};
    if (prec == AXS_FP32) {
        float *Yr = (float *)c.scratch(WS_YR, total * sizeof(float));
        float *Yi = (float *)c.scratch(WS_YI, total * sizeof(float));
        hipLaunchKernelGGL(modal_gemm_kernel<float>, grid, dim3(256), 0, c.stream, c.gemm, nrhs, s0.S32r,
                           s0.S32i, (const float *)c.scratch(WS_XR, 0), (const float *)c.scratch(WS_XI, 0),
                           Yr, Yi);
    } else {
        double *Yr = (double *)c.scratch(WS_YR, total * sizeof(double));
        double *Yi = (double *)c.scratch(WS_YI, total * sizeof(double));
        hipLaunchKernelGGL(modal_gemm_kernel<double>, grid, dim3(256), 0, c.stream, c.gemm, nrhs,
                           forward ? s0.A64r : s0.S64r, forward ? s0.A64i : s0.S64i,
                           (const double *)c.scratch(WS_XR, 0), (const double *)c.scratch(WS_XI, 0), Yr, Yi);
    }
    AXS_HIP(hipGetLastError());
}

void dft_inverse(Ctx &c, int prec, const void *sigma, double alpha, double beta, void *y, int nrhs) {
    dim3 grid((unsigned)ceil_div(c.max_NG, DFT_GI), nrhs, (unsigned)c.bodies.size());
    if (prec == AXS_FP32)
        hipLaunchKernelGGL(dft_inverse_kernel<float>, grid, dim3(DFT_BS), dft_smem(c, sizeof(float2)), c.stream,
                           c.body_dev, (const float *)c.scratch(WS_YR, 0), (const float *)c.scratch(WS_YI, 0),
                           c.N, nrhs, c.tw32, (const double2 *)sigma, alpha, beta, (double2 *)y);
    else
        hipLaunchKernelGGL(dft_inverse_kernel<double>, grid, dim3(DFT_BS), dft_smem(c, sizeof(double2)),
                           c.stream, c.body_dev, (const double *)c.scratch(WS_YR, 0),
                           (const double *)c.scratch(WS_YI, 0), c.N, nrhs, c.tw64, (const double2 *)sigma,
                           alpha, beta, (double2 *)y);
    AXS_HIP(hipGetLastError());
}

}  // namespace axs
