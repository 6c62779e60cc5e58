// Krylov solvers for the left-preconditioned system (Sec. 4, eq. "precond")
//     (I + D^{-1} B) sigma = b,   b = -D^{-1} v.
// GMRES (Saad-Schultz, cited by the paper) with classical Gram-Schmidt applied
// twice; the Arnoldi vectors, the orthogonalisation and the residual are FP64
// on the device; only the (j+1) Hessenberg scalars per right-hand side come to
// the host, where the Givens rotations run.
// Mixed mode: flexible GMRES (the outer Arnoldi process and operator in FP64)
// whose variable right preconditioner is an inner GMRES on the FP32 operator;
// the outer FP64 residual decides convergence, so the answer is FP64-accurate.
// The first inner run keeps its Krylov basis; later inner runs are augmented
// with it (GCRO style, see Recycle) instead of starting from nothing.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <memory>

#include "axs_internal.h"

namespace axs {

using cd = std::complex<double>;
constexpr int KR_BS = 256;

// partial[c][blk][i] = sum_{n in blk} conj(V_i[c][n]) w[c][n]
__global__ __launch_bounds__(KR_BS) void cdot_many_kernel(const double2 *__restrict__ V, int64_t ldv, int nvec,
                                                          const double2 *__restrict__ w, int64_t N,
                                                          double2 *__restrict__ partial) {
    const int c = blockIdx.y, nblk = gridDim.x, blk = blockIdx.x;
    const int64_t chunk = (N + nblk - 1) / nblk;
    const int64_t n0 = (int64_t)blk * chunk, n1 = min(N, n0 + chunk);
    __shared__ double sr[KR_BS / 64], si[KR_BS / 64];
    for (int i = 0; i < nvec; ++i) {
        const double2 *v = V + (int64_t)i * ldv + (int64_t)c * N;
        const double2 *ww = w + (int64_t)c * N;
        double re = 0, im = 0;
        for (int64_t n = n0 + threadIdx.x; n < n1; n += KR_BS) {
            const double2 a = v[n], b = ww[n];
            re += a.x * b.x + a.y * b.y;
            im += a.x * b.y - a.y * b.x;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            re += __shfl_xor(re, o, 64);
            im += __shfl_xor(im, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            sr[threadIdx.x >> 6] = re;
            si[threadIdx.x >> 6] = im;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double tr = 0, ti = 0;
            for (int k = 0; k < KR_BS / 64; ++k) {
                tr += sr[k];
                ti += si[k];
            }
            partial[((int64_t)c * nblk + blk) * nvec + i] = make_double2(tr, ti);
        }
        __syncthreads();
    }
}

__global__ void reduce_dots_kernel(const double2 *__restrict__ partial, int nblk, int nvec, int nrhs,
                                   double2 *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec * nrhs) return;
    const int c = t / nvec, i = t % nvec;
    double re = 0, im = 0;
    for (int b = 0; b < nblk; ++b) {
        const double2 v = partial[((int64_t)c * nblk + b) * nvec + i];
        re += v.x;
        im += v.y;
    }
    out[t] = make_double2(re, im);
}

// w[c][n] += sign * sum_i V_i[c][n] h[c][i]
__global__ void caxpy_many_kernel(const double2 *__restrict__ V, int64_t ldv, int nvec,
                                  const double2 *__restrict__ h, double sign, double2 *__restrict__ w,
                                  int64_t N, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    double re = 0, im = 0;
    for (int i = 0; i < nvec; ++i) {
        const double2 v = V[(int64_t)i * ldv + t], hh = h[c * nvec + i];
        re += v.x * hh.x - v.y * hh.y;
        im += v.x * hh.y + v.y * hh.x;
    }
    double2 o = w[t];
    o.x += sign * re;
    o.y += sign * im;
    w[t] = o;
}

// out[c][n] = in[c][n] * s[c]  (s real)
__global__ void cscale_kernel(const double2 *__restrict__ in, const double *__restrict__ s, double2 *__restrict__ out,
                              int64_t N, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const double f = s[t / N];
    const double2 v = in[t];
    out[t] = make_double2(v.x * f, v.y * f);
}

// out[c][n] += a[c][n] * s[c]  (s real)
__global__ void cadd_scaled_kernel(const double2 *__restrict__ a, const double *__restrict__ s,
                                   double2 *__restrict__ out, int64_t N, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const double f = s[t / N];
    const double2 v = a[t];
    double2 o = out[t];
    o.x += v.x * f;
    o.y += v.y * f;
    out[t] = o;
}

// w[c][n] /= sqrt(nrm[c].x), or 0 where that norm is 0 (the new Arnoldi vector)
__global__ void cnormalize_kernel(double2 *__restrict__ w, const double2 *__restrict__ nrm, int64_t N, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const double n2 = nrm[t / N].x;
    const double f = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    const double2 v = w[t];
    w[t] = make_double2(v.x * f, v.y * f);
}

// out = a - b
__global__ void csub_kernel(const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ out,
                            int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    out[t] = make_double2(a[t].x - b[t].x, a[t].y - b[t].y);
}

// p[c][i] = sum_l M[c][i][l] a[c][l]  (K x K per right-hand side, row-major)
__global__ void cmatvec_small_kernel(const double2 *__restrict__ M, const double2 *__restrict__ a, int K, int nrhs,
                                     double2 *__restrict__ p) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * nrhs) return;
    const int c = t / K, i = t % K;
    const double2 *m = M + ((int64_t)c * K + i) * K;
    const double2 *x = a + (int64_t)c * K;
    double re = 0, im = 0;
    for (int l = 0; l < K; ++l) {
        re += m[l].x * x[l].x - m[l].y * x[l].y;
        im += m[l].x * x[l].y + m[l].y * x[l].x;
    }
    p[t] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
// sqrt of a squared norm from the device: NaN or Inf stay non-finite (so the
// checks below see them), a tiny negative rounding becomes 0
static double norm_from_sq(double s) { return std::isfinite(s) ? std::sqrt(std::max(0.0, s)) : NAN; }

struct Dots {
    Ctx &c;
    int64_t N;
    int nrhs;
    int nblk;
    int cap = 0;                 // vectors per rhs the buffers hold (grown on demand)
    double2 *partial = nullptr, *dev = nullptr;
    std::vector<double2> host;
    Dots(Ctx &c_, int64_t N_, int nrhs_, int maxvec) : c(c_), N(N_), nrhs(nrhs_) {
        nblk = (int)std::min<int64_t>(512, std::max<int64_t>(1, ceil_div(N, 4096)));
        reserve(std::min(maxvec, 16));
    }
    ~Dots() {
        c.dfree(partial);
        c.dfree(dev);
    }
    // room for nvec coefficients per rhs; the old buffers are released in
    // stream order (their last readers were queued on c.stream before)
    void reserve(int nvec) {
        if (nvec <= cap) return;
        const int nc = std::max(nvec, 2 * cap);
        c.dfree(partial);
        c.dfree(dev);
        partial = nullptr;
        dev = nullptr;
        partial = (double2 *)c.dalloc((size_t)nrhs * nblk * nc * sizeof(double2));
        dev = (double2 *)c.dalloc((size_t)nrhs * nc * sizeof(double2));
        cap = nc;
    }
    // out[c][i] = V_i^H w on the device (stream-ordered, no host copy)
    void launch(const double2 *V, int64_t ldv, int nvec, const double2 *w, double2 *out) {
        reserve(nvec);
        hipLaunchKernelGGL(cdot_many_kernel, dim3(nblk, nrhs), dim3(KR_BS), 0, c.stream, V, ldv, nvec, w, N,
                           partial);
        AXS_HIP(hipGetLastError());
        hipLaunchKernelGGL(reduce_dots_kernel, dim3(ceil_div(nvec * nrhs, 128)), dim3(128), 0, c.stream, partial,
                           nblk, nvec, nrhs, out);
        AXS_HIP(hipGetLastError());
    }
    // h[c][i] = V_i^H w (device + host copies)
    void run(const double2 *V, int64_t ldv, int nvec, const double2 *w) {
        reserve(nvec);
        launch(V, ldv, nvec, w, dev);
        host.resize((size_t)nrhs * nvec);
        AXS_HIP(hipMemcpyAsync(host.data(), dev, (size_t)nvec * nrhs * sizeof(double2), hipMemcpyDeviceToHost,
                               c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
    }
    cd get(int c_, int i, int nvec) const { return cd(host[c_ * nvec + i].x, host[c_ * nvec + i].y); }
};

static void axpy_many(Ctx &c, const double2 *V, int64_t ldv, int nvec, const std::vector<cd> &h, int nrhs,
                      double sign, double2 *w, int64_t N, double2 *hdev) {
    std::vector<double2> hh(h.size());
    for (size_t k = 0; k < h.size(); ++k) hh[k] = make_double2(h[k].real(), h[k].imag());
    AXS_HIP(hipMemcpyAsync(hdev, hh.data(), hh.size() * sizeof(double2), hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(caxpy_many_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, V, ldv, nvec,
                       hdev, sign, w, N, nrhs);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));   // hh is pageable host memory
}

static void scale(Ctx &c, const double2 *in, const std::vector<double> &s, double2 *out, int64_t N, int nrhs,
                  double *sdev) {
    AXS_HIP(hipMemcpyAsync(sdev, s.data(), s.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(cscale_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, in, sdev, out, N,
                       nrhs);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));
}

// AXS_VERBOSE=1 in the environment prints one line per outer iteration to stderr
static int verbose_level() {
    static const int v = [] {
        const char *e = std::getenv("AXS_VERBOSE");
        return e ? std::atoi(e) : 0;
    }();
    return v;
}

// Arnoldi/GMRES state for nrhs independent systems sharing the operator.  The
// Hessenberg columns and rotations grow one step at a time, so host memory
// follows the iterations taken, not the iteration limit.
struct Gmres {
    int nrhs, maxit;
    std::vector<std::vector<std::vector<cd>>> H;   // per rhs, per column j: rows 0..j+1
    std::vector<std::vector<cd>> cs, sn, g;
    std::vector<int> done_at;              // iteration count at convergence (-1 = running)
    std::vector<double> bnorm;
    Gmres(int nrhs_, int maxit_) : nrhs(nrhs_), maxit(maxit_) {
        H.assign(nrhs, {});
        cs.assign(nrhs, {});
        sn.assign(nrhs, {});
        g.assign(nrhs, std::vector<cd>(1, 0.0));
        done_at.assign(nrhs, -1);
        bnorm.assign(nrhs, 1.0);
    }
    // start column j (zero) for every rhs
    void open_column(int j) {
        for (int c = 0; c < nrhs; ++c) {
            H[c].emplace_back((size_t)j + 2, cd(0.0));
            cs[c].push_back(0.0);
            sn[c].push_back(0.0);
            g[c].push_back(0.0);
        }
    }
    cd &h(int c, int i, int j) { return H[c][j][i]; }
    // apply previous rotations to column j, build the new one; returns |g_{j+1}|
    double rotate(int c, int j) {
        for (int i = 0; i < j; ++i) {
            cd t = cs[c][i] * h(c, i, j) + sn[c][i] * h(c, i + 1, j);
            h(c, i + 1, j) = -std::conj(sn[c][i]) * h(c, i, j) + cs[c][i] * h(c, i + 1, j);
            h(c, i, j) = t;
        }
        cd a = h(c, j, j), b = h(c, j + 1, j);
        double den = std::hypot(std::abs(a), std::abs(b));
        if (den == 0.0) {
            cs[c][j] = 1.0;
            sn[c][j] = 0.0;
        } else if (std::abs(a) == 0.0) {
            cs[c][j] = 0.0;
            sn[c][j] = std::conj(b) / std::abs(b);
        } else {
            cs[c][j] = std::abs(a) / den;
            sn[c][j] = (a / std::abs(a)) * std::conj(b) / den;
        }
        h(c, j, j) = cs[c][j] * a + sn[c][j] * b;
        h(c, j + 1, j) = 0.0;
        g[c][j + 1] = -std::conj(sn[c][j]) * g[c][j];
        g[c][j] = cs[c][j] * g[c][j];
        return std::abs(g[c][j + 1]);
    }
    // y = H(0:k,0:k)^{-1} g(0:k)
    std::vector<cd> lsq(int c, int k) {
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd s = g[c][i];
            for (int j = i + 1; j < k; ++j) s -= h(c, i, j) * y[j];
            y[i] = s / h(c, i, i);
        }
        return y;
    }
};

// A Krylov basis: up to `maxvec` vectors of `vb` bytes in one allocation that
// grows on demand (to at least 16 vectors, doubling), so that the memory of a
// solve follows the iterations it takes rather than its iteration limit.  The
// base pointer changes when the basis grows.
struct Basis {
    Ctx &c;
    size_t vb;
    int maxvec, cap = 0;
    double2 *p = nullptr;
    Basis(Ctx &c_, size_t vb_, int maxvec_) : c(c_), vb(vb_), maxvec(maxvec_) {}
    Basis(const Basis &) = delete;
    Basis &operator=(const Basis &) = delete;
    ~Basis() { c.dfree(p); }
    double2 *vec(int i) const { return p + (size_t)i * (vb / sizeof(double2)); }
    // room for n vectors; the first `keep` are carried over
    void reserve(int n, int keep) {
        if (n <= cap) return;
        AXS_REQUIRE(n <= maxvec, AXS_EINVAL, "Krylov basis beyond its iteration limit");
        const int nc = std::min(maxvec, std::max(n, std::max(16, 2 * cap)));
        double2 *q = (double2 *)c.dalloc((size_t)nc * vb);
        if (keep > 0) {
            AXS_HIP(hipMemcpyAsync(q, p, (size_t)keep * vb, hipMemcpyDeviceToDevice, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));   // the old block is released after the copy
        }
        c.dfree(p);
        p = q;
        cap = nc;
    }
};

// The Krylov relation A V_k = V_{k+1} Hbar of an earlier GMRES run on the same
// operator (per rhs, Hbar (k+1) x k), kept so that a later run on a new right-
// hand side minimises its residual over span(U) plus its own Krylov space
// (GCRO-style augmentation): with the thin QR Hbar = Q R, C = V_{k+1} Q is
// orthonormal and A U = C for U = V_k R^{-1}.  The later run orthogonalises
// its start vector and every new Arnoldi vector against C as well, which
// records B = C^H A V_j next to its own Hessenberg matrix, and takes
//   x = U (C^H r0 - B y) + V_j y
// with y from its own least-squares problem (Sec. 4 solves the system with
// GMRES; restarting an inner solve otherwise discards the space it built).
struct Recycle {
    const double2 *V = nullptr;               // the earlier basis, k + 1 vectors of nrhs * N
    int k = 0;
    std::vector<char> on;                     // per rhs: relation usable (no breakdown)
    std::vector<std::vector<cd>> Q, R;        // per rhs: Q (k+1) x k and R k x k, column-major
    double2 *M = nullptr;                     // device [nrhs][k+1][k+1]: Q Q^H, row-major
    Ctx *ctx = nullptr;                       // owner of M
    Recycle() = default;
    Recycle(const Recycle &) = delete;
    Recycle &operator=(const Recycle &) = delete;
    ~Recycle() {
        if (ctx) ctx->dfree(M);
    }
};

// Arnoldi record of a run, for building a Recycle: the unrotated Hessenberg
// columns per rhs ((maxit+1) x maxit column-major) and whether any step broke
// down (a zero new vector) for that rhs.
struct ArnoldiRecord {
    std::vector<std::vector<std::vector<cd>>> H;   // per rhs, per column j: rows 0..j+1
    std::vector<char> breakdown;
    int steps = 0;
};

// Run GMRES for nrhs systems: op(x, y) computes y = A x.  V grows to at most
// (maxit+1) vectors of nrhs*N.  Optional flexible mode: prec(v, z) gives
// z_j ~ A^{-1} v_j stored in Z (at most maxit vectors), and the solution update
// uses Z.  On entry r0 holds the initial residual. On exit x += (V or Z) y
// (+ the U part with rc).  rc (may be null): augment with an earlier run's
// Krylov relation; rec (may be null): record this run's.  Returns the
// iteration counts per rhs.
template <class Op, class Prec>
static std::vector<int> gmres_core(Ctx &c, int64_t N, int nrhs, int maxit, double tol, const double2 *r0,
                                   double2 *x, Basis &V, Basis *Z, const std::vector<double> &bnorm, Op op,
                                   Prec prec, bool flexible, std::vector<double> &rel_est,
                                   const Recycle *rc = nullptr, ArnoldiRecord *rec = nullptr) {
    const int64_t ldv = N * nrhs;
    Gmres G(nrhs, maxit);
    G.bnorm = bnorm;
    Dots D(c, N, nrhs, maxit + 1);
    double *sdev = (double *)c.dalloc(nrhs * sizeof(double));
    // per Arnoldi step: both Gram-Schmidt passes' coefficients [nrhs][j+1] and
    // the squared norm of the new vector [nrhs], read back in one copy; the
    // device buffer grows with the step (doubling), like the host copy
    double2 *cdev = nullptr;
    int64_t cdev_cap = 0;
    std::vector<double2> chost;
    if (rec) {
        rec->H.assign(nrhs, {});
        rec->breakdown.assign(nrhs, 0);
        rec->steps = 0;
    }
    // augmentation: coefficients against the earlier basis, two passes [2][nrhs][K]
    const int K = rc ? rc->k + 1 : 0;
    std::unique_ptr<Dots> DR;
    double2 *adev = nullptr, *pdev = nullptr;
    std::vector<double2> ahost;
    std::vector<std::vector<cd>> Bm;   // per rhs: B = C^H A V_j, k x maxit column-major
    std::vector<std::vector<cd>> cr0;  // per rhs: C^H r0
    auto project_out = [&](double2 *w, double2 *acoef) {
        // w -= C C^H w = V_rc (Q Q^H) (V_rc^H w); acoef receives V_rc^H w
        DR->launch(rc->V, ldv, K, w, acoef);
        hipLaunchKernelGGL(cmatvec_small_kernel, dim3(ceil_div(K * nrhs, 128)), dim3(128), 0, c.stream, rc->M,
                           acoef, K, nrhs, pdev);
        AXS_HIP(hipGetLastError());
        hipLaunchKernelGGL(caxpy_many_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, rc->V, ldv, K,
                           pdev, -1.0, w, N, nrhs);
        AXS_HIP(hipGetLastError());
    };
    // C^H w from the two passes' V_rc^H w
    auto qh = [&](int cc, const double2 *a0, const double2 *a1) {
        std::vector<cd> out(rc->k, 0.0);
        if (!rc->on[cc]) return out;
        for (int i = 0; i < rc->k; ++i) {
            cd sacc = 0.0;
            for (int l = 0; l < K; ++l) {
                const cd a(a0[(size_t)cc * K + l].x + a1[(size_t)cc * K + l].x,
                           a0[(size_t)cc * K + l].y + a1[(size_t)cc * K + l].y);
                sacc += std::conj(rc->Q[cc][(size_t)i * K + l]) * a;
            }
            out[i] = sacc;
        }
        return out;
    };
    const double2 *start = r0;
    if (rc) {
        DR.reset(new Dots(c, N, nrhs, K));
        adev = (double2 *)c.dalloc((size_t)2 * nrhs * K * sizeof(double2));
        pdev = (double2 *)c.dalloc((size_t)nrhs * K * sizeof(double2));
        ahost.resize((size_t)2 * nrhs * K);
        Bm.assign(nrhs, std::vector<cd>((size_t)rc->k * maxit, 0.0));
        // start vector: r0 less its component in range(C), twice
        V.reserve(2, 0);
        AXS_HIP(hipMemcpyAsync(V.vec(0), r0, (size_t)ldv * sizeof(double2), hipMemcpyDeviceToDevice, c.stream));
        for (int pass = 0; pass < 2; ++pass) project_out(V.vec(0), adev + (size_t)pass * nrhs * K);
        AXS_HIP(hipMemcpyAsync(ahost.data(), adev, ahost.size() * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        cr0.resize(nrhs);
        for (int cc = 0; cc < nrhs; ++cc) cr0[cc] = qh(cc, ahost.data(), ahost.data() + (size_t)nrhs * K);
        start = V.vec(0);
    }
    auto release = [&]() {
        c.dfree(sdev);
        c.dfree(cdev);
        c.dfree(adev);
        c.dfree(pdev);
    };
    // beta = ||r0|| (of the projected start vector with rc)
    D.run(start, ldv, 1, start);
    std::vector<double> beta(nrhs), inv(nrhs);
    rel_est.assign(nrhs, 0.0);
    bool all_done = true;
    for (int cc = 0; cc < nrhs; ++cc) {
        beta[cc] = norm_from_sq(D.get(cc, 0, 1).real());
        AXS_REQUIRE(std::isfinite(beta[cc]), AXS_ENONFINITE, "non-finite residual");
        G.g[cc][0] = beta[cc];
        inv[cc] = beta[cc] > 0 ? 1.0 / beta[cc] : 0.0;
        rel_est[cc] = beta[cc] / bnorm[cc];
        if (rel_est[cc] <= tol) G.done_at[cc] = 0;
        else all_done = false;
    }
    std::vector<int> iters(nrhs, 0);
    int j = 0;
    if (!all_done) {
        V.reserve(2, 0);
        scale(c, start, inv, V.vec(0), N, nrhs, sdev);
        for (; j < maxit; ++j) {
            V.reserve(j + 2, j + 1);
            double2 *vj = V.vec(j);
            double2 *w = V.vec(j + 1);
            if (flexible) {
                Z->reserve(j + 1, j);
                double2 *zj = Z->vec(j);
                prec(vj, zj);
                op(zj, w);
            } else {
                op(vj, w);
            }
            // classical Gram-Schmidt, twice (against range(C) first with rc), then
            // the norm and the normalisation of the new vector, all stream-ordered
            // on the device; the coefficients come to the host in one copy, the
            // only synchronisation of the step
            const int nv = j + 1;
            const int64_t nh = (int64_t)nrhs * nv;
            if (2 * nh + nrhs > cdev_cap) {
                const int64_t cap = std::max<int64_t>(2 * nh + nrhs, 2 * cdev_cap);
                c.dfree(cdev);
                cdev = nullptr;
                cdev = (double2 *)c.dalloc((size_t)cap * sizeof(double2));
                cdev_cap = cap;
            }
            chost.resize((size_t)(2 * nh + nrhs));
            G.open_column(j);
            for (int pass = 0; pass < 2; ++pass) {
                if (rc) project_out(w, adev + (size_t)pass * nrhs * K);
                double2 *hc = cdev + pass * nh;
                D.launch(V.p, ldv, nv, w, hc);
                hipLaunchKernelGGL(caxpy_many_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, V.p,
                                   ldv, nv, hc, -1.0, w, N, nrhs);
                AXS_HIP(hipGetLastError());
            }
            D.launch(w, ldv, 1, w, cdev + 2 * nh);
            hipLaunchKernelGGL(cnormalize_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, w,
                               cdev + 2 * nh, N, nrhs);
            AXS_HIP(hipGetLastError());
            AXS_HIP(hipMemcpyAsync(chost.data(), cdev, (size_t)(2 * nh + nrhs) * sizeof(double2),
                                   hipMemcpyDeviceToHost, c.stream));
            if (rc)
                AXS_HIP(hipMemcpyAsync(ahost.data(), adev, ahost.size() * sizeof(double2), hipMemcpyDeviceToHost,
                                       c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
            all_done = true;
            for (int cc = 0; cc < nrhs; ++cc) {
                const double hn = norm_from_sq(chost[2 * nh + cc].x);
                AXS_REQUIRE(std::isfinite(hn), AXS_ENONFINITE, "non-finite Arnoldi vector");
                for (int i = 0; i < nv; ++i) {
                    const double2 a = chost[(size_t)cc * nv + i], b = chost[nh + (size_t)cc * nv + i];
                    G.h(cc, i, j) = cd(a.x + b.x, a.y + b.y);
                }
                G.h(cc, j + 1, j) = hn;
                if (rec) {
                    rec->H[cc].emplace_back((size_t)nv + 1, cd(0.0));
                    for (int i = 0; i <= nv; ++i) rec->H[cc][j][i] = G.h(cc, i, j);
                    if (hn == 0.0) rec->breakdown[cc] = 1;
                }
                if (rc) {
                    const std::vector<cd> bcol = qh(cc, ahost.data(), ahost.data() + (size_t)nrhs * K);
                    for (int i = 0; i < rc->k; ++i) Bm[cc][(size_t)j * rc->k + i] = bcol[i];
                }
                if (G.done_at[cc] < 0) {
                    const double res = G.rotate(cc, j);
                    rel_est[cc] = res / bnorm[cc];
                    if (rel_est[cc] <= tol || hn == 0.0) G.done_at[cc] = j + 1;
                }
                if (G.done_at[cc] < 0) all_done = false;
            }
            if (verbose_level() > 0) {
                double worst = 0;
                for (int cc = 0; cc < nrhs; ++cc) worst = std::max(worst, rel_est[cc]);
                std::fprintf(stderr, "[axs] %s iteration %d: max relative residual %.3e\n",
                             flexible ? "outer" : "gmres", j + 1, worst);
            }
            if (all_done) {
                ++j;
                break;
            }
        }
    }
    if (rec) rec->steps = j;
    // x += basis * y, per rhs with its own k
    const double2 *basis = flexible ? Z->p : V.p;
    int kmax = 0;
    for (int cc = 0; cc < nrhs; ++cc) {
        iters[cc] = G.done_at[cc] < 0 ? j : G.done_at[cc];
        kmax = std::max(kmax, iters[cc]);
    }
    std::vector<std::vector<cd>> ys(nrhs);
    for (int cc = 0; cc < nrhs; ++cc)
        if (iters[cc] > 0) ys[cc] = G.lsq(cc, iters[cc]);
    if (kmax > 0) {
        std::vector<cd> y((size_t)nrhs * kmax, 0.0);
        for (int cc = 0; cc < nrhs; ++cc)
            for (int i = 0; i < iters[cc]; ++i) y[(size_t)cc * kmax + i] = ys[cc][i];
        double2 *ydev = (double2 *)c.dalloc(y.size() * sizeof(double2));
        axpy_many(c, basis, ldv, kmax, y, nrhs, 1.0, x, N, ydev);
        c.dfree(ydev);
    }
    if (rc) {
        // x += U (C^H r0 - B y) = V_k R^{-1} (C^H r0 - B y)
        const int k = rc->k;
        std::vector<cd> d((size_t)nrhs * k, 0.0);
        for (int cc = 0; cc < nrhs; ++cc) {
            if (!rc->on[cc]) continue;
            std::vector<cd> sv = cr0[cc];
            for (int jj = 0; jj < iters[cc]; ++jj)
                for (int i = 0; i < k; ++i) sv[i] -= Bm[cc][(size_t)jj * k + i] * ys[cc][jj];
            const std::vector<cd> &R = rc->R[cc];
            for (int i = k - 1; i >= 0; --i) {
                cd acc = sv[i];
                for (int l = i + 1; l < k; ++l) acc -= R[(size_t)l * k + i] * d[(size_t)cc * k + l];
                d[(size_t)cc * k + i] = acc / R[(size_t)i * k + i];
            }
        }
        double2 *ddev = (double2 *)c.dalloc(d.size() * sizeof(double2));
        axpy_many(c, rc->V, ldv, k, d, nrhs, 1.0, x, N, ddev);
        c.dfree(ddev);
    }
    release();
    return iters;
}

// Build the augmentation of later runs from the record of a run whose basis is
// V (rec.steps + 1 vectors): thin QR of each rhs's Hbar by classical
// Gram-Schmidt, twice; a rhs whose run broke down is left out.
static void build_recycle(Ctx &c, const ArnoldiRecord &rec, int maxit, const double2 *V, int nrhs, Recycle &rc) {
    const int k = rec.steps, K = k + 1;
    rc.V = V;
    rc.k = k;
    rc.on.assign(nrhs, 0);
    rc.Q.assign(nrhs, std::vector<cd>((size_t)K * k, 0.0));
    rc.R.assign(nrhs, std::vector<cd>((size_t)k * k, 0.0));
    std::vector<double2> M((size_t)nrhs * K * K, make_double2(0.0, 0.0));
    for (int cc = 0; cc < nrhs; ++cc) {
        if (rec.breakdown[cc] || k == 0) continue;
        std::vector<cd> &Q = rc.Q[cc], &R = rc.R[cc];
        bool ok = true;
        for (int jj = 0; jj < k && ok; ++jj) {
            std::vector<cd> q(K);
            for (int i = 0; i < K; ++i) q[i] = i < (int)rec.H[cc][jj].size() ? rec.H[cc][jj][i] : cd(0.0);
            for (int pass = 0; pass < 2; ++pass)
                for (int l = 0; l < jj; ++l) {
                    cd r = 0.0;
                    for (int i = 0; i < K; ++i) r += std::conj(Q[(size_t)l * K + i]) * q[i];
                    R[(size_t)jj * k + l] += r;
                    for (int i = 0; i < K; ++i) q[i] -= r * Q[(size_t)l * K + i];
                }
            double nq = 0.0;
            for (int i = 0; i < K; ++i) nq += std::norm(q[i]);
            nq = std::sqrt(nq);
            if (!(nq > 0.0) || !std::isfinite(nq)) ok = false;
            R[(size_t)jj * k + jj] = nq;
            for (int i = 0; i < K && ok; ++i) Q[(size_t)jj * K + i] = q[i] / nq;
        }
        if (!ok) continue;
        rc.on[cc] = 1;
        for (int i = 0; i < K; ++i)
            for (int l = 0; l < K; ++l) {
                cd sacc = 0.0;
                for (int jj = 0; jj < k; ++jj) sacc += Q[(size_t)jj * K + i] * std::conj(Q[(size_t)jj * K + l]);
                M[((size_t)cc * K + i) * K + l] = make_double2(sacc.real(), sacc.imag());
            }
    }
    rc.ctx = &c;
    rc.M = (double2 *)c.dalloc(M.size() * sizeof(double2));
    AXS_HIP(hipMemcpyAsync(rc.M, M.data(), M.size() * sizeof(double2), hipMemcpyHostToDevice, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));   // M is pageable host memory
}

static std::vector<double> norms(Ctx &c, const double2 *v, int64_t N, int nrhs) {
    Dots D(c, N, nrhs, 1);
    D.run(v, N * nrhs, 1, v);
    std::vector<double> out(nrhs);
    for (int cc = 0; cc < nrhs; ++cc) out[cc] = norm_from_sq(D.get(cc, 0, 1).real());
    return out;
}

axs_status solve_impl(Ctx &c, const void *incident, const void *sigma0, void *sigma_out, int nrhs, int mode,
                      double tol, int max_iters, axs_solve_info *info, const void *b_given) {
    const auto t0 = std::chrono::steady_clock::now();
    const bool certify = (mode & AXS_SOLVE_CERTIFY) != 0;
    const bool unprec = (mode & AXS_SOLVE_UNPRECONDITIONED) != 0;
    const bool restart_inner = (mode & AXS_SOLVE_RESTART_INNER) != 0;
    mode &= ~(AXS_SOLVE_CERTIFY | AXS_SOLVE_UNPRECONDITIONED | AXS_SOLVE_RESTART_INNER);
    // the operator of the solve: I + D^{-1} B (FP64), or D + B without the preconditioner
    auto op64 = [&](const double2 *in, double2 *out) {
        if (unprec) apply_unpreconditioned(c, in, out, nrhs);
        else apply_operator(c, in, out, nrhs, AXS_FP64);
    };
    const int64_t N = c.N, tot = N * nrhs;
    const size_t vb = (size_t)tot * sizeof(double2);
    double2 *x = (double2 *)sigma_out;
    double2 *b = (double2 *)c.dalloc(vb);
    double2 *r = (double2 *)c.dalloc(vb);
    double2 *tmp = (double2 *)c.dalloc(vb);
    // b = -D^{-1} v, or -v without the preconditioner, or given
    if (b_given) {
        AXS_HIP(hipMemcpyAsync(b, b_given, vb, hipMemcpyDeviceToDevice, c.stream));
    } else if (unprec) {
        AXS_HIP(hipMemsetAsync(tmp, 0, vb, c.stream));
        hipLaunchKernelGGL(csub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, tmp,
                           (const double2 *)incident, b, tot);
        AXS_HIP(hipGetLastError());
    } else {
        apply_precond(c, incident, b, nrhs, AXS_FP64, -1.0);
    }
    std::vector<double> bn = norms(c, b, N, nrhs);
    for (double v : bn) AXS_REQUIRE(std::isfinite(v), AXS_ENONFINITE, "non-finite incident field");
    for (auto &v : bn)
        if (v == 0.0) v = 1.0;
    // initial guess.  FP64 GMRES: sigma0 is the starting point if its FP64
    // residual is below ||b||, else zero (one FP64 application).  Mixed: the
    // guess enters the first application of the flexible preconditioner
    // instead, z_1 = (g + inner(b - A32 g)) / ||b||, which costs one FP32
    // application; it is kept where its FP32 residual is below ||b||, and
    // the FP64 outer residual certifies the result either way.
    std::vector<int> warm(nrhs, 0);
    const bool mixed_guess = sigma0 && mode == AXS_SOLVE_MIXED;
    double2 *g = nullptr, *w0 = nullptr;   // mixed: the kept guess and b - A32 g
    AXS_HIP(hipMemsetAsync(x, 0, vb, c.stream));
    AXS_HIP(hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, c.stream));
    if (sigma0 && !mixed_guess) {
        op64((const double2 *)sigma0, tmp);
        hipLaunchKernelGGL(csub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, b, tmp, tmp, tot);
        AXS_HIP(hipGetLastError());
        std::vector<double> rn = norms(c, tmp, N, nrhs);
        for (int cc = 0; cc < nrhs; ++cc) {
            if (std::isfinite(rn[cc]) && rn[cc] < bn[cc]) {
                warm[cc] = 1;
                AXS_HIP(hipMemcpyAsync(x + cc * N, (const double2 *)sigma0 + cc * N, N * sizeof(double2),
                                       hipMemcpyDeviceToDevice, c.stream));
                AXS_HIP(hipMemcpyAsync(r + cc * N, tmp + cc * N, N * sizeof(double2), hipMemcpyDeviceToDevice,
                                       c.stream));
            }
        }
    }
    if (mixed_guess) {
        g = (double2 *)c.dalloc(vb);
        w0 = (double2 *)c.dalloc(vb);
        AXS_HIP(hipMemcpyAsync(g, sigma0, vb, hipMemcpyDeviceToDevice, c.stream));
        apply_operator(c, g, tmp, nrhs, AXS_FP32);
        hipLaunchKernelGGL(csub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, b, tmp, w0, tot);
        AXS_HIP(hipGetLastError());
        std::vector<double> rn = norms(c, w0, N, nrhs);
        for (int cc = 0; cc < nrhs; ++cc) {
            if (std::isfinite(rn[cc]) && rn[cc] < bn[cc]) {
                warm[cc] = 1;
            } else {   // dropped: the first preconditioner application is the plain one
                AXS_HIP(hipMemsetAsync(g + cc * N, 0, N * sizeof(double2), c.stream));
                AXS_HIP(hipMemcpyAsync(w0 + cc * N, b + cc * N, N * sizeof(double2), hipMemcpyDeviceToDevice,
                                       c.stream));
            }
        }
    }
    std::vector<double> est;
    std::vector<int> outer;
    std::vector<int> inner_total(nrhs, 0);
    Basis V(c, vb, max_iters + 1);
    if (mode == AXS_SOLVE_FP64) {
        auto none = [&](const double2 *, double2 *) {};
        outer = gmres_core(c, N, nrhs, max_iters, tol, r, x, V, nullptr, bn, op64, none, false, est);
    } else {
        const int max_inner = 60;
        // Vr keeps the first inner run's Krylov basis: every later inner run is
        // augmented with that run's relation (Recycle) instead of starting over
        Basis Z(c, vb, max_iters), Vi(c, vb, max_inner + 1), Vr(c, vb, max_inner + 1);
        Recycle rc;
        bool have_rc = false;
        bool first_prec = true;
        std::vector<double> invb(nrhs);
        for (int cc = 0; cc < nrhs; ++cc) invb[cc] = 1.0 / bn[cc];
        double *sdev = (double *)c.dalloc(nrhs * sizeof(double));   // 1 / ||b|| per rhs
        AXS_HIP(hipMemcpyAsync(sdev, invb.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));   // invb is pageable host memory
        auto prec = [&](const double2 *v_in, double2 *z) {
            // with a kept guess the first application solves for the guess's
            // correction: v_1 = b / ||b||, so v_1 - A32 g / ||b|| = w0 / ||b||
            const double2 *v = v_in;
            const bool with_guess = mixed_guess && first_prec;
            first_prec = false;
            if (with_guess) {
                hipLaunchKernelGGL(cscale_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, w0, sdev,
                                   tmp, N, nrhs);
                AXS_HIP(hipGetLastError());
                v = tmp;
            }
            // inner GMRES on the FP32 operator, zero initial guess, rhs v; it only
            // has to reduce the outer residual by the factor still missing, with
            // a margin of 0.6 (the first run stops at 1e-5, about the FP32
            // operator's own accuracy)
            double worst = 0.0;
            for (double e : est) worst = std::max(worst, e);
            const double tin = std::min(1e-2, std::max(1e-5, 0.6 * tol / std::max(worst, 1e-300)));
            AXS_HIP(hipMemsetAsync(z, 0, vb, c.stream));
            std::vector<double> vn = norms(c, v, N, nrhs);
            for (auto &q : vn)
                if (q == 0.0) q = 1.0;
            // with the guess the inner tolerance is measured against ||v_1|| = 1,
            // not against the guess's smaller residual: a better guess then
            // shortens this run instead of demanding the same relative reduction
            if (with_guess) vn.assign(nrhs, 1.0);
            auto op32 = [&](const double2 *in, double2 *out) { apply_operator(c, in, out, nrhs, AXS_FP32); };
            auto none = [&](const double2 *, double2 *) {};
            std::vector<double> ie;
            std::vector<int> it;
            if (restart_inner) {
                it = gmres_core(c, N, nrhs, max_inner, tin, v, z, Vi, nullptr, vn, op32, none, false, ie);
            } else if (!have_rc) {
                ArnoldiRecord rec;
                it = gmres_core(c, N, nrhs, max_inner, tin, v, z, Vr, nullptr, vn, op32, none, false, ie, nullptr,
                                &rec);
                if (rec.steps > 0) {
                    build_recycle(c, rec, max_inner, Vr.p, nrhs, rc);
                    have_rc = true;
                }
            } else {
                it = gmres_core(c, N, nrhs, max_inner, tin, v, z, Vi, nullptr, vn, op32, none, false, ie, &rc);
            }
            for (int cc = 0; cc < nrhs; ++cc) inner_total[cc] += it[cc];
            if (with_guess) {   // z += g / ||b||
                hipLaunchKernelGGL(cadd_scaled_kernel, dim3(ceil_div(N * nrhs, 256)), dim3(256), 0, c.stream, g,
                                   sdev, z, N, nrhs);
                AXS_HIP(hipGetLastError());
            }
        };
        outer = gmres_core(c, N, nrhs, max_iters, tol, r, x, V, &Z, bn, op64, prec, true, est);
        c.dfree(sdev);
    }
    std::vector<double> relv = est;
    if (certify) {
        // explicit FP64 residual of the returned solution
        op64(x, tmp);
        hipLaunchKernelGGL(csub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, b, tmp, tmp, tot);
        AXS_HIP(hipGetLastError());
        std::vector<double> rn = norms(c, tmp, N, nrhs);
        for (int cc = 0; cc < nrhs; ++cc) relv[cc] = rn[cc] / bn[cc];
    } else {
        AXS_HIP(hipStreamSynchronize(c.stream));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all_ok = true;
    for (int cc = 0; cc < nrhs; ++cc) {
        AXS_REQUIRE(std::isfinite(relv[cc]), AXS_ENONFINITE, "non-finite final residual");
        const double rel = relv[cc];
        if (info) {
            info[cc].iterations = outer[cc];
            info[cc].inner_iterations = inner_total[cc];
            info[cc].rel_residual = rel;
            info[cc].seconds = secs;
            info[cc].used_warm_start = warm[cc];
            info[cc].converged = rel <= tol ? 1 : 0;
        }
        if (!(rel <= tol)) all_ok = false;
    }
    c.dfree(b);
    c.dfree(r);
    c.dfree(tmp);
    c.dfree(g);
    c.dfree(w0);
    return all_ok ? AXS_OK : AXS_NOT_CONVERGED;
}

}  // namespace axs
