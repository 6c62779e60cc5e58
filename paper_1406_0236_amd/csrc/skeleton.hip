// Skeletonization of the inter-body blocks (Sec. 5, eqs. ip0-ip6).
//
// Sec. 5 factors each off-diagonal block A_pq = U_p A~_pq V_q^* + R_pq with
// interpolative decompositions whose index sets make A~_pq = A_pq(I_p, I_q) a
// submatrix of B, then solves the smaller preconditioned system
//     s~ + S B~ s~ = -v~,   S_p = V_p^* A_pp^{-1} U_p,   v~_p = V_p^* A_pp^{-1} v_p,
// and lifts the result back with s_p = -A_pp^{-1} (v_p + U_p sum_q A~_pq s~_q).
//
// Two versions.  Point skeletons (single nodes from a randomized ID, as the
// paper prints it) are in the second half of this file.  Ring skeletons keep
// whole rings (contour nodes with all their azimuthal nodes): U_p = X (x) I
// and V_p^* = X^T (x) I with one NG x k matrix X per shape acting on the
// contour index.  Then
//   - B~ is the inter-body sum over the skeleton rings: the ring-order kernels
//     run on it unchanged;
//   - S_p is block diagonal in the Fourier modes, S~_m = X^T S_m X (k x k):
//     the DFT / per-mode MFMA GEMM / inverse DFT pipeline runs on it unchanged;
//   - the ID is over at most a few hundred contour nodes, a small pivoted
//     Gram-Schmidt on the GPU instead of a pivoted QR of a 10^4-row matrix.
// X is the row ID over the contour index of H = [IN_m | OUT_m^T]_(m = 0..M):
// IN_m, the field at the contour nodes of combined-field sources on a proxy
// sphere of radius R_p (every field the body can receive from outside it),
// OUT_m, the field of the body's nodes at proxy spheres of radii R_p and
// 1.25 R_p (every field it sends out).  A ring set that interpolates every
// mode interpolates every azimuthal node.  The compressed system lives in a
// child context built from the skeleton rings with S~_m in place of S_m.
#include "axs_internal.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <numeric>

namespace axs {

// H (row-major NG x C, C = (M+1)(n_in + n_o)): row i, column block m holds
// IN[i, :, m] * s_in then OUT[:, i, m] * s_out
__global__ void build_h_kernel(const double2 *__restrict__ kin, const double2 *__restrict__ kout, int NG,
                               int n_in, int n_o, int M, double s_in, double s_out, double2 *__restrict__ H) {
    const int64_t C = (int64_t)(M + 1) * (n_in + n_o);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * C) return;
    const int i = (int)(t / C);
    const int64_t col = t % C;
    const int m = (int)(col / (n_in + n_o)), j = (int)(col % (n_in + n_o));
    double2 v;
    double s;
    if (j < n_in) {
        v = kin[((int64_t)i * n_in + j) * (M + 1) + m];
        s = s_in;
    } else {
        v = kout[((int64_t)(j - n_in) * NG + i) * (M + 1) + m];
        s = s_out;
    }
    H[t] = make_double2(v.x * s, v.y * s);
}

// per-block partial sums of |a|^2, then one block adds the partials in order
__global__ void sumsq_partial_kernel(const double2 *__restrict__ a, int64_t n, double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256)
        acc = fma(a[t].x, a[t].x, fma(a[t].y, a[t].y, acc));
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// squared norms of the active rows (-1 for inactive ones); one block per row
__global__ void row_norms_kernel(const double2 *__restrict__ H, int64_t C, const int *__restrict__ active,
                                 double *__restrict__ nrm) {
    __shared__ double sh[256];
    const int i = blockIdx.x;
    if (!active[i]) {
        if (threadIdx.x == 0) nrm[i] = -1.0;
        return;
    }
    const double2 *h = H + (int64_t)i * C;
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < C; c += 256) acc = fma(h[c].x, h[c].x, fma(h[c].y, h[c].y, acc));
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) nrm[i] = sh[0];
}

// c_i = <h_i, u> = sum_c h_i[c] conj(u[c]) for the active rows, u = row p; the
// R entry of step s gains conj(c_i) / nu (H^* columns a_i = conj(h_i))
__global__ void row_dots_kernel(const double2 *__restrict__ H, int64_t C, int p, const int *__restrict__ active,
                                double nu, double2 *__restrict__ coef, double2 *__restrict__ Rrow) {
    __shared__ double sr[256], si[256];
    const int i = blockIdx.x;
    if (!active[i]) return;
    const double2 *h = H + (int64_t)i * C, *u = H + (int64_t)p * C;
    double ar = 0.0, ai = 0.0;
    for (int64_t c = threadIdx.x; c < C; c += 256) {
        ar = fma(h[c].x, u[c].x, fma(h[c].y, u[c].y, ar));
        ai = fma(h[c].y, u[c].x, fma(-h[c].x, u[c].y, ai));
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        coef[i] = make_double2(sr[0], si[0]);
        Rrow[i] = make_double2(Rrow[i].x + sr[0] / nu, Rrow[i].y - si[0] / nu);
    }
}

// h_i <- h_i - (c_i / nu^2) u for the active rows
__global__ void row_update_kernel(double2 *__restrict__ H, int64_t C, int NG, int p, const int *__restrict__ active,
                                  const double2 *__restrict__ coef, double inv_nu2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * C) return;
    const int i = (int)(t / C);
    if (!active[i]) return;
    const int64_t c = t % C;
    const double2 u = H[(int64_t)p * C + c], f = coef[i];
    const double fr = f.x * inv_nu2, fi = f.y * inv_nu2;
    H[t].x -= fr * u.x - fi * u.y;
    H[t].y -= fr * u.y + fi * u.x;
}

__global__ void set_entry_kernel(double2 *__restrict__ a, int64_t idx, double re, int *__restrict__ flags,
                                 int fidx) {
    a[idx] = make_double2(re, 0.0);
    flags[fidx] = 0;
}

// T = R11^{-1} R12 by back substitution, one thread per column of R12:
// R11[t][u] = R[t][piv[u]], R12[t][jj] = R[t][J[jj]]; R rows of length NG
__global__ void ttrsm_kernel(const double2 *__restrict__ R, int NG, int k, const int *__restrict__ piv,
                             const int *__restrict__ J, int nJ, double2 *__restrict__ T) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= nJ) return;
    for (int t = k - 1; t >= 0; --t) {
        const double2 *r = R + (int64_t)t * NG;
        double sr = r[J[jj]].x, si = r[J[jj]].y;
        for (int u = t + 1; u < k; ++u) {
            const double2 a = r[piv[u]], b = T[(int64_t)u * nJ + jj];
            sr -= a.x * b.x - a.y * b.y;
            si -= a.x * b.y + a.y * b.x;
        }
        const double2 d = r[piv[t]];
        const double den = d.x * d.x + d.y * d.y;
        T[(int64_t)t * nJ + jj] = make_double2((sr * d.x + si * d.y) / den, (si * d.x - sr * d.y) / den);
    }
}

// X (NG x k, row-major, columns in ascending ring order): X[piv[s], col[s]] = 1,
// X[J[jj], col[s]] = conj(T[s][jj])
__global__ void assemble_x_kernel(const double2 *__restrict__ T, const int *__restrict__ piv,
                                  const int *__restrict__ J, const int *__restrict__ colof, int k, int nJ,
                                  double2 *__restrict__ X) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k * (nJ + 1)) return;
    const int s = t / (nJ + 1), jj = t % (nJ + 1);
    if (jj == nJ) {
        X[(int64_t)piv[s] * k + colof[s]] = make_double2(1.0, 0.0);
    } else {
        const double2 v = T[(int64_t)s * nJ + jj];
        X[(int64_t)J[jj] * k + colof[s]] = make_double2(v.x, -v.y);
    }
}

// Y_m = S_m X (NG x k), then S~_m = X^T Y_m (k x k); S row-major [M+1][NG][NG]
__global__ void sx_kernel(const double2 *__restrict__ S, const double2 *__restrict__ X, int NG, int k, int M,
                          double2 *__restrict__ Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(M + 1) * NG * k) return;
    const int m = (int)(t / ((int64_t)NG * k)), i = (int)((t / k) % NG), c = (int)(t % k);
    const double2 *s = S + ((int64_t)m * NG + i) * NG;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < NG; ++j) {
        const double2 a = s[j], b = X[(int64_t)j * k + c];
        re = fma(a.x, b.x, fma(-a.y, b.y, re));
        im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    Y[t] = make_double2(re, im);
}

__global__ void xty_kernel(const double2 *__restrict__ X, const double2 *__restrict__ Y, int NG, int k, int M,
                           double2 *__restrict__ St) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(M + 1) * k * k) return;
    const int m = (int)(t / ((int64_t)k * k)), a = (int)((t / k) % k), c = (int)(t % k);
    const double2 *y = Y + (int64_t)m * NG * k;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < NG; ++i) {
        const double2 p = X[(int64_t)i * k + a], q = y[(int64_t)i * k + c];
        re = fma(p.x, q.x, fma(-p.y, q.y, re));
        im = fma(p.x, q.y, fma(p.y, q.x, im));
    }
    St[t] = make_double2(re, im);
}

// restriction out = alpha (X^T (x) I) y and prolongation out = add + (X (x) I) w,
// body by body; vectors [nrhs][N] (full) and [nrhs][Ns] (skeleton)
__global__ void restrict_kernel(const SkelBody *__restrict__ sb, int nb, const double2 *__restrict__ X,
                                const double2 *__restrict__ y, int64_t N, int64_t Ns, int nrhs, double alpha,
                                double2 *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Ns * nrhs) return;
    const int cc = (int)(t / Ns);
    const int64_t s = t % Ns;
    int b = 0;
    while (b + 1 < nb && sb[b + 1].s0 <= s) ++b;
    const SkelBody d = sb[b];
    const int64_t loc = s - d.s0;
    const int col = (int)(loc / d.NF), l = (int)(loc % d.NF);
    const double2 *x = X + d.xoff;
    const double2 *yy = y + (int64_t)cc * N + d.o0;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < d.NG; ++i) {
        const double2 a = x[(int64_t)i * d.k + col], v = yy[(int64_t)i * d.NF + l];
        re = fma(a.x, v.x, fma(-a.y, v.y, re));
        im = fma(a.x, v.y, fma(a.y, v.x, im));
    }
    out[t] = make_double2(alpha * re, alpha * im);
}

__global__ void prolong_kernel(const SkelBody *__restrict__ sb, int nb, const double2 *__restrict__ X,
                               const double2 *__restrict__ w, const double2 *__restrict__ add, int64_t N, int64_t Ns,
                               int nrhs, double2 *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int cc = (int)(t / N);
    const int64_t n = t % N;
    int b = 0;
    while (b + 1 < nb && sb[b + 1].o0 <= n) ++b;
    const SkelBody d = sb[b];
    const int64_t loc = n - d.o0;
    const int i = (int)(loc / d.NF), l = (int)(loc % d.NF);
    const double2 *x = X + d.xoff + (int64_t)i * d.k;
    const double2 *ww = w + (int64_t)cc * Ns + d.s0;
    double re = add ? add[t].x : 0.0, im = add ? add[t].y : 0.0;
    for (int c = 0; c < d.k; ++c) {
        const double2 a = x[c], v = ww[(int64_t)c * d.NF + l];
        re = fma(a.x, v.x, fma(-a.y, v.y, re));
        im = fma(a.x, v.y, fma(a.y, v.x, im));
    }
    out[t] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
double skel_sumsq(Ctx &c, const double2 *a, int64_t n);
static double sumsq(Ctx &c, const double2 *a, int64_t n) { return skel_sumsq(c, a, n); }
double skel_sumsq(Ctx &c, const double2 *a, int64_t n) {
    const int nblk = 256;
    double *part = (double *)c.scratch(WS_RED, nblk * sizeof(double));
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(nblk), dim3(256), 0, c.stream, a, n, part);
    AXS_HIP(hipGetLastError());
    std::vector<double> h(nblk);
    AXS_HIP(hipMemcpyAsync(h.data(), part, nblk * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));
    double s = 0.0;
    for (double v : h) s += v;
    return s;
}

// sum |a + b|^2 (the residual b - A s with b = -y is -(A s + y))
__global__ void sumsq_sum_partial_kernel(const double2 *__restrict__ a, const double2 *__restrict__ b, int64_t n,
                                         double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const double x = a[t].x + b[t].x, y = a[t].y + b[t].y;
        acc = fma(x, x, fma(y, y, acc));
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

double skel_residual_sumsq(Ctx &c, const double2 *a, const double2 *b, int64_t n) {
    const int nblk = 256;
    double *part = (double *)c.scratch(WS_RED, nblk * sizeof(double));
    hipLaunchKernelGGL(sumsq_sum_partial_kernel, dim3(nblk), dim3(256), 0, c.stream, a, b, n, part);
    AXS_HIP(hipGetLastError());
    std::vector<double> h(nblk);
    AXS_HIP(hipMemcpyAsync(h.data(), part, nblk * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    AXS_HIP(hipStreamSynchronize(c.stream));
    double s = 0.0;
    for (double v : h) s += v;
    return s;
}

// Gauss-Legendre rings in polar angle on the sphere of radius R
static void proxy_rings(double R, int n, std::vector<double> &r, std::vector<double> &z, std::vector<double> &nr,
                        std::vector<double> &nz, std::vector<double> &w) {
    std::vector<double> x, wq;
    gauss_legendre_rule(n, x, wq);
    r.resize(n);
    z.resize(n);
    nr.resize(n);
    nz.resize(n);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        const double th = 0.5 * M_PI * (x[j] + 1.0), wt = 0.5 * M_PI * wq[j];
        r[j] = R * std::sin(th);
        z[j] = R * std::cos(th);
        nr[j] = std::sin(th);
        nz[j] = std::cos(th);
        w[j] = R * R * std::sin(th) * wt;
    }
}

// k^G_m w of the proxy configuration of one shape (Sec. 5, first item):
// kin [NG n_in][M+1] -- target contour node i, source proxy node j on the
// sphere of radius R_p with its normal and weight (every field the body can
// receive); kout [(2 n_out) NG][M+1] -- target proxy node j on the spheres of
// radii R_p, then 1.25 R_p, source contour node i with its area weight (every
// field it sends out).  s_in, s_out: 1 / the Frobenius norms of the two.
static void proxy_fields(Ctx &c, const Shape &s, double R_p, int n_in, int n_out, double2 *&kin, double2 *&kout,
                         double &s_in, double &s_out) {
    const int NG = s.NG, M = s.M;
    double need = 4.0 * s.kappa * 1.25 * R_p + 64.0;
    int Nt = 64;
    while (Nt < need) Nt += 64;
    std::vector<double> nr(NG), nz(NG), aw(NG);
    for (int i = 0; i < NG; ++i) {
        const double sp = std::hypot(s.dr[i], s.dz[i]);
        nr[i] = -s.dz[i] / sp;
        nz[i] = s.dr[i] / sp;
        aw[i] = s.r[i] * sp * s.gw[i];
    }
    // the body's own kernel (real coupling eta at kappa = 0) for its outgoing
    // fields; the proxy's sources use i eta at every frequency, since at kappa = 0
    // the layer D + eta S on a sphere of radius R_p has no interior field of
    // degree l = eta R_p - 1 (its factor is eta R_p - (l + 1))
    const double gr = s.kappa > 0 ? 0.0 : s.eta, gi = s.kappa > 0 ? s.eta : 0.0;
    std::vector<double> pr, pz, pnr, pnz, pw;
    proxy_rings(R_p, n_in, pr, pz, pnr, pnz, pw);
    const int64_t Pin = (int64_t)NG * n_in;
    std::vector<double> h(7 * Pin);
    for (int i = 0; i < NG; ++i)
        for (int j = 0; j < n_in; ++j) {
            const int64_t q = (int64_t)i * n_in + j;
            h[q] = s.r[i];
            h[Pin + q] = pr[j];
            h[2 * Pin + q] = pr[j] - s.r[i];
            h[3 * Pin + q] = pz[j] - s.z[i];
            h[4 * Pin + q] = pnr[j];
            h[5 * Pin + q] = pnz[j];
            h[6 * Pin + q] = pw[j];
        }
    kin = (double2 *)c.dalloc((size_t)Pin * (M + 1) * sizeof(double2));
    modal_values(c, s.kappa, 0.0, s.eta, M, Nt, h, Pin, kin);
    const int64_t Pout = (int64_t)2 * n_out * NG;
    std::vector<double> g(7 * Pout);
    for (int rr = 0; rr < 2; ++rr) {
        proxy_rings(rr == 0 ? R_p : 1.25 * R_p, n_out, pr, pz, pnr, pnz, pw);
        for (int j = 0; j < n_out; ++j)
            for (int i = 0; i < NG; ++i) {
                const int64_t q = ((int64_t)(rr * n_out + j)) * NG + i;
                g[q] = pr[j];
                g[Pout + q] = s.r[i];
                g[2 * Pout + q] = s.r[i] - pr[j];
                g[3 * Pout + q] = s.z[i] - pz[j];
                g[4 * Pout + q] = nr[i];
                g[5 * Pout + q] = nz[i];
                g[6 * Pout + q] = aw[i] * pw[j];
            }
    }
    kout = (double2 *)c.dalloc((size_t)Pout * (M + 1) * sizeof(double2));
    modal_values(c, s.kappa, gr, gi, M, Nt, g, Pout, kout);
    s_in = 1.0 / std::sqrt(sumsq(c, kin, Pin * (M + 1)));
    s_out = 1.0 / std::sqrt(sumsq(c, kout, Pout * (M + 1)));
}

// row ID of one shape: skeleton rings (ascending) and X (device, NG x k)
static void ring_id(Ctx &c, const Shape &s, double R_p, double eps, std::vector<int> &rings, double2 *&X) {
    const int NG = s.NG, M = s.M, n_in = NG, n_o = 2 * NG;
    double2 *kin = nullptr, *kout = nullptr;
    double s_in = 0, s_out = 0;
    proxy_fields(c, s, R_p, NG, NG, kin, kout, s_in, s_out);
    // H with each block scaled to unit Frobenius norm
    const int64_t C = (int64_t)(M + 1) * (n_in + n_o);
    double2 *H = (double2 *)c.dalloc((size_t)NG * C * sizeof(double2));
    hipLaunchKernelGGL(build_h_kernel, dim3(ceil_div((int64_t)NG * C, 256)), dim3(256), 0, c.stream, kin, kout, NG,
                       n_in, n_o, M, s_in, s_out, H);
    AXS_HIP(hipGetLastError());
    // pivoted Gram-Schmidt over the rows (= column-pivoted QR of H^*), two
    // projections per step; stop when the pivot norm falls below eps x the first
    int *active = (int *)c.dalloc(NG * sizeof(int));
    std::vector<int> one(NG, 1);
    AXS_HIP(hipMemcpy(active, one.data(), NG * sizeof(int), hipMemcpyHostToDevice));
    double *nrm = (double *)c.dalloc(NG * sizeof(double));
    double2 *coef = (double2 *)c.dalloc(NG * sizeof(double2));
    double2 *R = (double2 *)c.dalloc((size_t)NG * NG * sizeof(double2));
    AXS_HIP(hipMemsetAsync(R, 0, (size_t)NG * NG * sizeof(double2), c.stream));
    std::vector<int> piv;
    std::vector<char> used(NG, 0);
    std::vector<double> hn(NG);
    double d0 = 0.0;
    for (int st = 0; st < NG; ++st) {
        hipLaunchKernelGGL(row_norms_kernel, dim3(NG), dim3(256), 0, c.stream, H, C, active, nrm);
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipMemcpyAsync(hn.data(), nrm, NG * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        int p = -1;
        for (int i = 0; i < NG; ++i)
            if (!used[i] && (p < 0 || hn[i] > hn[p])) p = i;
        const double nu = std::sqrt(std::max(hn[p], 0.0));
        AXS_REQUIRE(std::isfinite(nu), AXS_ENONFINITE, "non-finite proxy matrix");
        if (st == 0) d0 = nu;
        if (!(nu > eps * d0)) break;
        piv.push_back(p);
        used[p] = 1;
        double2 *Rrow = R + (int64_t)st * NG;
        hipLaunchKernelGGL(set_entry_kernel, dim3(1), dim3(1), 0, c.stream, Rrow, (int64_t)p, nu, active, p);
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(row_dots_kernel, dim3(NG), dim3(256), 0, c.stream, H, C, p, active, nu, coef, Rrow);
            hipLaunchKernelGGL(row_update_kernel, dim3(ceil_div((int64_t)NG * C, 256)), dim3(256), 0, c.stream, H,
                               C, NG, p, active, coef, 1.0 / (nu * nu));
            AXS_HIP(hipGetLastError());
        }
    }
    const int k = (int)piv.size();
    std::vector<int> J;
    for (int i = 0; i < NG; ++i)
        if (!used[i]) J.push_back(i);
    rings = piv;
    std::sort(rings.begin(), rings.end());
    std::vector<int> colof(k);
    for (int t = 0; t < k; ++t) colof[t] = (int)(std::lower_bound(rings.begin(), rings.end(), piv[t]) - rings.begin());
    const int nJ = (int)J.size();
    int *d_piv = (int *)c.dalloc((k + nJ + k + 1) * sizeof(int));
    int *d_J = d_piv + k, *d_col = d_J + nJ;
    AXS_HIP(hipMemcpy(d_piv, piv.data(), k * sizeof(int), hipMemcpyHostToDevice));
    if (nJ) AXS_HIP(hipMemcpy(d_J, J.data(), nJ * sizeof(int), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_col, colof.data(), k * sizeof(int), hipMemcpyHostToDevice));
    double2 *T = (double2 *)c.dalloc((size_t)std::max(1, k * nJ) * sizeof(double2));
    if (nJ) {
        hipLaunchKernelGGL(ttrsm_kernel, dim3(ceil_div(nJ, 64)), dim3(64), 0, c.stream, R, NG, k, d_piv, d_J, nJ, T);
        AXS_HIP(hipGetLastError());
    }
    X = (double2 *)c.dalloc((size_t)NG * k * sizeof(double2));
    AXS_HIP(hipMemsetAsync(X, 0, (size_t)NG * k * sizeof(double2), c.stream));
    hipLaunchKernelGGL(assemble_x_kernel, dim3(ceil_div(k * (nJ + 1), 256)), dim3(256), 0, c.stream, T, d_piv, d_J,
                       d_col, k, nJ, X);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));
    for (void *q : {(void *)kin, (void *)kout, (void *)H, (void *)active, (void *)nrm, (void *)coef, (void *)R,
                    (void *)d_piv, (void *)T})
        c.dfree(q);
}

void skeletonize(Ctx &c, double eps, double factor) {
    AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
    AXS_REQUIRE(eps > 0 && eps < 1 && factor > 1, AXS_EINVAL, "need 0 < eps < 1 and proxy factor > 1");
    auto sk = std::make_unique<Skeleton>();
    const size_t nsh = c.shapes.size(), nb = c.bodies.size();
    AXS_REQUIRE(nb >= 2, AXS_EINVAL, "skeletonization needs at least two bodies");
    // proxy radius per shape: the largest sphere around each of its bodies that
    // stays out of every other body's bounding ball, capped at factor x r_b
    std::vector<double> Rp(nsh, 1e300), rb(nsh, 0.0);
    for (size_t b = 0; b < nb; ++b) {
        const Body &B = c.bodies[b];
        double gap = 1e300;
        for (size_t q = 0; q < nb; ++q) {
            if (q == b) continue;
            const Body &Q = c.bodies[q];
            const double d = std::sqrt((B.centre[0] - Q.centre[0]) * (B.centre[0] - Q.centre[0]) +
                                       (B.centre[1] - Q.centre[1]) * (B.centre[1] - Q.centre[1]) +
                                       (B.centre[2] - Q.centre[2]) * (B.centre[2] - Q.centre[2]));
            gap = std::min(gap, d - Q.bound_radius);
        }
        Rp[B.shape] = std::min(Rp[B.shape], std::min(factor * B.bound_radius, gap));
        rb[B.shape] = std::max(rb[B.shape], B.bound_radius);
    }
    // per shape: ID (or the identity where no proxy sphere fits), S~_m = X^T S_m X
    std::vector<std::vector<int>> rings(nsh);
    std::vector<double2 *> Xs(nsh), St(nsh);
    int64_t xtot = 0;
    std::vector<int64_t> xoff(nsh);
    for (size_t k = 0; k < nsh; ++k) {
        const Shape &s = c.shapes[k];
        if (Rp[k] >= 1.05 * rb[k]) {
            ring_id(c, s, Rp[k], eps, rings[k], Xs[k]);
        } else {
            rings[k].resize(s.NG);
            std::iota(rings[k].begin(), rings[k].end(), 0);
            std::vector<double2> id((size_t)s.NG * s.NG, make_double2(0.0, 0.0));
            for (int i = 0; i < s.NG; ++i) id[(size_t)i * s.NG + i] = make_double2(1.0, 0.0);
            Xs[k] = (double2 *)c.dalloc(id.size() * sizeof(double2));
            AXS_HIP(hipMemcpy(Xs[k], id.data(), id.size() * sizeof(double2), hipMemcpyHostToDevice));
        }
        const int kk = (int)rings[k].size(), NG = s.NG, M = s.M;
        double2 *Y = (double2 *)c.dalloc((size_t)(M + 1) * NG * kk * sizeof(double2));
        St[k] = (double2 *)c.dalloc((size_t)(M + 1) * kk * kk * sizeof(double2));
        hipLaunchKernelGGL(sx_kernel, dim3(ceil_div((int64_t)(M + 1) * NG * kk, 256)), dim3(256), 0, c.stream,
                           (const double2 *)s.S64, Xs[k], NG, kk, M, Y);
        hipLaunchKernelGGL(xty_kernel, dim3(ceil_div((int64_t)(M + 1) * kk * kk, 256)), dim3(256), 0, c.stream, Xs[k],
                           Y, NG, kk, M, St[k]);
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(Y);
        xoff[k] = xtot;
        xtot += (int64_t)NG * kk;
    }
    // all X in one array (per shape offsets)
    sk->X = (double2 *)c.dalloc((size_t)xtot * sizeof(double2));
    for (size_t k = 0; k < nsh; ++k) {
        AXS_HIP(hipMemcpyAsync(sk->X + xoff[k], Xs[k], (size_t)c.shapes[k].NG * rings[k].size() * sizeof(double2),
                               hipMemcpyDeviceToDevice, c.stream));
    }
    AXS_HIP(hipStreamSynchronize(c.stream));
    for (auto *p : Xs) c.dfree(p);
    // the child context: skeleton rings of every shape, S~_m in place of S_m
    sk->child = std::make_unique<Ctx>();
    Ctx &ch = *sk->child;
    ch.device = c.device;
    ch.stream = c.stream;
    ch.alloc = c.alloc;
    ch.free_fn = c.free_fn;
    ch.user = c.user;
    ch.have_k = true;
    ch.kappa = c.kappa;
    ch.eta = c.eta;
    ch.gam_re = c.gam_re;
    ch.gam_im = c.gam_im;
    for (size_t k = 0; k < nsh; ++k) {
        const Shape &s = c.shapes[k];
        Shape t;
        t.n_panels = s.n_panels;
        t.p = s.p;
        t.NG = (int)rings[k].size();
        t.M = s.M;
        t.NF = s.NF;
        t.Nt = s.Nt;
        t.kappa = s.kappa;
        t.eta = s.eta;
        for (int i : rings[k]) {
            t.r.push_back(s.r[i]);
            t.z.push_back(s.z[i]);
            t.dr.push_back(s.dr[i]);
            t.dz.push_back(s.dz[i]);
            t.gw.push_back(s.gw[i]);
        }
        t.bodies = s.bodies;
        t.S64 = (double *)St[k];
        t.A64 = nullptr;
        ch.shapes.push_back(t);
        sk->rank.push_back(t.NG);
        sk->rings.push_back(rings[k]);
    }
    std::vector<SkelBody> desc;
    int64_t off = 0;
    for (size_t b = 0; b < nb; ++b) {
        Body B = c.bodies[b];
        const Shape &t = ch.shapes[B.shape];
        SkelBody d{};
        d.o0 = B.offset;
        d.s0 = off;
        d.NG = c.shapes[B.shape].NG;
        d.k = t.NG;
        d.NF = t.NF;
        d.xoff = xoff[B.shape];
        desc.push_back(d);
        B.offset = off;
        B.n = (int64_t)t.NG * t.NF;
        off += B.n;
        ch.bodies.push_back(B);
    }
    ch.N = off;
    // the child owns S~_m from here on (they were allocated by the parent)
    for (auto *p : St) {
        auto it = std::find(c.owned.begin(), c.owned.end(), (void *)p);
        if (it != c.owned.end()) c.owned.erase(it);
        ch.owned.push_back(p);
    }
    finish_precompute(ch);
    sk->desc = (SkelBody *)c.dalloc(desc.size() * sizeof(SkelBody));
    AXS_HIP(hipMemcpy(sk->desc, desc.data(), desc.size() * sizeof(SkelBody), hipMemcpyHostToDevice));
    sk->Ns = ch.N;
    sk->eps = eps;
    release_skeleton(c);
    c.skel = std::move(sk);
}

void release_skeleton(Ctx &c) {
    if (!c.skel) return;
    AXS_HIP(hipStreamSynchronize(c.stream));
    if (c.skel->X) c.dfree(c.skel->X);
    if (c.skel->desc) c.dfree(c.skel->desc);
    if (c.skel->pts) {
        for (auto *p : c.skel->pts->XT) c.dfree(p);
        for (auto *p : c.skel->pts->S64) c.dfree(p);
        for (auto *p : c.skel->pts->S32) c.dfree(p);
        if (c.skel->pts->sp_items) c.dfree(c.skel->pts->sp_items);
        if (c.skel->pts->rs_items) c.dfree(c.skel->pts->rs_items);
    }
    c.skel.reset();
}

static void point_restrict(Ctx &c, const void *y, void *out, int nrhs, double alpha);
static BodyMatItem *upload_items(Ctx &c, const std::vector<BodyMatItem> &bodies, int &count);
static void point_prolong(Ctx &c, const void *w, const void *add, void *out, int nrhs);

// restrict / prolong between the full and the skeleton vectors
void skel_restrict(Ctx &c, const void *y, void *out, int nrhs, double alpha) {
    if (c.skel->kind == 1) return point_restrict(c, y, out, nrhs, alpha);
    const Skeleton &sk = *c.skel;
    const int64_t tot = sk.Ns * nrhs;
    hipLaunchKernelGGL(restrict_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, sk.desc,
                       (int)c.bodies.size(), sk.X, (const double2 *)y, c.N, sk.Ns, nrhs, alpha, (double2 *)out);
    AXS_HIP(hipGetLastError());
}

void skel_prolong(Ctx &c, const void *w, const void *add, void *out, int nrhs) {
    if (c.skel->kind == 1) return point_prolong(c, w, add, out, nrhs);
    const Skeleton &sk = *c.skel;
    const int64_t tot = c.N * nrhs;
    hipLaunchKernelGGL(prolong_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, sk.desc,
                       (int)c.bodies.size(), sk.X, (const double2 *)w, (const double2 *)add, c.N, sk.Ns, nrhs,
                       (double2 *)out);
    AXS_HIP(hipGetLastError());
}

// ===========================================================================
// Point skeletons (Sec. 5 with single-node index sets I_p)
// ===========================================================================
// The row ID runs over the N_G N_F nodes (i, l) of a shape against the proxy
// matrix  H[(i, l), (m, c)] = Hm[i, c] e^{i m theta_l},  m = -M..M,
// Hm = [IN_|m| | OUT_|m|^T] (the proxy fields above with n_proxy polar points
// per sphere): a proxy ring with the azimuthal profile e^{i m phi} makes the
// field IN_|m|[i, c] e^{i m theta_l} at node (i, l), and a node's field along an
// outgoing proxy ring has the coefficient OUT_|m|[c, i] e^{-i m theta_l}.  By
// the remark of Sec. 5 on randomized sampling the ID is taken of a sketch:
//     A = Psi H^*  (ell x n),  Psi complex Gaussian (ell x (2M+1) C'),
// so A[s, (i, l)] = sum_m e^{-i m theta_l} W_m[s, i],  W_m = Psi_m conj(H_|m|)^T:
// 2M+1 GEMMs of ell x C' x NG and one DFT GEMM per contour node.  The columns
// of A (= nodes) are chosen by QR with randomized column pivoting in blocks
// of 64 (as in Martinsson, Quintana-Orti, Heavner and van de Geijn's HQRRP),
// left-looking: one 80-row Gaussian sketch of A, downdated after each block,
// chooses the pivots (pivoted Gram-Schmidt on the device); each panel is
// projected against the earlier blocks and orthonormalised by CholeskyQR2,
// and its rows of R_12 are one GEMM over the trailing columns, which are never
// updated (see hqrrp); the rank k is the first pivot with |R_kk| < eps
// |R_00|, and X(J, :) = (R_11^{-1} R_12)^* as in the ring version.  The sketch
// width ell starts at 256 (for later shapes at 1.25 k + 64 of the shape
// before) and grows (by the decay of |R_jj| seen so far) until k <= ell - 16.
// Then
//   S_p = X^T A_pp^{-1} X  (k x k, dense) from per-mode products with S_m,
//   B~ the inter-body sum over the skeleton nodes (point order; MFMA orders
//   from 16 rhs),
// and the compressed system runs in a child context whose operator is
// s~ + S B~ s~ (S_p applied per body by body_matvec_kernel, all bodies in one
// launch).
#define AXS_BLAS(call)                                                                                      \
    do {                                                                                                    \
        rocblas_status st_ = (call);                                                                        \
        if (st_ != rocblas_status_success)                                                                  \
            throw ::axs::Error{AXS_EHIP, std::string(#call) + ": " + rocblas_status_to_string(st_)};        \
    } while (0)

static rocblas_handle blas_of(Ctx &c) {
    if (!c.blas) {
        rocblas_handle h = nullptr;
        AXS_BLAS(rocblas_create_handle(&h));
        c.blas = h;
    }
    rocblas_handle h = (rocblas_handle)c.blas;
    AXS_BLAS(rocblas_set_stream(h, c.stream));
    return h;
}

void destroy_blas(Ctx &c) {
    if (c.blas) (void)rocblas_destroy_handle((rocblas_handle)c.blas);
    c.blas = nullptr;
}

static inline rocblas_double_complex *zc(double2 *p) { return (rocblas_double_complex *)p; }
static inline const rocblas_double_complex *zc(const double2 *p) { return (const rocblas_double_complex *)p; }

// the counter-based generator of the sketch: SplitMix64 (Steele, Lea and
// Flood) of seed * 0x632BE59BD9B4E019 + counter, top 53 bits centred in their
// interval; complex Gaussian by Box-Muller, sqrt(-2 ln u1) e^{2 pi i u2}
__device__ __forceinline__ uint64_t sk_splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}
__device__ __forceinline__ double sk_uniform01(uint64_t seed, uint64_t k) {
    return ((double)(sk_splitmix64(seed * 0x632BE59BD9B4E019ULL + k) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
__device__ __forceinline__ double2 sk_gauss(uint64_t seed, uint64_t e) {
    const double u1 = sk_uniform01(seed, 2 * e), u2 = sk_uniform01(seed, 2 * e + 1);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    return make_double2(rad * cs, rad * sn);
}

// G (rows x cols, column-major): G[r + q rows] = conj(gauss(seed, q_total_rows... )):
// entry (r, q) from draw e = r * stride_r + q * stride_q, conjugated if conj
__global__ void gauss_fill_kernel(double2 *__restrict__ G, int rows, int64_t cols, uint64_t seed, int64_t stride_r,
                                  int64_t stride_q, int conj) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    const int r = (int)(t % rows);
    const int64_t q = t / rows;
    double2 v = sk_gauss(seed, (uint64_t)(r * stride_r + q * stride_q));
    if (conj) v.y = -v.y;
    G[t] = v;
}

__global__ void conj_kernel(double2 *__restrict__ a, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t].y = -a[t].y;
}

// diagonal entries A[j0 + t, j0 + t], t < b (column-major, leading dimension ld)
__global__ void diag_kernel(const double2 *__restrict__ A, int64_t ld, int j0, int b, double2 *__restrict__ d) {
    const int t = threadIdx.x;
    if (t < b) d[t] = A[(int64_t)(j0 + t) + (int64_t)(j0 + t) * ld];
}

// column moves of A (rows x cols, leading dimension ld): phase 0 copies the
// source columns to tmp, phase 1 tmp to the destination columns
__global__ void move_cols_kernel(double2 *__restrict__ A, int64_t ld, int rows, const int2 *__restrict__ mv,
                                 int cnt, double2 *__restrict__ tmp, int phase) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cnt) return;
    const int r = (int)(t % rows), j = (int)(t / rows);
    if (phase == 0)
        tmp[t] = A[(int64_t)mv[j].y * ld + r];
    else
        A[(int64_t)mv[j].x * ld + r] = tmp[t];
}

// X^T (k x n, column-major, rows in ascending skeleton order colof[t]):
// column perm[q] = e_colof[q] for q < k, conj(T[:, q]) for q >= k, where T =
// R_11^{-1} R_12 sits in A[0:k, k:n] (leading dimension ld)
__global__ void assemble_xt_kernel(const double2 *__restrict__ A, int64_t ld, const int *__restrict__ perm,
                                   const int *__restrict__ colof, int k, int64_t n, double2 *__restrict__ XT) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)k * n) return;
    const int a = (int)(t % k);
    const int64_t q = t / k;
    const int64_t node = perm[q];
    double2 v;
    if (q < k) {
        v = make_double2(a == (int)q ? 1.0 : 0.0, 0.0);
    } else {
        const double2 tv = A[(int64_t)a + q * ld];
        v = make_double2(tv.x, -tv.y);
    }
    XT[(int64_t)colof[a] + node * k] = v;
}

__global__ void to_c64_kernel(const double2 *__restrict__ a, int64_t n, float2 *__restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = make_float2((float)a[t].x, (float)a[t].y);
}

// node arrays of the skeleton: rows of the parent's [7][N] FP64 arrays
__global__ void gather_geo_kernel(const double *__restrict__ g, int64_t N, const int64_t *__restrict__ idx,
                                  int64_t Ns, double *__restrict__ g64, float *__restrict__ g32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 7 * Ns) return;
    const int a = (int)(t / Ns);
    const int64_t j = t % Ns;
    const double v = g[a * N + idx[j]];
    g64[t] = v;
    if (a < 6) g32[t] = (float)v;
}

// MFMA source operands of the skeleton nodes: entries 4 idx[j] + c of the
// parent's two [4 N] halves
__global__ void gather_mf_kernel(const double *__restrict__ src, int64_t N, const int64_t *__restrict__ idx,
                                 int64_t Ns, double *__restrict__ dst64, float *__restrict__ dst32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 8 * Ns) return;
    const int64_t half = t / (4 * Ns), rem = t % (4 * Ns), j = rem / 4, comp = rem % 4;
    const double v = src[half * 4 * N + 4 * idx[j] + comp];
    dst64[t] = v;
    dst32[t] = (float)v;
}

// e^{sign i (m' - M) 2 pi l / NF} * scale as a column-major matrix: rows m'
// (2M+1) x cols l (NF) if mode_rows, else rows l x cols m'
static std::vector<double2> dft_matrix(int M, int NF, double sign, double scale, bool mode_rows) {
    const int nm = 2 * M + 1;
    std::vector<double2> E((size_t)nm * NF);
    for (int mp = 0; mp < nm; ++mp)
        for (int l = 0; l < NF; ++l) {
            // the angle reduced to (-pi, pi] before the sine and cosine
            const int64_t r = ((int64_t)(mp - M) * l) % NF;
            const double a = sign * 2.0 * M_PI * (double)r / NF;
            const double2 v = make_double2(scale * std::cos(a), scale * std::sin(a));
            if (mode_rows)
                E[(size_t)mp + (size_t)l * nm] = v;
            else
                E[(size_t)l + (size_t)mp * NF] = v;
        }
    return E;
}

static double2 *upload(Ctx &c, const std::vector<double2> &h) {
    double2 *d = (double2 *)c.dalloc(h.size() * sizeof(double2));
    AXS_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice));
    return d;
}

// Column selection on a small sketch G (rows x n, column-major) by pivoted
// Gram-Schmidt, one wavefront per column and the pivot chosen on the device:
// no host round trip per pivot.  nrm[j] < 0 marks a column already chosen.
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// the best remaining column of a block of 4 wavefronts (one column each, lane
// 0 holding its squared norm a, -1 for a chosen or absent column): part_v /
// part_i[blockIdx.x]; NaN never wins, ties go to the smaller column
__device__ __forceinline__ void gcol_block_best(double a, int64_t col, double *__restrict__ part_v,
                                                int *__restrict__ part_i) {
    __shared__ double sv[4];
    __shared__ int si[4];
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = a;
        si[threadIdx.x >> 6] = a >= 0.0 ? (int)col : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bv = -1.0;
        int bi = -1;
        for (int w = 0; w < 4; ++w)   // columns rise with w: the first maximum stays
            if (si[w] >= 0 && sv[w] > bv) {
                bv = sv[w];
                bi = si[w];
            }
        part_v[blockIdx.x] = bv;
        part_i[blockIdx.x] = bi;
    }
}

__global__ __launch_bounds__(256) void gcol_norms_kernel(const double2 *__restrict__ G, int rows, int64_t n,
                                                         double *__restrict__ nrm, double *__restrict__ part_v,
                                                         int *__restrict__ part_i) {
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double a = -1.0;
    if (col < n) {   // the same for the whole wavefront
        const double2 *g = G + col * rows;
        double acc = 0.0;
        for (int r = lane; r < rows; r += 64) acc = fma(g[r].x, g[r].x, fma(g[r].y, g[r].y, acc));
        a = wave_sum64(acc);
        if (lane == 0) nrm[col] = a;
    }
    gcol_block_best(a, col, part_v, part_i);
}

// the best of the blocks' candidates (ties to the smaller column): piv[t],
// nu2[t], and the column is marked chosen; piv[t] = -1 if none is left
__global__ __launch_bounds__(1024) void gcol_argmax_kernel(const double *__restrict__ part_v,
                                                           const int *__restrict__ part_i, int nparts,
                                                           double *__restrict__ nrm, int *__restrict__ piv,
                                                           double *__restrict__ nu2, int t) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    double bv = -1.0;
    int bi = -1;
    for (int q = threadIdx.x; q < nparts; q += 1024) {   // blocks rise within a thread
        const int i = part_i[q];
        const double v = part_v[q];
        if (i >= 0 && v > bv) {
            bv = v;
            bi = i;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o];
            const int i2 = si[threadIdx.x + o];
            const double v1 = sv[threadIdx.x];
            const int i1 = si[threadIdx.x];
            if (i2 >= 0 && (i1 < 0 || v2 > v1 || (v2 == v1 && i2 < i1))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        piv[t] = si[0];
        nu2[t] = sv[0];
        if (si[0] >= 0) nrm[si[0]] = -1.0;
    }
}

// one Gram-Schmidt step against the pivot column piv[t]: one projection, the
// squared norm recomputed from the updated column in the same pass (not
// downdated), and each block's best remaining column for the next argmax.
// A column (rows <= 128) is read once into registers, two entries per lane.
// Chosen columns (nrm < 0) are left alone.
__global__ __launch_bounds__(256) void gcol_step_kernel(double2 *__restrict__ G, int rows, int64_t n,
                                                        const int *__restrict__ piv, const double *__restrict__ nu2,
                                                        int t, double *__restrict__ nrm, double *__restrict__ part_v,
                                                        int *__restrict__ part_i) {
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = piv[t];
    const double s = nu2[t];
    double a = -1.0;
    if (col < n && p >= 0 && nrm[col] >= 0.0) {   // uniform across the wavefront
        double2 *g = G + col * rows;
        const double2 *u = G + (int64_t)p * rows;
        const bool h0 = lane < rows, h1 = lane + 64 < rows;
        const double2 z = make_double2(0.0, 0.0);
        double2 g0 = h0 ? g[lane] : z, g1 = h1 ? g[lane + 64] : z;
        const double2 u0 = h0 ? u[lane] : z, u1 = h1 ? u[lane + 64] : z;
        if (s > 0.0) {
            // <g, u> = sum g conj(u)
            double dr = fma(g0.x, u0.x, fma(g0.y, u0.y, fma(g1.x, u1.x, g1.y * u1.y)));
            double di = fma(g0.y, u0.x, fma(-g0.x, u0.y, fma(g1.y, u1.x, -g1.x * u1.y)));
            dr = wave_sum64(dr) / s;
            di = wave_sum64(di) / s;
            g0.x -= dr * u0.x - di * u0.y;
            g0.y -= dr * u0.y + di * u0.x;
            g1.x -= dr * u1.x - di * u1.y;
            g1.y -= dr * u1.y + di * u1.x;
            if (h0) g[lane] = g0;
            if (h1) g[lane + 64] = g1;
        }
        a = wave_sum64(fma(g0.x, g0.x, fma(g0.y, g0.y, fma(g1.x, g1.x, g1.y * g1.y))));
        if (lane == 0) nrm[col] = a;
    }
    gcol_block_best(a, col, part_v, part_i);
}

// Cholesky factor of a small Hermitian positive definite W (b x b, column-major,
// b <= 64): W = R^H R with R upper triangular (lower part set to zero), one
// wavefront, the upper triangle held packed in LDS (entry (i, t), i <= t, at
// t (t + 1) / 2 + i).  Step j: the pivot from a wavefront reduction of
// |R(i, j)|^2 over i < j, then row j by lane t > j.  info[0] = the first
// column whose pivot is not positive (or not finite), b if none; R is valid
// in the columns before it.
__global__ __launch_bounds__(64) void chol_small_kernel(const double2 *__restrict__ W, int b,
                                                        double2 *__restrict__ R, int *__restrict__ info) {
    __shared__ double2 U[64 * 65 / 2];
    __shared__ int fail;
    const int t = threadIdx.x;
    if (t == 0) fail = b;
    if (t < b)
        for (int i = 0; i <= t; ++i) U[t * (t + 1) / 2 + i] = W[i + t * b];
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        const int cj = j * (j + 1) / 2;
        double part = 0.0;
        if (t < j) part = U[cj + t].x * U[cj + t].x + U[cj + t].y * U[cj + t].y;
        part = wave_sum64(part);
        if (t == 0) {
            const double d = U[cj + j].x - part;
            if (d > 0.0 && d < INFINITY) U[cj + j] = make_double2(sqrt(d), 0.0);
            else fail = j;
        }
        __syncthreads();
        if (fail <= j) break;
        if (t > j && t < b) {
            // R(j, t) = (W(j, t) - sum_{i<j} conj(R(i, j)) R(i, t)) / R(j, j)
            const int ct = t * (t + 1) / 2;
            double2 a = U[ct + j];
            for (int i = 0; i < j; ++i) {
                const double2 u = U[cj + i], v = U[ct + i];
                a.x -= u.x * v.x + u.y * v.y;
                a.y -= u.x * v.y - u.y * v.x;
            }
            const double r = U[cj + j].x;
            U[ct + j] = make_double2(a.x / r, a.y / r);
        }
        __syncthreads();
    }
    if (t < b)
        for (int i = 0; i < b; ++i) R[i + t * b] = i <= t ? U[t * (t + 1) / 2 + i] : make_double2(0.0, 0.0);
    if (t == 0) info[0] = fail;
}

// y += x elementwise (complex)
__global__ void cadd_kernel(double2 *__restrict__ y, const double2 *__restrict__ x, int rows, int64_t cols,
                            int64_t ldy, int64_t ldx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    const int r = (int)(t % rows);
    const int64_t q = t / rows;
    y[r + q * ldy].x += x[r + q * ldx].x;
    y[r + q * ldy].y += x[r + q * ldx].y;
}

// C = s_c C + s_w sum_q W_q (m x n; C with leading dimension ldc, the W_q
// packed m x n one after another); s_c, s_w real
__global__ void sum_slices_kernel(double2 *__restrict__ C, int64_t ldc, const double2 *__restrict__ W, int m,
                                  int n, int nsl, double s_c, double s_w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * n) return;
    const int r = (int)(t % m);
    const int64_t q = t / m;
    double2 a = make_double2(0.0, 0.0);
    for (int sl = 0; sl < nsl; ++sl) {   // fixed order: reproducible
        const double2 w = W[(int64_t)sl * m * n + t];
        a.x += w.x;
        a.y += w.y;
    }
    double2 *c = C + r + q * ldc;
    const double2 c0 = s_c != 0.0 ? *c : make_double2(0.0, 0.0);
    *c = make_double2(s_c * c0.x + s_w * a.x, s_c * c0.y + s_w * a.y);
}

// C = s_w op(A) B + s_c C (op: none or conjugate transpose; s_w, s_c real)
// with the inner dimension K split into slices: a strided batch of GEMMs of
// the slices into W (at most wcap complex entries), then one reduction.  The
// products here have small outputs (64 x 64 Gram matrices, j0 x 64 and
// ell x 64 projections) and long inner dimensions, which one GEMM runs on a
// few workgroups, each down the whole of K.
static void gemm_splitk(Ctx &c, rocblas_handle h, rocblas_operation opA, int m, int n, int K, double s_w,
                        const double2 *A, int lda, const double2 *B, int ldb, double s_c, double2 *C, int ldc,
                        double2 *W, int64_t wcap, int64_t want = 512) {
    const int64_t tiles = ceil_div((int64_t)m, (int64_t)64) * ceil_div((int64_t)n, (int64_t)64);
    int nsl = (int)std::min<int64_t>(std::max<int64_t>(1, want / tiles), K / 64);
    nsl = (int)std::min<int64_t>(nsl, wcap / ((int64_t)m * n));
    const rocblas_double_complex w = {s_w, 0.0}, cc0 = {s_c, 0.0}, one = {1.0, 0.0}, zero = {0.0, 0.0};
    if (nsl < 2) {
        AXS_BLAS(rocblas_zgemm(h, opA, rocblas_operation_none, m, n, K, &w, zc(A), lda, zc(B), ldb, &cc0, zc(C), ldc));
        return;
    }
    const int sl = (K + nsl - 1) / nsl;
    const int full = K / sl, rem = K - full * sl;
    const rocblas_stride sa = opA == rocblas_operation_none ? (rocblas_stride)sl * lda : (rocblas_stride)sl;
    AXS_BLAS(rocblas_zgemm_strided_batched(h, opA, rocblas_operation_none, m, n, sl, &one, zc(A), lda, sa, zc(B), ldb,
                                           (rocblas_stride)sl, &zero, zc(W), m, (rocblas_stride)m * n, full));
    if (rem > 0)
        AXS_BLAS(rocblas_zgemm(h, opA, rocblas_operation_none, m, n, rem, &one, zc(A + full * sa), lda,
                               zc(B + (int64_t)full * sl), ldb, &zero, zc(W + (int64_t)full * m * n), m));
    hipLaunchKernelGGL(sum_slices_kernel, dim3(ceil_div((int64_t)m * n, 256)), dim3(256), 0, c.stream, C,
                       (int64_t)ldc, W, m, n, full + (rem > 0 ? 1 : 0), s_c, s_w);
    AXS_HIP(hipGetLastError());
}

// QR with randomized column pivoting of A (ell x n, leading dimension ell),
// blocks of 64 pivots, until |R_kk| < eps |R_00|; returns k and the column
// order perm (perm[q] = original column at position q).  Rm (ell x n, leading
// dimension ell) then holds R_11 and R_12 in its rows 0..k-1.  Blocked as in
// HQRRP, left-looking:
//   - one Gaussian sketch Y = Omega A (80 rows) of the whole matrix; each
//     block's 64 pivots are chosen on a copy of Y's trailing columns by
//     device-side pivoted Gram-Schmidt; after the block Y is downdated,
//     Y_t <- Y_t - (Y_p R_11^{-1}) R_12, so that it stays the sketch of the
//     trailing columns projected against every chosen column;
//   - the trailing columns of A are never updated: the chosen panel is
//     projected against the Q of the earlier blocks (first pass with the
//     R entries already known, a second pass that recomputes them), then
//     orthonormalised by CholeskyQR2 (Gram matrix, Cholesky, triangular
//     solve, twice); its rows of R_12 are Q_b^H A_t, one GEMM;
// so each block costs one GEMM over the trailing columns instead of the four
// of a right-looking update with reorthogonalisation.
static int hqrrp(Ctx &c, rocblas_handle h, double2 *A, double2 *Rm, int ell, int64_t n, double eps, uint64_t seed,
                 std::vector<int> &perm, std::vector<double> &diag) {
    constexpr int BMAX = 64, P = 16, YR = BMAX + P;
    static_assert(YR <= 128, "gcol_step_kernel holds a sketch column in two entries per lane");
    const int kmax = (int)std::min<int64_t>(ell, n);
    perm.resize(n);
    std::iota(perm.begin(), perm.end(), 0);
    diag.clear();
    double2 *Om = (double2 *)c.dalloc((size_t)YR * ell * sizeof(double2));
    double2 *Y = (double2 *)c.dalloc((size_t)YR * n * sizeof(double2));
    double2 *G = (double2 *)c.dalloc((size_t)YR * n * sizeof(double2));
    double *nrm = (double *)c.dalloc(n * sizeof(double));
    const int64_t maxblk = ceil_div(n, (int64_t)4);
    AXS_REQUIRE(maxblk <= INT32_MAX && n <= INT32_MAX, AXS_EINVAL, "too many nodes in one shape");
    double *part_v = (double *)c.dalloc(maxblk * sizeof(double));
    int *part_i = (int *)c.dalloc(maxblk * sizeof(int));
    int *dpiv = (int *)c.dalloc((BMAX + 2) * sizeof(int));
    int *dinfo = dpiv + BMAX;
    double *dnu2 = (double *)c.dalloc(BMAX * sizeof(double));
    double2 *tmp = (double2 *)c.dalloc((size_t)ell * 2 * BMAX * sizeof(double2));
    double2 *rawA = (double2 *)c.dalloc((size_t)ell * BMAX * sizeof(double2));   // the panel before projection
    double2 *rawR = (double2 *)c.dalloc((size_t)ell * BMAX * sizeof(double2));   // its R rows 0..j0-1
    int2 *mv = (int2 *)c.dalloc(2 * BMAX * sizeof(int2));
    double2 *W = (double2 *)c.dalloc(4 * BMAX * BMAX * sizeof(double2));
    double2 *R1 = W + BMAX * BMAX, *R2 = R1 + BMAX * BMAX, *Rp = R2 + BMAX * BMAX;
    double2 *S = (double2 *)c.dalloc((size_t)ell * BMAX * sizeof(double2));
    // split-K partial products: 8 slices of the ell x 64 panel products, 4 of
    // the 64-row R_12 block
    const int64_t wkcap = std::max<int64_t>((int64_t)ell * 8, n * 4) * BMAX;
    double2 *Wk = (double2 *)c.dalloc((size_t)wkcap * sizeof(double2));
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0}, mone = {-1.0, 0.0};
    // Y = Omega A
    hipLaunchKernelGGL(gauss_fill_kernel, dim3(ceil_div((int64_t)YR * ell, 256)), dim3(256), 0, c.stream, Om, YR,
                       (int64_t)ell, seed + 0x5851F42D4C957F2DULL, (int64_t)1, (int64_t)YR, 0);
    AXS_HIP(hipGetLastError());
    AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, YR, (rocblas_int)n, ell, &one, zc(Om),
                           YR, zc(A), ell, &zero, zc(Y), YR));
    std::vector<double2> hd(BMAX);
    double d0 = 0.0;
    int k = -1;
    for (int j0 = 0; j0 < kmax && k < 0;) {
        int b = std::min(BMAX, kmax - j0);
        const int64_t nrem = n - j0;
        // b pivots by pivoted Gram-Schmidt over a copy of the trailing sketch, chosen on the device
        AXS_HIP(hipMemcpyAsync(G, Y + (int64_t)j0 * YR, (size_t)YR * nrem * sizeof(double2),
                               hipMemcpyDeviceToDevice, c.stream));
        const unsigned gblk = (unsigned)ceil_div(nrem, (int64_t)4);
        hipLaunchKernelGGL(gcol_norms_kernel, dim3(gblk), dim3(256), 0, c.stream, G, YR, nrem, nrm, part_v,
                           part_i);
        hipLaunchKernelGGL(gcol_argmax_kernel, dim3(1), dim3(1024), 0, c.stream, part_v, part_i, (int)gblk, nrm, dpiv,
                           dnu2, 0);
        for (int t = 0; t + 1 < b; ++t) {
            hipLaunchKernelGGL(gcol_step_kernel, dim3(gblk), dim3(256), 0, c.stream, G, YR, nrem, dpiv, dnu2, t,
                               nrm, part_v, part_i);
            hipLaunchKernelGGL(gcol_argmax_kernel, dim3(1), dim3(1024), 0, c.stream, part_v, part_i, (int)gblk, nrm,
                               dpiv, dnu2, t + 1);
        }
        AXS_HIP(hipGetLastError());
        std::vector<int> loc(b);
        AXS_HIP(hipMemcpyAsync(loc.data(), dpiv, b * sizeof(int), hipMemcpyDeviceToHost, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        {
            std::vector<char> seen(nrem, 0);
            for (int t = 0; t < b; ++t) {
                AXS_REQUIRE(loc[t] >= 0 && loc[t] < nrem && !seen[loc[t]], AXS_ENONFINITE, "non-finite proxy sketch");
                seen[loc[t]] = 1;
            }
        }
        // move the chosen columns to positions j0 .. j0 + b - 1 (A and Rm: all
        // ell rows; Y: its YR rows)
        std::vector<int2> moves;
        std::vector<char> taken(b, 0);
        for (int t = 0; t < b; ++t)
            if (loc[t] < b) taken[loc[t]] = 1;
        std::vector<int> free_src;   // positions < b whose column is not chosen
        for (int t = 0; t < b; ++t)
            if (!taken[t]) free_src.push_back(t);
        size_t fs = 0;
        for (int t = 0; t < b; ++t) {
            if (loc[t] == t) continue;
            moves.push_back(make_int2(j0 + t, j0 + loc[t]));
            if (loc[t] >= b) moves.push_back(make_int2(j0 + loc[t], j0 + free_src[fs++]));
        }
        if (!moves.empty()) {
            std::vector<int> np(perm);
            for (const int2 &m2 : moves) np[m2.x] = perm[m2.y];
            perm.swap(np);
            AXS_HIP(hipMemcpyAsync(mv, moves.data(), moves.size() * sizeof(int2), hipMemcpyHostToDevice, c.stream));
            const int cnt = (int)moves.size();
            for (double2 *M : {A, Rm})
                for (int ph = 0; ph < 2; ++ph)
                    hipLaunchKernelGGL(move_cols_kernel, dim3(ceil_div((int64_t)ell * cnt, 256)), dim3(256), 0,
                                       c.stream, M, (int64_t)ell, ell, mv, cnt, tmp, ph);
            for (int ph = 0; ph < 2; ++ph)
                hipLaunchKernelGGL(move_cols_kernel, dim3(ceil_div((int64_t)YR * cnt, 256)), dim3(256), 0, c.stream,
                                   Y, (int64_t)YR, YR, mv, cnt, tmp, ph);
            AXS_HIP(hipGetLastError());
            AXS_HIP(hipStreamSynchronize(c.stream));   // moves is pageable host memory
        }
        // the panel Pn = A[:, j0:j0+b], kept raw (with its R rows 0..j0-1) so
        // that a panel shortened by the Cholesky can give its other columns
        // back to the trailing matrix unprojected
        double2 *Pn = A + (int64_t)j0 * ell;
        double2 *Rcol = Rm + (int64_t)j0 * ell;     // rows 0..j0-1 of the panel's columns
        AXS_HIP(hipMemcpy2DAsync(rawA, ell * sizeof(double2), Pn, ell * sizeof(double2), ell * sizeof(double2), b,
                                 hipMemcpyDeviceToDevice, c.stream));
        if (j0 > 0)
            AXS_HIP(hipMemcpy2DAsync(rawR, ell * sizeof(double2), Rcol, ell * sizeof(double2),
                                     (size_t)j0 * sizeof(double2), b, hipMemcpyDeviceToDevice, c.stream));
        for (int pass = 0; pass < 2;) {
            if (pass == 0 && j0 > 0) {
                // project against Q = A[:, 0:j0]: first with the known R rows
                // (Q^H of the raw columns), then recomputed (reorthogonalisation)
                gemm_splitk(c, h, rocblas_operation_none, ell, b, j0, -1.0, A, ell, Rcol, ell, 1.0, Pn, ell, Wk,
                            wkcap);
                gemm_splitk(c, h, rocblas_operation_conjugate_transpose, j0, b, ell, 1.0, A, ell, Pn, ell, 0.0, S,
                            j0, Wk, wkcap);
                gemm_splitk(c, h, rocblas_operation_none, ell, b, j0, -1.0, A, ell, S, j0, 1.0, Pn, ell, Wk, wkcap);
                hipLaunchKernelGGL(cadd_kernel, dim3(ceil_div((int64_t)j0 * b, 256)), dim3(256), 0, c.stream, Rcol,
                                   S, j0, (int64_t)b, (int64_t)ell, (int64_t)j0);
                AXS_HIP(hipGetLastError());
            }
            // CholeskyQR2 of the projected panel: Pn = Q Rp, Q in place of Pn
            double2 *Rk = pass == 0 ? R1 : R2;
            gemm_splitk(c, h, rocblas_operation_conjugate_transpose, b, b, ell, 1.0, Pn, ell, Pn, ell, 0.0, W, b, Wk,
                        wkcap);
            hipLaunchKernelGGL(chol_small_kernel, dim3(1), dim3(64), 0, c.stream, W, b, Rk, dinfo);
            AXS_HIP(hipGetLastError());
            int info = 0;
            AXS_HIP(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));
            if (info < b) {
                if (info == 0) {   // no rank left in the trailing matrix
                    AXS_REQUIRE(j0 > 0, AXS_ENONFINITE, "non-finite or zero proxy sketch");
                    k = j0;
                    break;
                }
                // give every panel column back raw, then retry with the first info
                AXS_HIP(hipMemcpy2DAsync(Pn, ell * sizeof(double2), rawA, ell * sizeof(double2),
                                         ell * sizeof(double2), b, hipMemcpyDeviceToDevice, c.stream));
                if (j0 > 0)
                    AXS_HIP(hipMemcpy2DAsync(Rcol, ell * sizeof(double2), rawR, ell * sizeof(double2),
                                             (size_t)j0 * sizeof(double2), b, hipMemcpyDeviceToDevice, c.stream));
                b = info;
                pass = 0;
                continue;
            }
            AXS_BLAS(rocblas_ztrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                   rocblas_diagonal_non_unit, ell, b, &one, zc(Rk), b, zc(Pn), ell));
            ++pass;
        }
        if (k >= 0) break;
        // Rp = R2 R1 (upper triangular), into rows j0.. of Rm
        AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, b, b, b, &one, zc(R2), b, zc(R1), b,
                               &zero, zc(Rp), b));
        AXS_HIP(hipMemcpy2DAsync(Rm + j0 + (int64_t)j0 * ell, ell * sizeof(double2), Rp, b * sizeof(double2),
                                 b * sizeof(double2), b, hipMemcpyDeviceToDevice, c.stream));
        // rows j0..j0+b-1 of R_12 = Q_b^H A_t, and the sketch downdate
        const int64_t nt = nrem - b;
        if (nt > 0) {
            const int64_t jt = j0 + b;
            // one row of 64 x 64 tiles down an inner dimension of ell: split along
            // it so that each CU holds several tiles
            gemm_splitk(c, h, rocblas_operation_conjugate_transpose, b, (int)nt, ell, 1.0, Pn, ell, A + jt * ell, ell,
                        0.0, Rm + j0 + jt * ell, ell, Wk, wkcap, 1024);
            double2 *Yp = Y + (int64_t)j0 * YR;
            AXS_BLAS(rocblas_ztrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                   rocblas_diagonal_non_unit, YR, b, &one, zc(Rp), b, zc(Yp), YR));
            AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, YR, (rocblas_int)nt, b, &mone,
                                   zc(Yp), YR, zc(Rm + j0 + jt * ell), ell, &one, zc(Y + jt * YR), YR));
        }
        hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(BMAX), 0, c.stream, Rm, (int64_t)ell, j0, b, W);
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipMemcpyAsync(hd.data(), W, b * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
        AXS_HIP(hipStreamSynchronize(c.stream));
        for (int t = 0; t < b; ++t) {
            const double d = std::hypot(hd[t].x, hd[t].y);
            AXS_REQUIRE(std::isfinite(d), AXS_ENONFINITE, "non-finite proxy sketch");
            diag.push_back(d);
            if (j0 + t == 0) d0 = d;
            if (!(d > eps * d0)) {
                k = j0 + t;
                break;
            }
        }
        j0 += b;
    }
    if (k < 0) k = kmax;
    for (void *q : {(void *)Om, (void *)Y, (void *)G, (void *)nrm, (void *)part_v, (void *)part_i, (void *)dpiv,
                    (void *)dnu2, (void *)tmp,
                    (void *)rawA, (void *)rawR, (void *)mv, (void *)W, (void *)S, (void *)Wk})
        c.dfree(q);
    return k;
}

// The next sketch width after one that ran out of rows before |R_jj| fell
// below eps |R_00|: the decay of log |R_jj| over the second half of the pivots
// seen, extrapolated to eps |R_00|, with a margin of 25 % + 64; at least 1.5x
// and at most 8x the width tried (2x where the decay cannot be read).
static int64_t next_sketch_width(const std::vector<double> &diag, double eps, int ell) {
    const int64_t lo = (3 * (int64_t)ell + 1) / 2, hi = 8 * (int64_t)ell;
    const size_t m = diag.size();
    if (m < 32 || !(diag[0] > 0.0)) return 2 * (int64_t)ell;
    const size_t a = m / 2, b = m - 1;
    if (!(diag[a] > 0.0) || !(diag[b] > 0.0)) return 2 * (int64_t)ell;
    const double slope = (std::log(diag[b]) - std::log(diag[a])) / (double)(b - a);
    if (!(slope < 0.0)) return hi;
    const double need = (std::log(eps * diag[0]) - std::log(diag[b])) / slope;   // pivots still to go
    const double est = (double)b + std::max(need, 0.0);
    const int64_t want = (int64_t)(1.25 * est) + 64;
    return std::max(lo, std::min(hi, want));
}

// point ID of one shape: ascending skeleton nodes and X^T (device, k x n); the
// sketch starts max(256, ell0) rows wide and grows as next_sketch_width says
static void point_id(Ctx &c, const Shape &s, double R_p, double eps, int npx, uint64_t seed, int ell0,
                     std::vector<int> &nodes, double2 *&XT, int &ell_used) {
    rocblas_handle h = blas_of(c);
    const int NG = s.NG, M = s.M, NF = s.NF, nm = 2 * M + 1;
    const int64_t n = (int64_t)NG * NF;
    double2 *kin = nullptr, *kout = nullptr;
    double s_in = 0, s_out = 0;
    proxy_fields(c, s, R_p, npx, npx, kin, kout, s_in, s_out);
    const int Cp = 3 * npx;
    const int64_t C = (int64_t)(M + 1) * Cp, Cpm = (int64_t)nm * Cp;
    // conj(H_m) for m = 0..M, row-major NG x C (= column-major C x NG)
    double2 *Bc = (double2 *)c.dalloc((size_t)NG * C * sizeof(double2));
    hipLaunchKernelGGL(build_h_kernel, dim3(ceil_div((int64_t)NG * C, 256)), dim3(256), 0, c.stream, kin, kout, NG,
                       npx, 2 * npx, M, s_in, s_out, Bc);
    hipLaunchKernelGGL(conj_kernel, dim3(ceil_div((int64_t)NG * C, 256)), dim3(256), 0, c.stream, Bc,
                       (int64_t)NG * C);
    AXS_HIP(hipGetLastError());
    c.dfree(kin);
    c.dfree(kout);
    double2 *Es = upload(c, dft_matrix(M, NF, -1.0, 1.0, true));    // (2M+1) x NF: e^{-i m theta_l}
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    const int64_t cap = std::min<int64_t>(n, Cpm);
    int ell = (int)std::min<int64_t>(std::max(256, ell0), cap);
    double2 *Rm = nullptr;
    std::vector<int> perm;
    int k = 0;
    for (;;) {
        // Psi = Omega^* (ell x Cpm): entry (s, r) = conj(gauss(seed, s Cpm + r))
        double2 *Psi = (double2 *)c.dalloc((size_t)ell * Cpm * sizeof(double2));
        hipLaunchKernelGGL(gauss_fill_kernel, dim3(ceil_div((int64_t)ell * Cpm, 256)), dim3(256), 0, c.stream, Psi,
                           ell, Cpm, seed, Cpm, (int64_t)1, 1);
        AXS_HIP(hipGetLastError());
        // W_m = Psi_m conj(H_|m|)^T, stored as column (i (2M+1) + m + M) of W (ell x NG (2M+1))
        double2 *W = (double2 *)c.dalloc((size_t)ell * NG * nm * sizeof(double2));
        for (int m = -M; m <= M; ++m)
            AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, ell, NG, Cp, &one,
                                   zc(Psi + (int64_t)(m + M) * Cp * ell), ell, zc(Bc + (int64_t)std::abs(m) * Cp),
                                   (rocblas_int)C, &zero, zc(W + (int64_t)(m + M) * ell), ell * nm));
        c.dfree(Psi);
        // A[:, i NF + l] = sum_m W[:, i (2M+1) + m + M] e^{-i m theta_l}
        double2 *A = (double2 *)c.dalloc((size_t)ell * n * sizeof(double2));
        AXS_BLAS(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, ell, NF, nm, &one,
                                               zc(W), ell, (rocblas_stride)ell * nm, zc(Es), nm, 0, &zero, zc(A), ell,
                                               (rocblas_stride)ell * NF, NG));
        c.dfree(W);
        Rm = (double2 *)c.dalloc((size_t)ell * n * sizeof(double2));
        std::vector<double> diag;
        k = hqrrp(c, h, A, Rm, ell, n, eps, seed, perm, diag);
        c.dfree(A);
        if (k <= ell - 16 || ell == cap) break;
        c.dfree(Rm);
        ell = (int)std::min<int64_t>(next_sketch_width(diag, eps, ell), cap);
    }
    c.dfree(Es);
    c.dfree(Bc);
    AXS_REQUIRE(k >= 1, AXS_EINVAL, "the proxy matrix of a shape is zero");
    ell_used = ell;
    // T = R_11^{-1} R_12 in place of R_12
    if (n > k)
        AXS_BLAS(rocblas_ztrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                               rocblas_diagonal_non_unit, k, (rocblas_int)(n - k), &one, zc(Rm), ell,
                               zc(Rm + (int64_t)k * ell), ell));
    nodes.assign(perm.begin(), perm.begin() + k);
    std::sort(nodes.begin(), nodes.end());
    std::vector<int> colof(k);
    for (int t = 0; t < k; ++t)
        colof[t] = (int)(std::lower_bound(nodes.begin(), nodes.end(), perm[t]) - nodes.begin());
    int *d_perm = (int *)c.dalloc((n + k) * sizeof(int));
    AXS_HIP(hipMemcpy(d_perm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_perm + n, colof.data(), k * sizeof(int), hipMemcpyHostToDevice));
    XT = (double2 *)c.dalloc((size_t)k * n * sizeof(double2));
    hipLaunchKernelGGL(assemble_xt_kernel, dim3(ceil_div((int64_t)k * n, 256)), dim3(256), 0, c.stream, Rm,
                       (int64_t)ell, d_perm, d_perm + n, k, n, XT);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));
    c.dfree(d_perm);
    c.dfree(Rm);
}

// S_p = X^T A_pp^{-1} X (k x k, column-major) for one shape: the columns of X
// through the per-mode inverses (forward DFT over the azimuth, S_|m|, inverse
// DFT), all as GEMMs on X^T
static void point_sp(Ctx &c, const Shape &s, int k, const double2 *XT, double2 *&S64, float2 *&S32) {
    rocblas_handle h = blas_of(c);
    const int NG = s.NG, M = s.M, NF = s.NF, nm = 2 * M + 1;
    const int64_t n = (int64_t)NG * NF;
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    double2 *Ef = upload(c, dft_matrix(M, NF, -1.0, 1.0, false));          // NF x (2M+1)
    double2 *Ei = upload(c, dft_matrix(M, NF, 1.0, 1.0 / NF, true));       // (2M+1) x NF
    double2 *Xh = (double2 *)c.dalloc((size_t)k * NG * nm * sizeof(double2));
    AXS_BLAS(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, k, nm, NF, &one, zc(XT),
                                           k, (rocblas_stride)k * NF, zc(Ef), NF, 0, &zero, zc(Xh), k,
                                           (rocblas_stride)k * nm, NG));
    double2 *Yh = (double2 *)c.dalloc((size_t)k * NG * nm * sizeof(double2));
    // S_|m| is stored row-major, i.e. column-major S_|m|^T: Yh_m = Xh_m S_|m|^T
    for (int m = -M; m <= M; ++m)
        AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, k, NG, NG, &one,
                               zc(Xh + (int64_t)(m + M) * k), k * nm, zc((const double2 *)s.S64 + (int64_t)std::abs(m) * NG * NG),
                               NG, &zero, zc(Yh + (int64_t)(m + M) * k), k * nm));
    c.dfree(Xh);
    double2 *YT = (double2 *)c.dalloc((size_t)k * n * sizeof(double2));
    AXS_BLAS(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, k, NF, nm, &one, zc(Yh),
                                           k, (rocblas_stride)k * nm, zc(Ei), nm, 0, &zero, zc(YT), k,
                                           (rocblas_stride)k * NF, NG));
    c.dfree(Yh);
    S64 = (double2 *)c.dalloc((size_t)k * k * sizeof(double2));
    AXS_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_transpose, k, k, (rocblas_int)n, &one, zc(XT),
                           k, zc(YT), k, &zero, zc(S64), k));
    S32 = (float2 *)c.dalloc((size_t)k * k * sizeof(float2));
    hipLaunchKernelGGL(to_c64_kernel, dim3(ceil_div((int64_t)k * k, 256)), dim3(256), 0, c.stream, S64,
                       (int64_t)k * k, S32);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));
    c.dfree(YT);
    c.dfree(Ef);
    c.dfree(Ei);
}

void skeletonize_points(Ctx &c, double eps, double factor, int n_proxy, uint64_t seed) {
    AXS_REQUIRE(c.precomputed, AXS_ESTATE, "call axs_precompute_scattering first");
    AXS_REQUIRE(eps > 0 && eps < 1 && factor > 1, AXS_EINVAL, "need 0 < eps < 1 and proxy factor > 1");
    AXS_REQUIRE(n_proxy >= 0 && n_proxy <= 4096, AXS_EINVAL, "n_proxy must be in [0, 4096]");
    const size_t nsh = c.shapes.size(), nb = c.bodies.size();
    AXS_REQUIRE(nb >= 2, AXS_EINVAL, "skeletonization needs at least two bodies");
    std::vector<double> Rp(nsh, 1e300), rb(nsh, 0.0);
    for (size_t b = 0; b < nb; ++b) {
        const Body &B = c.bodies[b];
        double gap = 1e300;
        for (size_t q = 0; q < nb; ++q) {
            if (q == b) continue;
            const Body &Q = c.bodies[q];
            const double d = std::sqrt((B.centre[0] - Q.centre[0]) * (B.centre[0] - Q.centre[0]) +
                                       (B.centre[1] - Q.centre[1]) * (B.centre[1] - Q.centre[1]) +
                                       (B.centre[2] - Q.centre[2]) * (B.centre[2] - Q.centre[2]));
            gap = std::min(gap, d - Q.bound_radius);
        }
        Rp[B.shape] = std::min(Rp[B.shape], std::min(factor * B.bound_radius, gap));
        rb[B.shape] = std::max(rb[B.shape], B.bound_radius);
    }
    for (size_t k = 0; k < nsh; ++k)
        AXS_REQUIRE(Rp[k] >= 1.05 * rb[k], AXS_EINVAL,
                    "point skeletons need a proxy sphere of 1.05 x the bounding radius around every body");
    auto sk = std::make_unique<Skeleton>();
    sk->kind = 1;
    sk->pts = std::make_unique<PointSkel>();
    PointSkel &P = *sk->pts;
    P.k.resize(nsh);
    P.n.resize(nsh);
    P.ell.resize(nsh);
    P.R_p = Rp;
    P.nodes.resize(nsh);
    P.XT.assign(nsh, nullptr);
    P.S64.assign(nsh, nullptr);
    P.S32.assign(nsh, nullptr);
    try {
        // the first shape's sketch starts 256 wide; each later one at the width
        // the rank of the one before would have asked for (shapes of one
        // scene have similar ranks), which saves the narrower attempts
        int ell0 = 256;
        for (size_t k = 0; k < nsh; ++k) {
            const Shape &s = c.shapes[k];
            const int npx = n_proxy > 0 ? n_proxy : 40 + (int)std::ceil(1.25 * s.kappa * Rp[k]);
            point_id(c, s, Rp[k], eps, npx, seed, ell0, P.nodes[k], P.XT[k], P.ell[k]);
            P.k[k] = (int)P.nodes[k].size();
            ell0 = (int)(1.25 * P.k[k]) + 64;
            P.n[k] = s.NG * s.NF;
            point_sp(c, s, P.k[k], P.XT[k], P.S64[k], P.S32[k]);
            sk->rank.push_back(P.k[k]);
        }
    } catch (...) {
        for (auto *p : P.XT) c.dfree(p);
        for (auto *p : P.S64) c.dfree(p);
        for (auto *p : P.S32) c.dfree(p);
        throw;
    }
    // runs of consecutive bodies of one shape, skeleton offsets, node list
    std::vector<int64_t> gidx;
    int64_t off = 0;
    for (size_t b = 0; b < nb; ++b) {
        const Body &B = c.bodies[b];
        const int sh = B.shape;
        if (P.runs.empty() || P.runs.back().shape != sh ||
            P.runs.back().o0 + (int64_t)P.runs.back().nb * P.n[sh] != B.offset) {
            PointRun r{sh, (int)b, 0, P.k[sh], P.n[sh], B.offset, off};
            P.runs.push_back(r);
        }
        P.runs.back().nb += 1;
        for (int j : P.nodes[sh]) gidx.push_back(B.offset + j);
        off += P.k[sh];
    }
    const int64_t Ns = off;
    // the child context: the skeleton nodes of every body, point-order sum
    sk->child = std::make_unique<Ctx>();
    Ctx &ch = *sk->child;
    ch.device = c.device;
    ch.stream = c.stream;
    ch.alloc = c.alloc;
    ch.free_fn = c.free_fn;
    ch.user = c.user;
    ch.have_k = true;
    ch.kappa = c.kappa;
    ch.eta = c.eta;
    ch.gam_re = c.gam_re;
    ch.gam_im = c.gam_im;
    ch.N = Ns;
    off = 0;
    for (size_t b = 0; b < nb; ++b) {
        Body B = c.bodies[b];
        B.offset = off;
        B.n = P.k[B.shape];
        off += B.n;
        ch.bodies.push_back(B);
    }
    int64_t *d_idx = (int64_t *)ch.dalloc(Ns * sizeof(int64_t));
    AXS_HIP(hipMemcpy(d_idx, gidx.data(), Ns * sizeof(int64_t), hipMemcpyHostToDevice));
    ch.g64 = (double *)ch.dalloc(7 * Ns * sizeof(double));
    ch.g32 = (float *)ch.dalloc(6 * Ns * sizeof(float));
    hipLaunchKernelGGL(gather_geo_kernel, dim3(ceil_div(7 * Ns, 256)), dim3(256), 0, c.stream, c.g64, c.N, d_idx, Ns,
                       ch.g64, ch.g32);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));
    ch.dfree(d_idx);
    ch.sctab = c.sctab;            // the parent's table (it outlives the child)
    ch.scene_phase_ok = c.scene_phase_ok;   // the skeleton nodes are a subset of the parent's
    // no rings: the point order below 16 rhs; from 16 rhs the MFMA orders, with
    // the parent's body frames and bounds, the skeleton nodes' MFMA operands
    // gathered from the parent's and 32-node blocks of the skeleton bodies
    ch.no_rings = true;
    ch.near_phase_ok = c.near_phase_ok;
    ch.mf16_ok = c.mf16_ok;
    ch.mf16_gexp = c.mf16_gexp;
    ch.frame32 = c.frame32;
    ch.frame64 = c.frame64;
    {
        std::vector<int64_t> bo;
        std::vector<int32_t> bk(1, 0);
        for (const Body &B : ch.bodies) {
            bo.push_back(B.offset);
            bk.push_back(bk.back() + (int32_t)ceil_div(B.n, (int64_t)32));
        }
        bo.push_back(Ns);
        ch.nblk = bk.back();
        ch.body_off = (int64_t *)ch.dalloc(bo.size() * sizeof(int64_t));
        AXS_HIP(hipMemcpy(ch.body_off, bo.data(), bo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        ch.blk_off = (int32_t *)ch.dalloc(bk.size() * sizeof(int32_t));
        AXS_HIP(hipMemcpy(ch.blk_off, bk.data(), bk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (c.mf_src64) {
        int64_t *d_gi = (int64_t *)ch.dalloc(Ns * sizeof(int64_t));
        AXS_HIP(hipMemcpy(d_gi, gidx.data(), Ns * sizeof(int64_t), hipMemcpyHostToDevice));
        ch.mf_src64 = (double *)ch.dalloc(8 * Ns * sizeof(double));
        ch.mf_src = (float *)ch.dalloc(8 * Ns * sizeof(float));
        hipLaunchKernelGGL(gather_mf_kernel, dim3(ceil_div(8 * Ns, 256)), dim3(256), 0, c.stream, c.mf_src64, c.N,
                           d_gi, Ns, ch.mf_src64, ch.mf_src);
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipStreamSynchronize(c.stream));
        ch.dfree(d_gi);
    }
    ch.pop = sk->pts.get();
    ch.precomputed = true;
    {
        std::vector<BodyMatItem> sp, rs;
        for (size_t b = 0; b < nb; ++b) {
            const Body &B = c.bodies[b];
            const int sh = B.shape;
            const int64_t s0 = ch.bodies[b].offset;
            sp.push_back(BodyMatItem{P.S32[sh], P.S64[sh], s0, s0, P.k[sh], P.k[sh], 0, 0});
            rs.push_back(BodyMatItem{nullptr, P.XT[sh], B.offset, s0, P.k[sh], P.n[sh], 0, 0});
        }
        P.sp_items = upload_items(c, sp, P.n_sp);
        P.rs_items = upload_items(c, rs, P.n_rs);
    }
    sk->Ns = Ns;
    sk->eps = eps;
    release_skeleton(c);
    c.skel = std::move(sk);
}

// child of point skeletons: y = s + S (B~ s), B~ in `prec`, S_p in the same precision
// C = alpha op(A) B + beta C for every body of a run and every rhs, A shared.
// B holds a body's kk-vector per (body j, rhs c) at j bk + c bN, C its
// m-vector at j ck + c cN.  With at least as many rhs as bodies: one GEMM per
// body whose columns are the rhs (ld = the rhs stride); else one GEMM per rhs
// whose columns are the bodies.  Either way A is streamed min(nb, nrhs) times,
// not once per (body, rhs) column.
template <typename T, typename Gemm>
static void run_gemm(rocblas_handle h, Gemm gemm, rocblas_operation op, int m, int kk, int nb, int nrhs, const T *alpha,
                     const T *A, int lda, const T *B, int64_t bk, int64_t bN, const T *beta, T *C, int64_t ck,
                     int64_t cN) {
    if (nrhs >= nb)
        AXS_BLAS(gemm(h, op, rocblas_operation_none, m, nrhs, kk, alpha, A, lda, 0, B, (rocblas_int)bN,
                      (rocblas_stride)bk, beta, C, (rocblas_int)cN, (rocblas_stride)ck, nb));
    else
        AXS_BLAS(gemm(h, op, rocblas_operation_none, m, nb, kk, alpha, A, lda, 0, B, (rocblas_int)bk,
                      (rocblas_stride)bN, beta, C, (rocblas_int)ck, (rocblas_stride)cN, nrhs));
}

// out_b = alpha A_b in_b (+ out_b) for every body b of a work list and every
// rhs: one workgroup per 256 rows of a body's block and NR rhs, one row per
// thread, NR complex accumulators per thread.  The input rows of a 64-column
// chunk (NR rhs) are staged in LDS and read back as broadcasts; A is read
// once per (row, column) and rhs group, down its columns, so a wavefront's
// load covers 64 consecutive rows.  With one body per launch of a GEMM
// library the same product fills a few dozen workgroups; here every body of
// every shape is in one launch.  In FP32 (R = float) the complex64 copy of A
// is used and the input is rounded to FP32 as it is staged.
template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };
constexpr int BM_KC = 64;

template <typename R, int NR>
__global__ __launch_bounds__(256) void body_matvec_kernel(const BodyMatItem *__restrict__ items,
                                                          const double2 *__restrict__ in, int64_t inN, int nrhs,
                                                          double2 *__restrict__ out, int64_t outN, double alpha,
                                                          int accumulate) {
    using C = typename CplxOf<R>::T;
    __shared__ C sw[BM_KC * NR];
    const BodyMatItem it = items[blockIdx.x];
    const int c0 = blockIdx.y * NR;
    const int i = it.row0 + (int)threadIdx.x;
    const bool row_ok = i < it.m;
    const C *A = sizeof(R) == 4 ? (const C *)(const void *)it.A32 : (const C *)(const void *)it.A64;
    R ar[NR], ai[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) ar[q] = ai[q] = R(0);
    for (int j0 = 0; j0 < it.K; j0 += BM_KC) {
        const int kc = min(BM_KC, it.K - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < BM_KC * NR; t += 256) {
            const int j = t % BM_KC, q = t / BM_KC;
            C v;
            v.x = R(0);
            v.y = R(0);
            if (j < kc && c0 + q < nrhs) {
                const double2 x = in[(int64_t)(c0 + q) * inN + it.in0 + j0 + j];
                v.x = (R)x.x;
                v.y = (R)x.y;
            }
            sw[j * NR + q] = v;
        }
        __syncthreads();
        if (row_ok) {
            const C *col = A + (int64_t)j0 * it.m + i;
            int j = 0;
            for (; j + 8 <= kc; j += 8) {
                C a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = col[(int64_t)(j + u) * it.m];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const C x = sw[(j + u) * NR + q];
                        ar[q] = fma(a[u].x, x.x, fma(-a[u].y, x.y, ar[q]));
                        ai[q] = fma(a[u].x, x.y, fma(a[u].y, x.x, ai[q]));
                    }
            }
            for (; j < kc; ++j) {
                const C a = col[(int64_t)j * it.m];
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const C x = sw[j * NR + q];
                    ar[q] = fma(a.x, x.x, fma(-a.y, x.y, ar[q]));
                    ai[q] = fma(a.x, x.y, fma(a.y, x.x, ai[q]));
                }
            }
        }
    }
    if (!row_ok) return;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (c0 + q >= nrhs) break;
        double2 *o = out + (int64_t)(c0 + q) * outN + it.out0 + i;
        double2 v = accumulate ? *o : make_double2(0.0, 0.0);
        v.x += alpha * (double)ar[q];
        v.y += alpha * (double)ai[q];
        *o = v;
    }
}

template <typename R>
static void launch_body_matvec(Ctx &c, const BodyMatItem *items, int nitems, const double2 *in, int64_t inN,
                               int nrhs, double2 *out, int64_t outN, double alpha, bool accumulate) {
    if (nitems == 0) return;
    const int nr = nrhs >= 16 ? 16 : nrhs >= 8 ? 8 : nrhs >= 4 ? 4 : nrhs >= 2 ? 2 : 1;
    const dim3 grid(nitems, ceil_div(nrhs, nr));
    const int acc = accumulate ? 1 : 0;
    switch (nr) {
    case 16:
        hipLaunchKernelGGL((body_matvec_kernel<R, 16>), grid, dim3(256), 0, c.stream, items, in, inN, nrhs, out, outN,
                           alpha, acc);
        break;
    case 8:
        hipLaunchKernelGGL((body_matvec_kernel<R, 8>), grid, dim3(256), 0, c.stream, items, in, inN, nrhs, out, outN,
                           alpha, acc);
        break;
    case 4:
        hipLaunchKernelGGL((body_matvec_kernel<R, 4>), grid, dim3(256), 0, c.stream, items, in, inN, nrhs, out, outN,
                           alpha, acc);
        break;
    case 2:
        hipLaunchKernelGGL((body_matvec_kernel<R, 2>), grid, dim3(256), 0, c.stream, items, in, inN, nrhs, out, outN,
                           alpha, acc);
        break;
    default:
        hipLaunchKernelGGL((body_matvec_kernel<R, 1>), grid, dim3(256), 0, c.stream, items, in, inN, nrhs, out, outN,
                           alpha, acc);
    }
    AXS_HIP(hipGetLastError());
}

// work items for one product per body: blocks A32/A64 of m_b x K_b rows, in
// 256-row slices
static BodyMatItem *upload_items(Ctx &c, const std::vector<BodyMatItem> &bodies, int &count) {
    std::vector<BodyMatItem> v;
    for (const BodyMatItem &b : bodies)
        for (int r0 = 0; r0 < b.m; r0 += 256) {
            BodyMatItem t = b;
            t.row0 = r0;
            v.push_back(t);
        }
    count = (int)v.size();
    if (v.empty()) return nullptr;
    BodyMatItem *d = (BodyMatItem *)c.dalloc(v.size() * sizeof(BodyMatItem));
    AXS_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(BodyMatItem), hipMemcpyHostToDevice));
    return d;
}

void point_operator(Ctx &c, const void *sigma, void *y, int nrhs, int prec) {
    const PointSkel &P = *c.pop;
    const int64_t Ns = c.N, tot = Ns * nrhs;
    interbody_partials(c, sigma, nrhs, prec);
    double2 *w = (double2 *)c.scratch(WS_XR, tot * sizeof(double2));
    interbody_reduce_to_c128(c, w, nrhs, prec);
    if (y != sigma) AXS_HIP(hipMemcpyAsync(y, sigma, tot * sizeof(double2), hipMemcpyDeviceToDevice, c.stream));
    if (prec == AXS_FP64)
        launch_body_matvec<double>(c, P.sp_items, P.n_sp, w, Ns, nrhs, (double2 *)y, Ns, 1.0, true);
    else
        launch_body_matvec<float>(c, P.sp_items, P.n_sp, w, Ns, nrhs, (double2 *)y, Ns, 1.0, true);
}

// out = alpha X^T y per body (full [nrhs][N] -> skeleton [nrhs][Ns])
static void point_restrict(Ctx &c, const void *y, void *out, int nrhs, double alpha) {
    const PointSkel &P = *c.skel->pts;
    launch_body_matvec<double>(c, P.rs_items, P.n_rs, (const double2 *)y, c.N, nrhs, (double2 *)out, c.skel->Ns,
                               alpha, false);
}

// out = add + X w per body (skeleton -> full)
static void point_prolong(Ctx &c, const void *w, const void *add, void *out, int nrhs) {
    const PointSkel &P = *c.skel->pts;
    const int64_t N = c.N, Ns = c.skel->Ns;
    if (add)
        AXS_HIP(hipMemcpyAsync(out, add, (size_t)N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, c.stream));
    else
        AXS_HIP(hipMemsetAsync(out, 0, (size_t)N * nrhs * sizeof(double2), c.stream));
    rocblas_handle h = blas_of(c);
    const rocblas_double_complex one = {1.0, 0.0};
    for (const PointRun &r : P.runs)
        run_gemm(h, rocblas_zgemm_strided_batched, rocblas_operation_transpose, r.n, r.k, r.nb, nrhs, &one,
                 zc(P.XT[r.shape]), r.k, zc((const double2 *)w + r.s0), r.k, Ns, &one, zc((double2 *)out + r.o0), r.n,
                 N);
}

}  // namespace axs
