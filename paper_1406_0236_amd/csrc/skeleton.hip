// Skeletonization of the inter-body blocks (Sec. 5, eqs. ip0-ip6).
//
// Sec. 5 factors each off-diagonal block A_pq = U_p A~_pq V_q^* + R_pq with
// interpolative decompositions whose index sets make A~_pq = A_pq(I_p, I_q) a
// submatrix of B, then solves the smaller preconditioned system
//     s~ + S B~ s~ = -v~,   S_p = V_p^* A_pp^{-1} U_p,   v~_p = V_p^* A_pp^{-1} v_p,
// and lifts the result back with s_p = -A_pp^{-1} (v_p + U_p sum_q A~_pq s~_q).
//
// For bodies of revolution the skeletons here are whole rings (contour nodes
// with all their azimuthal nodes): U_p = X (x) I and V_p^* = X^T (x) I with one
// NG x k matrix X per shape acting on the contour index.  Then
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

#include <algorithm>
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

// row ID of one shape: skeleton rings (ascending) and X (device, NG x k)
static void ring_id(Ctx &c, const Shape &s, double R_p, double eps, std::vector<int> &rings, double2 *&X) {
    const int NG = s.NG, M = s.M, n_in = NG, n_o = 2 * NG;
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
    const double gr = s.kappa > 0 ? 0.0 : s.eta, gi = s.kappa > 0 ? s.eta : 0.0;
    // incoming: target contour node i, source proxy node j (its normal and weight)
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
    double2 *kin = (double2 *)c.dalloc((size_t)Pin * (M + 1) * sizeof(double2));
    modal_values(c, s.kappa, gr, gi, M, Nt, h, Pin, kin);
    // outgoing: target proxy node j on radii R_p, 1.25 R_p, source contour node i
    const int64_t Pout = (int64_t)n_o * NG;
    std::vector<double> g(7 * Pout);
    for (int rr = 0; rr < 2; ++rr) {
        proxy_rings(rr == 0 ? R_p : 1.25 * R_p, NG, pr, pz, pnr, pnz, pw);
        for (int j = 0; j < NG; ++j)
            for (int i = 0; i < NG; ++i) {
                const int64_t q = ((int64_t)(rr * NG + j)) * NG + i;
                g[q] = pr[j];
                g[Pout + q] = s.r[i];
                g[2 * Pout + q] = s.r[i] - pr[j];
                g[3 * Pout + q] = s.z[i] - pz[j];
                g[4 * Pout + q] = nr[i];
                g[5 * Pout + q] = nz[i];
                g[6 * Pout + q] = aw[i] * pw[j];
            }
    }
    double2 *kout = (double2 *)c.dalloc((size_t)Pout * (M + 1) * sizeof(double2));
    modal_values(c, s.kappa, gr, gi, M, Nt, g, Pout, kout);
    // H with each block scaled to unit Frobenius norm
    const double s_in = 1.0 / std::sqrt(sumsq(c, kin, Pin * (M + 1)));
    const double s_out = 1.0 / std::sqrt(sumsq(c, kout, Pout * (M + 1)));
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
    if (c.skel) {
        if (c.skel->X) c.dfree(c.skel->X);
        if (c.skel->desc) c.dfree(c.skel->desc);
    }
    c.skel = std::move(sk);
}

// restrict / prolong between the full and the skeleton vectors
void skel_restrict(Ctx &c, const void *y, void *out, int nrhs, double alpha) {
    const Skeleton &sk = *c.skel;
    const int64_t tot = sk.Ns * nrhs;
    hipLaunchKernelGGL(restrict_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, sk.desc,
                       (int)c.bodies.size(), sk.X, (const double2 *)y, c.N, sk.Ns, nrhs, alpha, (double2 *)out);
    AXS_HIP(hipGetLastError());
}

void skel_prolong(Ctx &c, const void *w, const void *add, void *out, int nrhs) {
    const Skeleton &sk = *c.skel;
    const int64_t tot = c.N * nrhs;
    hipLaunchKernelGGL(prolong_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, c.stream, sk.desc,
                       (int)c.bodies.size(), sk.X, (const double2 *)w, (const double2 *)add, c.N, sk.Ns, nrhs,
                       (double2 *)out);
    AXS_HIP(hipGetLastError());
}

}  // namespace axs
