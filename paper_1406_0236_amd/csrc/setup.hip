// Precomputation of the local scattering matrices, FP64 on the GPU (Sec. 3.2:
// "we can pre-compute and store the block diagonal matrix A~^{-1}").
//
// For one generating contour (NG nodes, p-point Gauss panels) and modes
// m = 0..M the modal Nystrom matrix is A~_m = 1/2 I + K_m with
//   far entries   K_m(i, j) = k^G_m(y_i, y_j) r_j |gamma'_j| w_j,
//   near entries  K_m(i, j) = int_{-1}^{1} k^G_m(y_i, y(s)) l_j(s) r(s) |gamma'(s)| ds
// on the target's own panel, its neighbours and any panel closer to y_i than
// that panel's arc length (the paper cites Kolm-Rokhlin corrected quadrature
// for this step; here it is product integration with a graded Gauss rule:
// geometric bisection towards the (near-)singular parameter, 46 levels of 10
// Gauss points per side, which resolves the logarithmic singularity).
// On a near panel the curve is the polynomial interpolant of the node
// positions and its derivative gives the normal and line element; on the
// target's own panel the displacement y(s) - y_i is formed from the Lagrange
// form with the exact factor (s - s_i), so n'.(y' - y) keeps full relative
// accuracy as y' -> y.
//
// The modal kernel k^G_m = (k^D_m + gamma k^S_m) / (4 pi) is evaluated exactly
// (gamma = i eta for kappa > 0; eta at kappa = 0, the Laplace equation of Sec. 6.1):
//   k^S_m = sum_l c_l q_{m-l} + i s_m,  c_l, s_m: Fourier coefficients of the
//   entire functions cos(kR(t)) and sin(kR)/R (sampled at Nt points),
//   q_m = 2 Q_{|m|-1/2}(chi) / sqrt(r r') with Q the toroidal harmonic
//   (AGM elliptic integrals, then the three-term recurrence: forward near
//   chi = 1, backward continued fraction otherwise);
//   k^D_m = normal derivative at the source of the same expression.
// Pipeline per batch of target rows:
//   gen_far / gen_near  -> evaluation points (source data + weight)
//   toroidal_kernel     -> q_mu, n.grad q_mu per point            (thread per point)
//   modal_kernel        -> k^G_m * weight per point, m = 0..M    (wavefront per point)
//   scatter / near_reduce -> entries of A~_m
// then 1/2 on the diagonal and S_m = A~_m^{-1} by Gauss-Jordan elimination
// with partial pivoting (one workgroup per mode).
#include <cmath>

#include "axs_internal.h"

namespace axs {

constexpr int NLEV = 46;       // graded levels per side
constexpr int NGL = 10;        // Gauss points per level
constexpr int PMAX = 16;       // max nodes per panel supported

struct Pts {
    double *rt, *rp, *dr, *dz, *nr, *nz, *wj;   // [P]
    double *lag;                                 // [P][p] (near points only)
};

struct NearDesc {
    int32_t i, P;
    double sstar;
};

// ---------------------------------------------------------------------------
// evaluation points
// ---------------------------------------------------------------------------
__global__ void gen_far_kernel(const int2 *__restrict__ pairs, int n, const double *__restrict__ r,
                               const double *__restrict__ z, const double *__restrict__ nr,
                               const double *__restrict__ nz, const double *__restrict__ aw, Pts pts,
                               int64_t base) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = pairs[idx].x, j = pairs[idx].y;
    const int64_t o = base + idx;
    pts.rt[o] = r[i];
    pts.rp[o] = r[j];
    pts.dr[o] = r[j] - r[i];
    pts.dz[o] = z[j] - z[i];
    pts.nr[o] = nr[j];
    pts.nz[o] = nz[j];
    pts.wj[o] = aw[j];
}

__global__ void gen_near_kernel(const NearDesc *__restrict__ desc, int npairs, int p,
                                const double *__restrict__ snode, const double *__restrict__ lden,
                                const double *__restrict__ glu, const double *__restrict__ glw,
                                const double *__restrict__ r, const double *__restrict__ z, Pts pts,
                                int64_t base) {
    const int per = 2 * NLEV * NGL;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)npairs * per) return;
    const int pair = (int)(idx / per);
    const int rem = (int)(idx - (int64_t)pair * per);
    const int side = rem / (NLEV * NGL);
    const int lev = (rem / NGL) % NLEV;
    const int kq = rem % NGL;
    const NearDesc d = desc[pair];
    const int64_t o = base + idx;
    const double sst = d.sstar;
    const double dir = side == 0 ? -1.0 : 1.0;
    const double Ls = side == 0 ? sst + 1.0 : 1.0 - sst;
    double* lag = pts.lag + o * p;
    bool ok = Ls > 1e-14;
    double off = 0, wq = 0;
    if (ok) {
        const double hi = Ls * ldexp(1.0, -lev);
        const double lo = (lev == NLEV - 1) ? 0.0 : 0.5 * hi;
        off = lo + (hi - lo) * 0.5 * (glu[kq] + 1.0);
        wq = glw[kq] * 0.5 * (hi - lo);
    }
    const double s = sst + dir * off;
    const int own = (d.i / p) == d.P;
    const int iloc = d.i - d.P * p;
    const double *rP = r + d.P * p, *zP = z + d.P * p;
    // Lagrange basis and its derivative at s; on the own panel the factor
    // (s - s_iloc) is the exact signed offset.
    double diff[PMAX];
    for (int k = 0; k < p; ++k) diff[k] = (own && k == iloc) ? dir * off : s - snode[k];
    double L[PMAX], D[PMAX];
    for (int j = 0; j < p; ++j) {
        double prod = lden[j];
        for (int k = 0; k < p; ++k)
            if (k != j) prod *= diff[k];
        L[j] = prod;
        double der = 0;
        for (int m = 0; m < p; ++m) {
            if (m == j) continue;
            double t = lden[j];
            for (int k = 0; k < p; ++k)
                if (k != j && k != m) t *= diff[k];
            der += t;
        }
        D[j] = der;
    }
    double rp = 0, zp = 0, rs = 0, zs = 0, dr = 0, dz = 0;
    for (int k = 0; k < p; ++k) {
        rp += L[k] * rP[k];
        zp += L[k] * zP[k];
        rs += D[k] * rP[k];
        zs += D[k] * zP[k];
    }
    if (own) {
        for (int k = 0; k < p; ++k) {
            if (k == iloc) continue;
            dr += L[k] * (rP[k] - r[d.i]);
            dz += L[k] * (zP[k] - z[d.i]);
        }
    } else {
        dr = rp - r[d.i];
        dz = zp - z[d.i];
    }
    const double sp = sqrt(rs * rs + zs * zs);
    ok = ok && rp > 1e-13 && (dr * dr + dz * dz) > 0.0;
    pts.rt[o] = r[d.i];
    pts.rp[o] = ok ? rp : -1.0;     // rp < 0 marks a point that contributes nothing
    pts.dr[o] = dr;
    pts.dz[o] = dz;
    pts.nr[o] = -zs / sp;
    pts.nz[o] = rs / sp;
    pts.wj[o] = ok ? wq * rp * sp : 0.0;
    for (int k = 0; k < p; ++k) lag[k] = L[k];
}

// ---------------------------------------------------------------------------
// toroidal harmonics: q_mu = 2 Q_{mu-1/2}(chi)/sqrt(r r') and its normal derivative
// ---------------------------------------------------------------------------
__global__ void toroidal_kernel(Pts pts, int64_t npts, int nmax, double *__restrict__ qv,
                                double *__restrict__ dqv) {
    int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= npts) return;
    const int nq = nmax + 1;
    double *q = qv + pt * nq, *dq = dqv + pt * nq;
    const double rp = pts.rp[pt];
    if (!(rp > 0.0)) {
        for (int mu = 0; mu < nq; ++mu) q[mu] = dq[mu] = 0.0;
        return;
    }
    const double rt = pts.rt[pt], dr = pts.dr[pt], dz = pts.dz[pt], nrp = pts.nr[pt], nzp = pts.nz[pt];
    const double rr = rt * rp;
    const double d0sq = dr * dr + dz * dz;
    const double chim1 = d0sq / (2.0 * rr);
    const double chi = 1.0 + chim1;
    const double pm = chim1 / (chi + 1.0);           // 1 - m, m = 2/(chi+1)
    // complete elliptic integrals K(m), E(m) by the arithmetic-geometric mean
    double a = 1.0, b = sqrt(pm), csum = 0.5 * (1.0 - pm), pw = 0.5;
    for (int it = 0; it < 64; ++it) {
        const double an = 0.5 * (a + b), cn = 0.5 * (a - b);
        b = sqrt(a * b);
        a = an;
        pw *= 2.0;
        csum += pw * cn * cn;
        if (fabs(cn) <= 1e-17 * a) break;
    }
    const double K = M_PI / (2.0 * a);
    const double E = K * (1.0 - csum);
    const double kk = sqrt(2.0 / (chi + 1.0));
    const double Q0 = kk * K;
    const double eta = chim1 < 1e-3 ? 2.0 * asinh(sqrt(0.5 * chim1)) : acosh(chi);
    q[0] = Q0;
    if (nq > 1) {
        if (!(2.0 * nq * eta > 2.0)) {       // forward recurrence (also taken for a NaN argument)
            double qa = Q0, qb = chi * kk * K - sqrt(2.0 * (chi + 1.0)) * E;
            q[1] = qb;
            for (int mu = 1; mu + 1 < nq; ++mu) {
                const double qc = (2.0 * mu * chi * qb - (mu - 0.5) * qa) / (mu + 0.5);
                q[mu + 1] = qc;
                qa = qb;
                qb = qc;
            }
        } else {
            // rho_mu = Q_{mu+1/2}/Q_{mu-1/2} by the backward recurrence
            // rho_{mu-1} = (mu - 1/2) / (2 mu chi - (mu + 1/2) rho_mu), started at e^{-eta}
            const int top = nq + (int)ceil(20.0 / eta) + 20;
            double rho = 1.0 / (chi + sqrt(chim1 * (chi + 1.0)));
            for (int mu = top; mu >= 1; --mu) {
                rho = (mu - 0.5) / (2.0 * mu * chi - (mu + 0.5) * rho);
                if (mu < nq) q[mu] = rho;            // slot mu holds rho_{mu-1}
            }
            for (int mu = 1; mu < nq; ++mu) q[mu] = q[mu - 1] * q[mu];
        }
    }
    const double c2m1 = chim1 * (chi + 1.0);
    const double srr = sqrt(rr);
    const double ndel = nrp * dr + nzp * dz;
    const double ndchi = ndel / rr - nrp * d0sq / (2.0 * rr * rp);
    const double q1 = nq > 1 ? q[1] : 0.0;   // Q_{-3/2} = Q_{1/2}
    double prev = q1;
    for (int mu = 0; mu < nq; ++mu) {
        const double Qm = q[mu];
        const double dQ = (mu - 0.5) * (chi * Qm - prev) / c2m1;
        prev = Qm;
        const double qq = 2.0 * Qm / srr;
        q[mu] = qq;
        dq[mu] = 2.0 * dQ * ndchi / srr - nrp * qq / (2.0 * rp);
    }
}

// ---------------------------------------------------------------------------
// modal kernel values per point: one wavefront per point
// ---------------------------------------------------------------------------
__device__ double tcos_series(double x) {
    // (x cos x - sin x) / x^3 = sum_{k>=1} (-1)^k 2k x^{2k-2} / (2k+1)!
    double x2 = x * x, term = 1.0, sum = 0.0;
    double fact = 6.0;  // (2k+1)! for k = 1
    for (int k = 1; k <= 11; ++k) {
        sum += ((k & 1) ? -1.0 : 1.0) * (2.0 * k) * term / fact;
        term *= x2;
        fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
    }
    return sum;
}

template <int WPB>
__global__ __launch_bounds__(64 * WPB) void modal_kernel(Pts pts, int64_t npts, int Nt, int M,
                                                         const double *__restrict__ qv,
                                                         const double *__restrict__ dqv, double kappa,
                                                         double gam_re, double gam_im,
                                                         double2 *__restrict__ kout) {
    extern __shared__ double sm[];
    const int Nh = Nt / 2 + 1, L = Nt / 2 - 1, nq = M + L + 1;
    const int per = 4 * Nh + 2 * (L + 1) + 2 * (M + 1) + 2 * nq;
    double *cosT = sm;                               // [Nt]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *base = sm + Nt + wave * per;
    double *Cs = base, *Ss = Cs + Nh, *Dc = Ss + Nh, *Ds = Dc + Nh;
    double *cl = Ds + Nh, *dcl = cl + (L + 1), *sm_ = dcl + (L + 1), *dsm = sm_ + (M + 1);
    double *ql = dsm + (M + 1), *dql = ql + nq;
    for (int j = threadIdx.x; j < Nt; j += 64 * WPB) cosT[j] = cospi(2.0 * j / Nt);
    const int64_t pt = (int64_t)blockIdx.x * WPB + wave;
    const bool inrange = pt < npts;
    const double rp = inrange ? pts.rp[pt] : -1.0;
    const bool active = rp > 0.0;       // rp <= 0 marks a point without contribution
    double rt = 0, dr = 0, dz = 0, nrp = 0, nzp = 0, wj = 0;
    if (active) {
        rt = pts.rt[pt];
        dr = pts.dr[pt];
        dz = pts.dz[pt];
        nrp = pts.nr[pt];
        nzp = pts.nz[pt];
        wj = pts.wj[pt];
    }
    const double d0sq = dr * dr + dz * dz, ndel = nrp * dr + nzp * dz;
    // samples t_k = 2 pi k / Nt, k = 0..Nt/2 (all factors are even in t)
    if (active) {
        for (int k = lane; k < Nh; k += 64) {
            const double sh = sinpi((double)k / Nt);
            const double s2 = sh * sh;                   // sin^2(t/2)
            const double R = sqrt(d0sq + 4.0 * rt * rp * s2);
            const double x = kappa * R;
            double sn, cs;
            sincos(x, &sn, &cs);
            const double sd = R > 0.0 ? sn / R : kappa;
            const double T = x > 0.2 ? (x * cs - sn) / (R * R * R) : kappa * kappa * kappa * tcos_series(x);
            const double g = ndel + 2.0 * nrp * rt * s2;
            Cs[k] = cs;
            Ss[k] = sd;
            Dc[k] = -kappa * sd * g;
            Ds[k] = T * g;
        }
        for (int mu = lane; mu < nq; mu += 64) {
            ql[mu] = qv[pt * nq + mu];
            dql[mu] = dqv[pt * nq + mu];
        }
    }
    __syncthreads();
    // cosine-series coefficients:  f_l = (1/Nt) [f_0 + (-1)^l f_{Nt/2} + 2 sum_{k=1}^{Nt/2-1} f_k cos(2 pi l k / Nt)]
    if (active) {
        const int Lc = L > M ? L : M;
        for (int l = lane; l <= Lc; l += 64) {
            const double sgn = (l & 1) ? -1.0 : 1.0;
            double a0 = Cs[0] + sgn * Cs[Nh - 1], a1 = Ss[0] + sgn * Ss[Nh - 1];
            double a2 = Dc[0] + sgn * Dc[Nh - 1], a3 = Ds[0] + sgn * Ds[Nh - 1];
            double b0 = 0, b1 = 0, b2 = 0, b3 = 0;
            int idx = 0;
            for (int k = 1; k < Nh - 1; ++k) {
                idx += l;
                if (idx >= Nt) idx -= Nt;
                const double cw = cosT[idx];
                b0 = fma(Cs[k], cw, b0);
                b1 = fma(Ss[k], cw, b1);
                b2 = fma(Dc[k], cw, b2);
                b3 = fma(Ds[k], cw, b3);
            }
            const double inv = 1.0 / Nt;
            if (l <= L) {
                cl[l] = (a0 + 2.0 * b0) * inv;
                dcl[l] = (a2 + 2.0 * b2) * inv;
            }
            if (l <= M) {
                sm_[l] = (a1 + 2.0 * b1) * inv * (2.0 * M_PI);
                dsm[l] = (a3 + 2.0 * b3) * inv * (2.0 * M_PI);
            }
        }
    }
    __syncthreads();
    if (!inrange) return;
    double2 *out = kout + pt * (M + 1);
    const double inv4pi = 0.25 / M_PI;
    for (int m = lane; m <= M; m += 64) {
        if (!active) {
            out[m] = make_double2(0.0, 0.0);
            continue;
        }
        double sr = 0.0, dr_ = 0.0;
        for (int l = -L; l <= L; ++l) {
            const int al = l < 0 ? -l : l;
            const int mm = m - l < 0 ? l - m : m - l;
            sr = fma(cl[al], ql[mm], sr);
            dr_ = fma(dcl[al], ql[mm], fma(cl[al], dql[mm], dr_));
        }
        const double si = sm_[m], di = dsm[m];
        // (kD + gamma kS) / (4 pi)
        const double re = (dr_ + gam_re * sr - gam_im * si) * inv4pi;
        const double im = (di + gam_re * si + gam_im * sr) * inv4pi;
        out[m] = make_double2(re * wj, im * wj);
    }
}

// ---------------------------------------------------------------------------
// assembly of A~_m
// ---------------------------------------------------------------------------
__global__ void scatter_far_kernel(const int2 *__restrict__ pairs, int n, int M, int NG,
                                   const double2 *__restrict__ kval, int64_t base, double2 *__restrict__ A) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * (M + 1)) return;
    const int pr = (int)(idx / (M + 1)), m = (int)(idx % (M + 1));
    const int i = pairs[pr].x, j = pairs[pr].y;
    A[((int64_t)m * NG + i) * NG + j] = kval[(base + pr) * (M + 1) + m];
}

__global__ void near_reduce_kernel(const NearDesc *__restrict__ desc, int M, int NG, int p,
                                   const double2 *__restrict__ kval, const double *__restrict__ lag,
                                   int64_t base, double2 *__restrict__ A) {
    const int pair = blockIdx.x;
    const NearDesc d = desc[pair];
    const int per = 2 * NLEV * NGL;
    const int64_t p0 = base + (int64_t)pair * per;
    for (int t = threadIdx.x; t < (M + 1) * p; t += blockDim.x) {
        const int m = t / p, j = t % p;
        double re = 0, im = 0;
        for (int q = 0; q < per; ++q) {
            const double2 v = kval[(p0 + q) * (M + 1) + m];
            const double l = lag[(p0 + q) * p + j];
            re = fma(v.x, l, re);
            im = fma(v.y, l, im);
        }
        A[((int64_t)m * NG + d.i) * NG + d.P * p + j] = make_double2(re, im);
    }
}

__global__ void add_half_identity_kernel(double2 *A, int M, int NG) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (M + 1) * NG) return;
    const int m = idx / NG, i = idx % NG;
    A[((int64_t)m * NG + i) * NG + i].x += 0.5;
}

// Gauss-Jordan inverse with partial pivoting (ties -> lowest row), one block
// per matrix; the matrices of every shape (all modes) in one launch.
struct GJItem {
    const double2 *A;   // NG x NG, row-major
    double2 *work;      // NG x 2 NG
    double2 *S;         // NG x NG, row-major: A^{-1}
    int NG, pad;
};
template <int BS>
__global__ __launch_bounds__(BS) void gauss_jordan_kernel(const GJItem *__restrict__ items) {
    const GJItem it = items[blockIdx.x];
    const int NG = it.NG;
    const int W = 2 * NG;
    const double2 *a = it.A;
    double2 *g = it.work;
    double2 *s = it.S;
    __shared__ double rmax[BS];
    __shared__ int ridx[BS];
    __shared__ double2 piv_inv;
    extern __shared__ double2 fac[];   // [NG]
    for (int64_t t = threadIdx.x; t < (int64_t)NG * W; t += BS) {
        const int r = (int)(t / W), c = (int)(t % W);
        g[t] = c < NG ? a[(int64_t)r * NG + c] : make_double2(c - NG == r ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < NG; ++k) {
        double best = -1.0;
        int bi = k;
        for (int r = k + threadIdx.x; r < NG; r += BS) {
            const double2 v = g[(int64_t)r * W + k];
            const double mag = fabs(v.x) + fabs(v.y) > 0 ? hypot(v.x, v.y) : 0.0;
            if (mag > best) {
                best = mag;
                bi = r;
            }
        }
        rmax[threadIdx.x] = best;
        ridx[threadIdx.x] = bi;
        __syncthreads();
        for (int o = BS / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double b2 = rmax[threadIdx.x + o];
                const int i2 = ridx[threadIdx.x + o];
                if (b2 > rmax[threadIdx.x] || (b2 == rmax[threadIdx.x] && i2 < ridx[threadIdx.x])) {
                    rmax[threadIdx.x] = b2;
                    ridx[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        const int pr = ridx[0];
        if (pr != k) {
            for (int c = k + threadIdx.x; c < W; c += BS) {
                const double2 t0 = g[(int64_t)k * W + c];
                g[(int64_t)k * W + c] = g[(int64_t)pr * W + c];
                g[(int64_t)pr * W + c] = t0;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double2 pv = g[(int64_t)k * W + k];
            const double den = pv.x * pv.x + pv.y * pv.y;
            piv_inv = make_double2(pv.x / den, -pv.y / den);
        }
        __syncthreads();
        const double2 pinv = piv_inv;
        for (int c = k + threadIdx.x; c < W; c += BS) {
            const double2 v = g[(int64_t)k * W + c];
            g[(int64_t)k * W + c] = make_double2(v.x * pinv.x - v.y * pinv.y, v.x * pinv.y + v.y * pinv.x);
        }
        for (int r = threadIdx.x; r < NG; r += BS) fac[r] = g[(int64_t)r * W + k];
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)NG * (W - k); t += BS) {
            const int r = (int)(t / (W - k)), c = k + (int)(t % (W - k));
            if (r == k) continue;
            const double2 f = fac[r], u = g[(int64_t)k * W + c];
            double2 v = g[(int64_t)r * W + c];
            v.x -= f.x * u.x - f.y * u.y;
            v.y -= f.x * u.y + f.y * u.x;
            g[(int64_t)r * W + c] = v;
        }
        __syncthreads();
    }
    for (int64_t t = threadIdx.x; t < (int64_t)NG * NG; t += BS) {
        const int r = (int)(t / NG), c = (int)(t % NG);
        s[t] = g[(int64_t)r * W + NG + c];
    }
}

// S (complex128 row-major [M+1][NG][NG]) -> planar column-major FP64 and FP32 copies
__global__ void split_planar_kernel(const double2 *__restrict__ S, int M, int NG, double *__restrict__ r64,
                                    double *__restrict__ i64, float *__restrict__ r32,
                                    float *__restrict__ i32) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)NG * NG;
    if (t >= (M + 1) * nn) return;
    const int64_t m = t / nn, e = t % nn;
    const int k = (int)(e / NG), i = (int)(e % NG);      // output (column-major): element (i, k) at k*NG + i
    const double2 v = S[m * nn + (int64_t)i * NG + k];
    r64[t] = v.x;
    i64[t] = v.y;
    if (r32) {
        r32[t] = (float)v.x;
        i32[t] = (float)v.y;
    }
}

// ---------------------------------------------------------------------------
// host: Gauss-Legendre rule by Newton's method on the three-term recurrence
// ---------------------------------------------------------------------------
void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w);
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) { gauss_legendre_rule(n, x, w); }
void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) {
                // final derivative at the converged root
                p0 = 1.0;
                p1 = t;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (t * p1 - p0) / (t * t - 1.0);
                break;
            }
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[n - 1 - i] = t;                    // ascending
        w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

void gauss_legendre_public(int n, std::vector<double> &x, std::vector<double> &w) { gauss_legendre(n, x, w); }

static double interp_at(const std::vector<double> &sn, const double *f, int p, double s) {
    double v = 0;
    for (int j = 0; j < p; ++j) {
        double l = 1.0;
        for (int k = 0; k < p; ++k)
            if (k != j) l *= (s - sn[k]) / (sn[j] - sn[k]);
        v += l * f[j];
    }
    return v;
}

static int modal_nt(const Shape &s) {
    double rmax = 1e-3;
    for (double v : s.r) rmax = std::max(rmax, v);
    double need = 4.0 * s.kappa * rmax + 64.0;
    int nt = 64;
    while (nt < need) nt += 64;
    return nt;
}

void precompute_shape(Ctx &c, Shape &s) {
    const int NG = s.NG, p = s.p, M = s.M, np_ = s.n_panels;
    AXS_REQUIRE(p <= PMAX, AXS_EINVAL, "at most 16 nodes per panel are supported");
    s.Nt = modal_nt(s);
    const int Nt = s.Nt, L = Nt / 2 - 1, nq = M + L + 1;

    std::vector<double> sn, sw, gu, gwq;
    gauss_legendre(p, sn, sw);
    gauss_legendre(NGL, gu, gwq);
    std::vector<double> lden(p);
    for (int j = 0; j < p; ++j) {
        double d = 1.0;
        for (int k = 0; k < p; ++k)
            if (k != j) d *= (sn[j] - sn[k]);
        lden[j] = 1.0 / d;
    }
    // node data
    std::vector<double> nr(NG), nz(NG), aw(NG), plen(np_, 0.0);
    for (int i = 0; i < NG; ++i) {
        const double sp = std::hypot(s.dr[i], s.dz[i]);
        nr[i] = -s.dz[i] / sp;
        nz[i] = s.dr[i] / sp;
        aw[i] = s.r[i] * sp * s.gw[i];
        plen[i / p] += sp * s.gw[i];
    }
    // near panels and split points per target (host geometry)
    std::vector<std::vector<std::pair<int, double>>> near(NG);
    std::vector<double> endr(2 * np_), endz(2 * np_);
    for (int P = 0; P < np_; ++P) {
        endr[2 * P] = interp_at(sn, &s.r[P * p], p, -1.0);
        endr[2 * P + 1] = interp_at(sn, &s.r[P * p], p, 1.0);
        endz[2 * P] = interp_at(sn, &s.z[P * p], p, -1.0);
        endz[2 * P + 1] = interp_at(sn, &s.z[P * p], p, 1.0);
    }
    for (int i = 0; i < NG; ++i) {
        const int own = i / p;
        for (int P = 0; P < np_; ++P) {
            double best = 1e300, bs = 0;
            auto consider = [&](double rr, double zz, double sv) {
                double d = std::hypot(rr - s.r[i], zz - s.z[i]);
                if (d < best) {
                    best = d;
                    bs = sv;
                }
            };
            consider(endr[2 * P], endz[2 * P], -1.0);
            for (int k = 0; k < p; ++k) consider(s.r[P * p + k], s.z[P * p + k], sn[k]);
            consider(endr[2 * P + 1], endz[2 * P + 1], 1.0);
            const bool is_near = std::abs(P - own) <= 1 || best < plen[P];
            if (!is_near) continue;
            const double sst = P == own ? sn[i - own * p] : bs;
            near[i].push_back({P, sst});
        }
    }
    // device constants
    double *d_sn = (double *)c.dalloc(p * sizeof(double));
    double *d_lden = (double *)c.dalloc(p * sizeof(double));
    double *d_gu = (double *)c.dalloc(NGL * sizeof(double));
    double *d_gw = (double *)c.dalloc(NGL * sizeof(double));
    double *d_r = (double *)c.dalloc(NG * sizeof(double));
    double *d_z = (double *)c.dalloc(NG * sizeof(double));
    double *d_nr = (double *)c.dalloc(NG * sizeof(double));
    double *d_nz = (double *)c.dalloc(NG * sizeof(double));
    double *d_aw = (double *)c.dalloc(NG * sizeof(double));
    AXS_HIP(hipMemcpy(d_sn, sn.data(), p * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_lden, lden.data(), p * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_gu, gu.data(), NGL * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_gw, gwq.data(), NGL * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_r, s.r.data(), NG * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_z, s.z.data(), NG * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_nr, nr.data(), NG * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_nz, nz.data(), NG * sizeof(double), hipMemcpyHostToDevice));
    AXS_HIP(hipMemcpy(d_aw, aw.data(), NG * sizeof(double), hipMemcpyHostToDevice));

    const int64_t nmat = (int64_t)(M + 1) * NG * NG;
    double2 *A = (double2 *)c.dalloc(nmat * sizeof(double2));
    AXS_HIP(hipMemsetAsync(A, 0, nmat * sizeof(double2), c.stream));
    s.A64 = (double *)A;

    // batches of target rows, bounded number of evaluation points
    const int per_near = 2 * NLEV * NGL;
    const int64_t max_pts = 1 << 19;
    int i0 = 0;
    while (i0 < NG) {
        int i1 = i0;
        int64_t npts = 0;
        while (i1 < NG) {
            int64_t add = (NG - (int64_t)near[i1].size() * p) + (int64_t)near[i1].size() * per_near;
            if (i1 > i0 && npts + add > max_pts) break;
            npts += add;
            ++i1;
        }
        std::vector<int2> far;
        std::vector<NearDesc> nd;
        for (int i = i0; i < i1; ++i) {
            std::vector<char> isnear(np_, 0);
            for (auto &pr : near[i]) {
                isnear[pr.first] = 1;
                nd.push_back(NearDesc{i, pr.first, pr.second});
            }
            for (int j = 0; j < NG; ++j)
                if (!isnear[j / p]) far.push_back(make_int2(i, j));
        }
        const int64_t nfar = far.size(), nnear = (int64_t)nd.size() * per_near;
        const int64_t P = nfar + nnear;
        // point storage
        double *pbuf = (double *)c.scratch(WS_MISC, (size_t)P * (7 + p) * sizeof(double));
        Pts pts{pbuf, pbuf + P, pbuf + 2 * P, pbuf + 3 * P, pbuf + 4 * P, pbuf + 5 * P, pbuf + 6 * P, pbuf + 7 * P};
        double *qv = (double *)c.scratch(WS_TMP, (size_t)P * nq * sizeof(double));
        double *dqv = (double *)c.scratch(WS_TMP2, (size_t)P * nq * sizeof(double));
        double2 *kv = (double2 *)c.scratch(WS_TMP3, (size_t)P * (M + 1) * sizeof(double2));
        int2 *d_far = nullptr;
        NearDesc *d_nd = nullptr;
        if (nfar) {
            d_far = (int2 *)c.scratch(WS_RED, nfar * sizeof(int2));
            AXS_HIP(hipMemcpy(d_far, far.data(), nfar * sizeof(int2), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(gen_far_kernel, dim3(ceil_div(nfar, 256)), dim3(256), 0, c.stream, d_far,
                               (int)nfar, d_r, d_z, d_nr, d_nz, d_aw, pts, (int64_t)0);
            AXS_HIP(hipGetLastError());
        }
        if (nnear) {
            d_nd = (NearDesc *)c.scratch(WS_GEMM, nd.size() * sizeof(NearDesc));
            AXS_HIP(hipMemcpy(d_nd, nd.data(), nd.size() * sizeof(NearDesc), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(gen_near_kernel, dim3(ceil_div(nnear, 128)), dim3(128), 0, c.stream, d_nd,
                               (int)nd.size(), p, d_sn, d_lden, d_gu, d_gw, d_r, d_z, pts, nfar);
            AXS_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(toroidal_kernel, dim3(ceil_div(P, 64)), dim3(64), 0, c.stream, pts, P, nq - 1, qv,
                           dqv);
        AXS_HIP(hipGetLastError());
        constexpr int WPB = 4;
        const int per = 4 * (Nt / 2 + 1) + 2 * (L + 1) + 2 * (M + 1) + 2 * nq;
        const size_t shm = (Nt + WPB * per) * sizeof(double);
        AXS_REQUIRE(shm <= 160 * 1024, AXS_EINVAL, "mode count or wavenumber too large for the modal kernel");
        hipLaunchKernelGGL(modal_kernel<WPB>, dim3(ceil_div(P, WPB)), dim3(64 * WPB), shm, c.stream, pts, P, Nt,
                           M, qv, dqv, s.kappa, s.kappa > 0 ? 0.0 : s.eta, s.kappa > 0 ? s.eta : 0.0, kv);
        AXS_HIP(hipGetLastError());
        if (nfar) {
            hipLaunchKernelGGL(scatter_far_kernel, dim3(ceil_div(nfar * (M + 1), 256)), dim3(256), 0, c.stream,
                               d_far, (int)nfar, M, NG, kv, (int64_t)0, A);
            AXS_HIP(hipGetLastError());
        }
        if (nnear) {
            hipLaunchKernelGGL(near_reduce_kernel, dim3(nd.size()), dim3(256), 0, c.stream, d_nd, M, NG, p, kv,
                               pts.lag, nfar, A);
            AXS_HIP(hipGetLastError());
        }
        AXS_HIP(hipStreamSynchronize(c.stream));
        i0 = i1;
    }
    hipLaunchKernelGGL(add_half_identity_kernel, dim3(ceil_div((M + 1) * NG, 256)), dim3(256), 0, c.stream, A,
                       M, NG);
    AXS_HIP(hipGetLastError());
    AXS_HIP(hipStreamSynchronize(c.stream));   // the inverses follow for all shapes at once
    for (void *ptr : {(void *)d_sn, (void *)d_lden, (void *)d_gu, (void *)d_gw, (void *)d_r, (void *)d_z,
                      (void *)d_nr, (void *)d_nz, (void *)d_aw})
        c.dfree(ptr);
}

// S_m = A~_m^{-1} for every shape and mode: one Gauss-Jordan launch over all
// the matrices (per shape only M + 1 workgroups would run), in groups whose
// work arrays (NG x 2 NG per matrix) stay within 4 GiB
void invert_shapes(Ctx &c) {
    constexpr size_t WORK_CAP = (size_t)4 << 30;
    size_t k = 0;
    while (k < c.shapes.size()) {
        size_t k1 = k, bytes = 0;
        int maxNG = 0;
        while (k1 < c.shapes.size()) {
            const Shape &s = c.shapes[k1];
            const size_t b = (size_t)(s.M + 1) * s.NG * 2 * s.NG * sizeof(double2);
            if (k1 > k && bytes + b > WORK_CAP) break;
            bytes += b;
            maxNG = std::max(maxNG, s.NG);
            ++k1;
        }
        double2 *work = (double2 *)c.dalloc(bytes);
        std::vector<GJItem> items;
        size_t off = 0;
        for (size_t q = k; q < k1; ++q) {
            Shape &s = c.shapes[q];
            const int64_t nn = (int64_t)s.NG * s.NG;
            double2 *S = (double2 *)c.dalloc((size_t)(s.M + 1) * nn * sizeof(double2));
            s.S64 = (double *)S;
            for (int m = 0; m <= s.M; ++m) {
                items.push_back(GJItem{(const double2 *)s.A64 + m * nn, work + off, S + m * nn, s.NG, 0});
                off += (size_t)2 * nn;
            }
        }
        GJItem *d_items = (GJItem *)c.dalloc(items.size() * sizeof(GJItem));
        AXS_HIP(hipMemcpy(d_items, items.data(), items.size() * sizeof(GJItem), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(gauss_jordan_kernel<256>, dim3((unsigned)items.size()), dim3(256),
                           maxNG * sizeof(double2), c.stream, d_items);
        AXS_HIP(hipGetLastError());
        AXS_HIP(hipStreamSynchronize(c.stream));
        c.dfree(d_items);
        c.dfree(work);
        k = k1;
    }
}

void modal_values(Ctx &c, double kappa, double gam_re, double gam_im, int M, int Nt,
                  const std::vector<double> &h, int64_t P, double2 *kout) {
    const int L = Nt / 2 - 1, nq = M + L + 1;
    double *pbuf = (double *)c.scratch(WS_MISC, (size_t)P * 7 * sizeof(double));
    AXS_HIP(hipMemcpy(pbuf, h.data(), (size_t)P * 7 * sizeof(double), hipMemcpyHostToDevice));
    Pts pts{pbuf, pbuf + P, pbuf + 2 * P, pbuf + 3 * P, pbuf + 4 * P, pbuf + 5 * P, pbuf + 6 * P, nullptr};
    double *qv = (double *)c.scratch(WS_TMP, (size_t)P * nq * sizeof(double));
    double *dqv = (double *)c.scratch(WS_TMP2, (size_t)P * nq * sizeof(double));
    hipLaunchKernelGGL(toroidal_kernel, dim3(ceil_div(P, 64)), dim3(64), 0, c.stream, pts, P, nq - 1, qv, dqv);
    AXS_HIP(hipGetLastError());
    constexpr int WPB = 4;
    const int per = 4 * (Nt / 2 + 1) + 2 * (L + 1) + 2 * (M + 1) + 2 * nq;
    const size_t shm = (Nt + WPB * per) * sizeof(double);
    AXS_REQUIRE(shm <= 160 * 1024, AXS_EINVAL, "mode count or wavenumber too large for the modal kernel");
    hipLaunchKernelGGL(modal_kernel<WPB>, dim3(ceil_div(P, WPB)), dim3(64 * WPB), shm, c.stream, pts, P, Nt, M,
                       qv, dqv, kappa, gam_re, gam_im, kout);
    AXS_HIP(hipGetLastError());
}

void split_planar(Ctx &c, Shape &s, const double *src, double *r64, double *i64, float *r32, float *i32) {
    const int64_t nmat = (int64_t)(s.M + 1) * s.NG * s.NG;
    hipLaunchKernelGGL(split_planar_kernel, dim3(ceil_div(nmat, 256)), dim3(256), 0, c.stream,
                       (const double2 *)src, s.M, s.NG, r64, i64, r32, i32);
    AXS_HIP(hipGetLastError());
}

}  // namespace axs
