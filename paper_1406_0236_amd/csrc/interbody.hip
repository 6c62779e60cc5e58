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
//   - FP32 path: the phase in revolutions, less whole revolutions per
//     (wavefront, source body), fed to the hardware sin/cos (which take
//     revolutions and reduce up to 256 of them), 1/R from v_rsq;
//   - FP64 path: the same structure with sin/cos from a 1024-entry LDS table
//     and short polynomials, and a Newton-refined hardware 1/sqrt.
// Two source orders ("variants") compute the same sum:
//   - points: each staged source carries x, y, z, n and q (with one
//     right-hand side: x and n scaled by powers of kappa / 2 pi, and the
//     six density terms of the ring order's one-rhs form);
//   - rings: a body's N_F nodes on one contour node form a ring; per target
//     and ring the constants p (target in the source body's frame), |p|^2 + r^2,
//     r p_x, r p_y, n_r p_x, n_r p_y are formed once, after which R^2 and n.d
//     cost two FMAs each per pair and the staged source carries only
//     (cos th_l, sin th_l, q).  Coordinates are scaled by kappa / 2 pi inside
//     those constants so that R * kappa / 2 pi (the phase in revolutions)
//     is R^2 * rsq(R^2) with no further multiply.
#include "axs_internal.h"

namespace axs {

template <typename R> struct C2T;
template <> struct C2T<float> { using T = float2; };
template <> struct C2T<double> { using T = double2; };

__device__ __forceinline__ void sincos_rev(float ph, float &s, float &c) {
    float f = __builtin_amdgcn_fractf(ph);   // [0, 1)
    s = __builtin_amdgcn_sinf(f);            // hardware sin/cos take revolutions
    c = __builtin_amdgcn_cosf(f);
}
// the same for |ph| <= 256 revolutions, the documented input range of the
// hardware sin/cos, which reduce the argument themselves
__device__ __forceinline__ void sincos_rev_near(float ph, float &s, float &c) {
    s = __builtin_amdgcn_sinf(ph);
    c = __builtin_amdgcn_cosf(ph);
}

// sin and cos of 2 pi t in FP64 for |t| < 2^40 revolutions, with a 1024-entry
// table of (cos, sin)(2 pi j / 1024) held in LDS:
//   y = t + 1.5 * 2^42 (one add; the sum has an ulp of 1/1024) rounds t to the
//   nearest multiple j / 1024, and the low word of y is j, which indexes the
//   table; y - 1.5 * 2^42 is j / 1024 exactly, and so is r = t - j / 1024, in
//   [-1/2048, 1/2048];
//   with x = 2 pi r, |x| <= h = pi / 1024: cos x to x^4 (Taylor; the first
//   dropped term below 1.2e-18) and sin x to x^3, with the x^5 term of its
//   Taylor series economised into x and x^3 by the Chebyshev polynomial T5 on
//   [-h, h] (x^5 ~ (5/4) h^2 x^3 - (5/16) h^4 x, error h^5 / 16 there), so the
//   truncation stays below h^5 / 1920 + h^7 / 5040 = 1.5e-16; both as
//   polynomials in r (coefficients times powers of 2 pi);
//   then the angle sum with the table entry.
constexpr int SC_N = 1024;
constexpr double SC_MAGIC = 6597069766656.0;   // 1.5 * 2^42
constexpr double SC_A = 6.283185307179586476925287;
constexpr double SC_H = SC_A / (2 * SC_N);
constexpr double SC_S1 = SC_A * (1.0 - SC_H * SC_H * SC_H * SC_H / 384.0),
                 SC_S3 = SC_A * SC_A * SC_A * (-1.0 / 6.0 + SC_H * SC_H / 96.0);
constexpr double SC_C2 = -SC_A * SC_A / 2.0, SC_C4 = SC_A * SC_A * SC_A * SC_A / 24.0;
__device__ __forceinline__ void sincos_rev_tab(double t, const double2 *tab, double &s, double &c) {
    const double y = t + SC_MAGIC;
    const double r = t - (y - SC_MAGIC);          // exact
    const double r2 = r * r;
    const double sx = r * fma(r2, SC_S3, SC_S1);
    const double cx = fma(r2, fma(r2, SC_C4, SC_C2), 1.0);
    const double2 e = tab[__double2loint(y) & (SC_N - 1)];   // (cos, sin)(2 pi j / 1024)
    s = fma(e.y, cx, e.x * sx);
    c = fma(e.x, cx, -e.y * sx);
}
// precision-generic entry points used by the kernels (the table is unused in FP32)
__device__ __forceinline__ void sincos_any(float ph, const double2 *, float &s, float &c) { sincos_rev(ph, s, c); }
__device__ __forceinline__ void sincos_any(double t, const double2 *tab, double &s, double &c) {
    sincos_rev_tab(t, tab, s, c);
}
// sin and cos of 2 pi R' from r2 = R'^2 and u = 1/R' (R' = R k / 2 pi, the
// phase in revolutions).  FP32: the hardware sin/cos of R' - n0, n0 the whole
// revolutions of the (wavefront, source body), which keeps the argument in
// their input range.  FP64: as sincos_rev_tab, with the product r2 u rounded
// to the table's 1/1024 steps inside one FMA, y = r2 u + 1.5 * 2^42, and the
// remainder r = r2 u - J, J = y - 1.5 * 2^42, formed by a second FMA, so the
// remainder carries the product's full precision (R' < 2^40 revolutions).
__device__ __forceinline__ void sincos_phase(float r2, float u, float n0, const double2 *, float &s, float &c) {
    sincos_rev_near(fma(r2, u, -n0), s, c);
}
__device__ __forceinline__ void sincos_phase(double r2, double u, double, const double2 *tab, double &s, double &c) {
    const double y = fma(r2, u, SC_MAGIC);
    const double r = fma(r2, u, -(y - SC_MAGIC));
    const double rr = r * r;
    const double sx = r * fma(rr, SC_S3, SC_S1);
    const double cx = fma(rr, fma(rr, SC_C4, SC_C2), 1.0);
    const double2 e = tab[__double2loint(y) & (SC_N - 1)];   // (cos, sin)(2 pi j / 1024)
    s = fma(e.y, cx, e.x * sx);
    c = fma(e.x, cx, -e.y * sx);
}
// copy the FP64 table to LDS (the kernels' first barrier publishes it)
template <typename R, int BS>
__device__ __forceinline__ void load_sctab(double2 *dst, const double2 *__restrict__ src) {
    if constexpr (sizeof(R) == 8)
        for (int i = threadIdx.x; i < SC_N; i += BS) dst[i] = src[i];
}

// floor(max(min over the wavefront of v, 0)), the same in every lane; in FP32
// moved to a scalar register so that the phase FMA reads two VGPRs, not three
__device__ __forceinline__ float wave_floor_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    v = floorf(fmaxf(v, 0.f));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_floor_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return floor(fmax(v, 0.0));
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// 1/sqrt(x) for finite x > 0: the hardware estimate y (relative error up to
// 5.2e-8 measured over 4M arguments; one Newton step leaves 4e-15) corrected
// to second order in e = 1 - x y^2: 1/sqrt(x) = y (1 - e)^(-1/2)
// = y (1 + e/2 + 3 e^2/8 + ...), the first dropped term 5 e^3/16 below 1e-21
__device__ __forceinline__ double rsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y, e * fma(e, 0.375, 0.5), y);
}

// LDS stride (in elements) of one staged source: x y z nx ny nz + NR complex q,
// or with one right-hand side (FOLD) the scaled position, the scaled normal
// and the six density terms of ring_term1; rounded up to 16 bytes so the
// compiler can use 128-bit LDS reads.
template <typename R, int NR, bool FOLD> struct SrcStride {
    static constexpr int raw = FOLD ? 12 : 6 + 2 * NR;
    static constexpr int per16 = 16 / sizeof(R);
    static constexpr int value = (raw + per16 - 1) / per16 * per16;
};

// One pair of the point order with one right-hand side, as ring_term1: r2 =
// R'^2 and nd = nd' in revolutions, qv the staged density terms.  near: every
// phase of the launch is under 255 revolutions, so the FP32 hardware sin/cos
// take it without the fraction step; FP64 uses the table form, good for any
// phase below 2^40 revolutions.
template <typename R>
__device__ __forceinline__ void point_term1(R r2, R nd, int near, const double2 *s_tab, const R *qv, R &ar,
                                            R &ai) {
    const R u = rsq(r2);
    R sn, cs_;
    if constexpr (sizeof(R) == 4) {
        const R ph = r2 * u;
        if (near)
            sincos_rev_near(ph, sn, cs_);
        else
            sincos_rev(ph, sn, cs_);
    } else {
        sincos_phase(r2, u, R(0), s_tab, sn, cs_);
    }
    const R w = nd * u;
    const R zr = fma(w, fma(u, qv[0], qv[2]), qv[4]);
    const R zi = fma(w, fma(u, qv[1], qv[3]), qv[5]);
    const R er = cs_ * u, ei = sn * u;
    ar = fma(er, zr, fma(-ei, zi, ar));
    ai = fma(er, zi, fma(ei, zr, ai));
}

template <typename R, int TPT, int NR, int BS, bool LAP>
__global__ __launch_bounds__(BS) void interbody_kernel(
    const IBWork *__restrict__ work, const R *__restrict__ geo, const typename C2T<R>::T *__restrict__ q,
    int64_t N, int nrhs, int c0, R kappa, R k2pi, R eta, const double2 *__restrict__ sctab, int near,
    typename C2T<R>::T *__restrict__ part) {
    using R2 = typename C2T<R>::T;
    // one right-hand side: positions scaled by k/2pi, so R'^2 = |d'|^2 and
    // nd' = (k/2pi)^2 n.d' (= n.d (k/2pi)^3) as in the ring order, and the
    // density terms staged with the source (ring_term1)
    constexpr bool FOLD = NR == 1 && !LAP;
    constexpr int ST = SrcStride<R, NR, FOLD>::value;
    __shared__ __align__(16) R tile[BS * ST];
    __shared__ double2 s_tab[sizeof(R) == 8 ? SC_N : 1];
    load_sctab<R, BS>(s_tab, sctab);

    const IBWork w = work[blockIdx.x];
    const int tid = threadIdx.x;
    const int cb = c0 + blockIdx.y * NR;   // first rhs of this block's group
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
        if constexpr (FOLD) {
            tx[k] *= k2pi;
            ty[k] *= k2pi;
            tz[k] *= k2pi;
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) ar[k][c] = ai[k][c] = R(0);
    }
    const R s2 = k2pi * k2pi, etap = eta * k2pi;

#pragma unroll 1
    for (int rng = 0; rng < 2; ++rng) {
        const int lo = rng == 0 ? w.s0 : w.s2;
        const int hi = rng == 0 ? w.s1 : w.s3;
#pragma unroll 1
        for (int base = lo; base < hi; base += BS) {
            const int cnt = min(BS, hi - base);
            __syncthreads();
            if (FOLD && tid < cnt) {
                const int64_t j = base + tid;
                R *d = tile + tid * ST;
                const R2 v = q[(int64_t)cb * N + j];
                const R tp = R(6.283185307179586476925287);
                d[0] = gx[j] * k2pi;
                d[1] = gy[j] * k2pi;
                d[2] = gz[j] * k2pi;
                d[3] = gnx[j] * s2;
                d[4] = gny[j] * s2;
                d[5] = gnz[j] * s2;
                d[6] = v.x, d[7] = v.y, d[8] = tp * v.y, d[9] = -tp * v.x, d[10] = -etap * v.y, d[11] = etap * v.x;
            } else if (!FOLD && tid < cnt) {
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
                    R2 v = q[(int64_t)(cb + c) * N + j];
                    d[6 + 2 * c] = v.x;
                    d[7 + 2 * c] = v.y;
                }
            }
            __syncthreads();
            if constexpr (FOLD) {
#pragma unroll 2
                for (int js = 0; js < cnt; ++js) {
                    const R *s = tile + js * ST;
                    const R sx = s[0], sy = s[1], sz = s[2], snx = s[3], sny = s[4], snz = s[5];
                    R qv[6];
#pragma unroll
                    for (int i = 0; i < 6; ++i) qv[i] = s[6 + i];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        const R dx = tx[k] - sx, dy = ty[k] - sy, dz = tz[k] - sz;
                        const R r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                        const R nd = fma(snx, dx, fma(sny, dy, snz * dz));
                        point_term1<R>(r2, nd, near, s_tab, qv, ar[k][0], ai[k][0]);
                    }
                }
                continue;
            }
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
                    const R nd = fma(snx, dx, fma(sny, dy, snz * dz));
                    if constexpr (LAP) {
                        // kappa = 0 (Sec. 6.1): 4 pi G = (n.d / R^2 + eta) / R, real
                        const R G = ri * fma(nd, ri * ri, eta);
#pragma unroll
                        for (int c = 0; c < NR; ++c) {
                            ar[k][c] = fma(G, qr[c], ar[k][c]);
                            ai[k][c] = fma(G, qi[c], ai[k][c]);
                        }
                        continue;
                    }
                    const R rr = r2 * ri;
                    R sn, cs;
                    sincos_any(rr * k2pi, s_tab, sn, cs);
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
                part[((int64_t)w.slot * nrhs + cb + c) * N + w.t0 + t] = v;
            }
        }
    }
}

// LDS stride of one staged mirror pair: cos, sin + NR complex q of azimuth l
// + NR complex q of azimuth N_F - l, 16-byte rounded.  With one right-hand
// side (FOLD) each node carries the six density terms of ring_term1 instead.
template <typename R, int NR, bool FOLD> struct RingStride {
    static constexpr int raw = FOLD ? 14 : 2 + 4 * NR;
    static constexpr int per16 = 16 / sizeof(R);
    static constexpr int value = (raw + per16 - 1) / per16 * per16;
};

// Ring variant.  Work items hold ring-id ranges; rings are numbered in node
// order.  A ring's azimuths are theta_l = 2 pi l / N_F, so in the source
// body's frame the nodes l and N_F - l are mirror images in y: same cos, sin
// of opposite sign.  The ring is staged as N_F/2 + 1 entries e, each holding
// node e and its mirror N_F - e (none for e = 0 and e = N_F/2), and R'^2,
// nd' of both come from one shared partial sum: 3 FMAs per pair instead of 4
// (an entry without a mirror carries zero density).  Sources are staged in
// LDS a tile of whole rings at a time (at most BS entries).
struct RingTabs {
    const int32_t *off, *nf, *body;   // [nrings]
    const int32_t *eoff;              // [nrings + 1]: first entry of each ring
    const int2 *pair;                 // [entries]: node of azimuth e, node of N_F - e (-1: none)
};

// One pair's contribution, accumulated into NR right-hand sides.
// r2 = R'^2, nd = nd' (R' = R k/2pi, nd' = n.d (k/2pi)^3), n0 whole revolutions.
template <typename R, int NR, bool LAP>
__device__ __forceinline__ void ring_term(R r2, R nd, R n0, R eta, R etap, const double2 *s_tab,
                                          const R *qr, const R *qi, R *ar, R *ai) {
    const R u = rsq(r2);   // 1 / R'
    if constexpr (LAP) {
        // kappa = 0 (scale factor 1): 4 pi G = (n.d / R^2 + eta) / R, real; the
        // caller passes nd = beta and eta + kap, since n.d / R^2 = kap + beta / R^2
        const R G = u * fma(nd, u * u, eta);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            ar[c] = fma(G, qr[c], ar[c]);
            ai[c] = fma(G, qi[c], ai[c]);
        }
    } else {
        const R twopi = R(6.283185307179586476925287);
        R sn, cs_;
        sincos_phase(r2, u, n0, s_tab, sn, cs_);   // phase R' = kR / 2pi revolutions
        const R t = nd * (u * u);
        const R P = t * u;                     // n.d / R^3
        const R Q = fma(-twopi, t, etap * u);  // eta / R - k n.d / R^2
        const R gr = fma(cs_, P, -sn * Q);
        const R gi = fma(cs_, Q, sn * P);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            ar[c] = fma(gr, qr[c], fma(-gi, qi[c], ar[c]));
            ai[c] = fma(gr, qi[c], fma(gi, qr[c], ai[c]));
        }
    }
}

// One pair's contribution to a single right-hand side.  With u = 1/R',
//   G q = e^{2 pi i R'} (P + iQ) q = e^{2 pi i R'} u z,
//   z = i eta' q + (nd' u) (u - 2 pi i) q,
// so the terms of q that do not depend on the pair are staged with the source,
// qv = (q_r, q_i, 2 pi q_i, -2 pi q_r, -eta' q_i, eta' q_r), and the pair
// costs 11 operations after sin/cos instead of 13.
template <typename R>
__device__ __forceinline__ void ring_term1(R r2, R nd, R n0, const double2 *s_tab, const R *qv, R &ar, R &ai) {
    const R u = rsq(r2);
    R sn, cs_;
    sincos_phase(r2, u, n0, s_tab, sn, cs_);   // phase R' (less whole revolutions in FP32)
    const R w = nd * u;
    const R zr = fma(w, fma(u, qv[0], qv[2]), qv[4]);
    const R zi = fma(w, fma(u, qv[1], qv[3]), qv[5]);
    const R er = cs_ * u, ei = sn * u;
    ar = fma(er, zr, fma(-ei, zi, ar));
    ai = fma(er, zi, fma(ei, zr, ai));
}

template <typename R, int TPT, int NR, int BS, bool LAP>
__global__ __launch_bounds__(BS) void interbody_ring_kernel(
    const IBWork *__restrict__ work, const R *__restrict__ geo, const R *__restrict__ cs,
    const typename C2T<R>::T *__restrict__ q, RingTabs rt, const R *__restrict__ rg, int nrings,
    const R *__restrict__ frame, int64_t N, int nrhs, int c0, R k2pi, R eta, const double2 *__restrict__ sctab,
    typename C2T<R>::T *__restrict__ part) {
    using R2 = typename C2T<R>::T;
    constexpr bool FOLD = NR == 1 && !LAP;
    constexpr int ST = RingStride<R, NR, FOLD>::value;
    constexpr int QB = FOLD ? 8 : 2 + 2 * NR;   // offset of the mirror's densities in an entry
    __shared__ __align__(16) R tile[BS * ST];
    __shared__ double2 s_tab[sizeof(R) == 8 ? SC_N : 1];
    load_sctab<R, BS>(s_tab, sctab);

    const IBWork w = work[blockIdx.x];
    const int tid = threadIdx.x;
    const int cb = c0 + blockIdx.y * NR;   // first rhs of this block's group
    const R *gx = geo, *gy = geo + N, *gz = geo + 2 * N;
    const R *gc = cs, *gs = cs + N;
    const R *rr_ = rg, *rz_ = rg + nrings, *rnr = rg + 2 * nrings, *rnz = rg + 3 * nrings;
    const R *rho_ = rg + 4 * nrings;
    const R s2 = k2pi * k2pi, c1 = k2pi * k2pi * k2pi;
    const R etap = eta * k2pi;

    R tx[TPT], ty[TPT], tz[TPT];
    R px[TPT], py[TPT], pz[TPT], n0 = R(0);
    R ar[TPT][NR], ai[TPT][NR];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        int t = tid + k * BS;
        int64_t gi = w.t0 + (t < w.tn ? t : 0);
        tx[k] = gx[gi];
        ty[k] = gy[gi];
        tz[k] = gz[gi];
        px[k] = py[k] = pz[k] = R(0);
#pragma unroll
        for (int c = 0; c < NR; ++c) ar[k][c] = ai[k][c] = R(0);
    }
    int prev_body = -1;

#pragma unroll 1
    for (int rng = 0; rng < 2; ++rng) {
        const int lo = rng == 0 ? w.s0 : w.s2;
        const int hi = rng == 0 ? w.s1 : w.s3;
        int r0 = lo;
#pragma unroll 1
        while (r0 < hi) {
            // a tile of whole rings [r0, r1) holding at most BS entries
            const int e0 = rt.eoff[r0];
            int r1 = r0;
            while (r1 < hi && rt.eoff[r1 + 1] - e0 <= BS) ++r1;
            if (r1 == r0) break;   // a ring wider than a tile: the host never launches this
            const int cnt = rt.eoff[r1] - e0;
            __syncthreads();
            if (tid < cnt) {
                const int2 pr = rt.pair[e0 + tid];
                R *d = tile + tid * ST;
                d[0] = gc[pr.x];
                d[1] = gs[pr.x];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const R2 v = q[(int64_t)(cb + c) * N + pr.x];
                    R2 m;
                    m.x = m.y = R(0);
                    if (pr.y >= 0) m = q[(int64_t)(cb + c) * N + pr.y];
                    if constexpr (FOLD) {
                        const R tp = R(6.283185307179586476925287);
                        d[2] = v.x, d[3] = v.y, d[4] = tp * v.y, d[5] = -tp * v.x, d[6] = -etap * v.y, d[7] = etap * v.x;
                        d[8] = m.x, d[9] = m.y, d[10] = tp * m.y, d[11] = -tp * m.x, d[12] = -etap * m.y,
                        d[13] = etap * m.x;
                    } else {
                        d[2 + 2 * c] = v.x;
                        d[3 + 2 * c] = v.y;
                        d[QB + 2 * c] = m.x;
                        d[QB + 1 + 2 * c] = m.y;
                    }
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int ring = r0; ring < r1; ++ring) {
                const int b = rt.body[ring];
                if (b != prev_body) {
                    // targets in the source body's frame: p = Rot^T (x - c).  Every
                    // source of the body is at R' >= (|p| - r_b)k/2pi, and the
                    // wavefront's targets lie in one body of radius r_t, so the
                    // phase less the whole revolutions n0 = floor(min (|p| - r_b)k/2pi)
                    // stays in [0, 2 (r_t + r_b) k/2pi + 1]
                    const R *f = frame + FRAME * b;
                    R m = R(1e30);
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        const R dx = tx[k] - f[0], dy = ty[k] - f[1], dz = tz[k] - f[2];
                        px[k] = fma(f[3], dx, fma(f[6], dy, f[9] * dz));
                        py[k] = fma(f[4], dx, fma(f[7], dy, f[10] * dz));
                        pz[k] = fma(f[5], dx, fma(f[8], dy, f[11] * dz));
                        const R pn = sqrt(fma(px[k], px[k], fma(py[k], py[k], pz[k] * pz[k])));
                        m = fmin(m, (pn - f[12]) * k2pi);
                    }
                    if constexpr (!LAP) n0 = wave_floor_min(m);
                    prev_body = b;
                }
                const R rj = rr_[ring], zj = rz_[ring], nrj = rnr[ring], nzj = rnz[ring];
                const int ne = rt.eoff[ring + 1] - rt.eoff[ring];
                const R *src = tile + (rt.eoff[ring] - e0) * ST;
                // per target: R'^2 = al + Ax cos + Ay sin and nd' = be + Bx cos + By sin
                // with (Bx, By) = kap (Ax, Ay), kap = -(k/2pi) n_r / (2 r) the same for
                // every target, so nd' = kap R'^2 + beta, beta = be - kap al (one FMA
                // per pair).  kap stays bounded for contours that meet the axis at
                // a right angle (n_r ~ r there).  The ring table holds
                // rho = -n_r / (2 r), 0 for a ring of radius 0 (zero area weight,
                // hence zero density).
                const R kap = rho_[ring] * k2pi;
                const R etak = eta + kap;   // zero frequency: n.d/R^2 + eta = beta/R^2 + (kap + eta)
                R al[TPT], Ax[TPT], Ay[TPT], beta[TPT];
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    const R pzp = pz[k] - zj;
                    al[k] = fma(px[k], px[k], fma(py[k], py[k], fma(pzp, pzp, rj * rj))) * s2;
                    Ax[k] = (R(-2) * s2 * rj) * px[k];
                    Ay[k] = (R(-2) * s2 * rj) * py[k];
                    beta[k] = fma(-kap, al[k], fma(nzj, pzp, -nrj * rj) * c1);
                }
                if constexpr (FOLD) {
                    // entry 0 is azimuth 0 (cos 1, sin 0), which has no mirror: one pair
                    {
                        const R cl = src[0];
                        R qv[6];
#pragma unroll
                        for (int i = 0; i < 6; ++i) qv[i] = src[2 + i];
#pragma unroll
                        for (int k = 0; k < TPT; ++k) {
                            const R ra = fma(Ax[k], cl, al[k]);
                            ring_term1<R>(ra, fma(kap, ra, beta[k]), n0, s_tab, qv, ar[k][0], ai[k][0]);
                        }
                    }
#pragma unroll 1
                    for (int l = 1; l < ne; ++l) {
                        const R *s = src + l * ST;
                        const R cl = s[0], sl = s[1];
                        R qv[6], mv[6];
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            qv[i] = s[2 + i];
                            mv[i] = s[8 + i];
                        }
#pragma unroll
                        for (int k = 0; k < TPT; ++k) {
                            const R br = fma(Ax[k], cl, al[k]);
                            const R ra = fma(Ay[k], sl, br), rb = fma(-Ay[k], sl, br);
                            ring_term1<R>(ra, fma(kap, ra, beta[k]), n0, s_tab, qv, ar[k][0], ai[k][0]);
                            ring_term1<R>(rb, fma(kap, rb, beta[k]), n0, s_tab, mv, ar[k][0], ai[k][0]);
                        }
                    }
                    continue;
                }
#pragma unroll 1
                for (int l = 0; l < ne; ++l) {
                    const R *s = src + l * ST;
                    const R cl = s[0], sl = s[1];
                    R qr[NR], qi[NR], mr[NR], mi[NR];
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        qr[c] = s[2 + 2 * c];
                        qi[c] = s[3 + 2 * c];
                        mr[c] = s[QB + 2 * c];
                        mi[c] = s[QB + 1 + 2 * c];
                    }
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        const R br = fma(Ax[k], cl, al[k]);
                        const R ra = fma(Ay[k], sl, br), rb = fma(-Ay[k], sl, br);
                        if constexpr (LAP) {
                            ring_term<R, NR, true>(ra, beta[k], n0, etak, etap, s_tab, qr, qi, ar[k], ai[k]);
                            ring_term<R, NR, true>(rb, beta[k], n0, etak, etap, s_tab, mr, mi, ar[k], ai[k]);
                        } else {
                            ring_term<R, NR, false>(ra, fma(kap, ra, beta[k]), n0, eta, etap, s_tab, qr, qi, ar[k],
                                                    ai[k]);
                            ring_term<R, NR, false>(rb, fma(kap, rb, beta[k]), n0, eta, etap, s_tab, mr, mi, ar[k],
                                                    ai[k]);
                        }
                    }
                }
            }
            r0 = r1;
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
                part[((int64_t)w.slot * nrhs + cb + c) * N + w.t0 + t] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA-assisted source order (kappa > 0).  With the source y and its normal n
// in the source body's frame and the target p = Rot^T (x - c) in the same frame,
//   R'^2 = s2 (|p|^2 - 2 p.y + |y|^2),   nd' = c1 n.(p - y)
// (s2 = (k/2pi)^2, c1 = (k/2pi)^3, so R' is the phase in revolutions) are
// 16 x 16 blocks (sources x targets) of the products of the 4-vectors
// [s2(-2y, |y|^2)] and [p, 1] plus s2 |p|^2, and of [c1(n, -n.y)] and [p, 1]:
// one 16x16x4 MFMA each per 256 pairs, which takes the FMAs of R^2 and n.d
// off the VALU.  Since |y| is at most the body's bounding radius and R at
// least the gap to the next body, the cancellation in |p|^2 - 2p.y + |y|^2
// stays bounded.  A wave owns G groups of 16 targets; lane l receives four
// sources of each 16-source block for target l%16 of each group: sources
// 4(l/16)+v in FP32 and (l/16)+4v in FP64 (v = 0..3; the two MFMAs place their
// result rows differently).
//   NR < 16 right-hand sides: the complex multiply-accumulate stays on the
//   VALU; the four source partial sums of a target are added across lanes at
//   the end (fixed order).
//   NR = 16: the multiply-accumulate is MFMA too: per group and per v, the
//   16 x 4 block of kernel values (targets x the lane's sources, taken straight
//   from the lanes that computed them) times the 4 x 16 block of densities
//   (sources x right-hand sides), three real MFMAs for the complex product
//   (Gauss: Gr qr, Gi qi, (Gr + Gi)(qr + qi)).
// MFMAs and VALU instructions do not overlap on a SIMD (the co-execution
// counter stays at zero for this kernel), and one 16x16x4 MFMA costs what the
// VALU FMAs it replaces cost (FP32: 16 instructions at twice the FMA rate;
// FP64: the same rate), so the order pays off where it shares one kernel
// evaluation among 16 right-hand sides without holding 16 complex
// accumulators per target in registers.
// Sources are staged through LDS in chunks of MfChunk nodes of one body,
// padded with zero densities to a multiple of 16.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R> struct MfT;
template <> struct MfT<float> {
    using V = f32x4;
    static constexpr int chunk = 256;
    // row of the lane's v-th result in a 16x16x4 MFMA output block
    static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};
template <> struct MfT<double> {
    using V = f64x4;
    static constexpr int chunk = 128;
    static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};

__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 4 pi G from R'^2 and nd' (the same arithmetic as the ring order)
template <typename R>
__device__ __forceinline__ void kernel_value(R r2, R nd, R n0, R etap, const double2 *tab, R &gr, R &gi) {
    const R u = rsq(r2);                   // 1 / R'
    R sn, cs_;
    sincos_phase(r2, u, n0, tab, sn, cs_);   // R' (less whole revolutions n0 in FP32)
    const R t = nd * (u * u);
    const R P = t * u;                     // n.d / R^3
    const R Q = fma(R(-6.283185307179586476925287), t, etap * u);   // eta / R - k n.d / R^2
    gr = fma(cs_, P, -sn * Q);
    gi = fma(cs_, Q, sn * P);
}

// the body whose node range holds node s: boff[b] <= s < boff[b + 1]
__device__ __forceinline__ int body_of(const int64_t *__restrict__ boff, int nb, int64_t s) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename R, int G, int NR>
__global__ __launch_bounds__(256) void interbody_mfma_kernel(
    const IBWork *__restrict__ work, const R *__restrict__ geo, const typename MfT<R>::V *__restrict__ sop,
    const typename C2T<R>::T *__restrict__ q, const int64_t *__restrict__ boff, int nbodies,
    const R *__restrict__ frame, int64_t N, int nrhs, int c0, R s2, R etap, const double2 *__restrict__ sctab,
    typename C2T<R>::T *__restrict__ part) {
    using V = typename MfT<R>::V;
    using R2 = typename C2T<R>::T;
    constexpr int CH = MfT<R>::chunk;
    constexpr bool MACC = NR == 16;
    static_assert(NR == 1 || NR == 2 || NR == 4 || NR == 8 || NR == 16, "rhs group");
    __shared__ V s_sr[CH], s_sn[CH];
    // densities: NR < 16 as [src][c](re, im); NR = 16 as planes re[src][c], im[src][c]
    __shared__ R s_q[CH * 2 * NR];
    __shared__ double2 s_tab[sizeof(R) == 8 ? SC_N : 1];
    load_sctab<R, 256>(s_tab, sctab);

    const IBWork w = work[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int cb = c0 + blockIdx.y * NR;
    const R *gx = geo, *gy = geo + N, *gz = geo + 2 * N;
    const V zero4 = {R(0), R(0), R(0), R(0)};

    R tx[G], ty[G], tz[G], bT[G], n0 = R(0);
    V cR[G];
    R ar[G][MACC ? 1 : NR], ai[G][MACC ? 1 : NR];
    V kr[G], ki[G], ks[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = (wv * G + g) * 16 + col;
        const int64_t gi = w.t0 + (t < w.tn ? t : 0);
        tx[g] = gx[gi];
        ty[g] = gy[gi];
        tz[g] = gz[gi];
        bT[g] = R(0);
        cR[g] = zero4;
        kr[g] = ki[g] = ks[g] = zero4;
#pragma unroll
        for (int c = 0; c < (MACC ? 1 : NR); ++c) ar[g][c] = ai[g][c] = R(0);
    }
    int prev = -1;

#pragma unroll 1
    for (int rng = 0; rng < 2; ++rng) {
        const int64_t lo = rng == 0 ? w.s0 : w.s2;
        const int64_t hi = rng == 0 ? w.s1 : w.s3;
        int64_t s = lo;
#pragma unroll 1
        while (s < hi) {
            const int b = body_of(boff, nbodies, s);
            const int64_t e = min(hi, min(boff[b + 1], s + (int64_t)CH));
            const int n = (int)(e - s), n16 = (n + 15) & ~15;
            if (b != prev) {
                // B operand: component kq of (p, 1); C operand: s2 |p|^2;
                // whole revolutions n0 as in the ring order
                const R *f = frame + FRAME * b;
                const R k2pi = sqrt(s2);
                R m = R(1e30);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const R dx = tx[g] - f[0], dy = ty[g] - f[1], dz = tz[g] - f[2];
                    const R px = fma(f[3], dx, fma(f[6], dy, f[9] * dz));
                    const R py = fma(f[4], dx, fma(f[7], dy, f[10] * dz));
                    const R pz = fma(f[5], dx, fma(f[8], dy, f[11] * dz));
                    bT[g] = kq == 0 ? px : kq == 1 ? py : kq == 2 ? pz : R(1);
                    const R p2 = fma(px, px, fma(py, py, pz * pz));
                    const R c2 = s2 * p2;
                    cR[g] = (V){c2, c2, c2, c2};
                    m = fmin(m, (sqrt(p2) - f[12]) * k2pi);
                }
                n0 = wave_floor_min(m);
                prev = b;
            }
            __syncthreads();
            for (int i = tid; i < n16; i += 256) {
                const bool ok = i < n;
                s_sr[i] = ok ? sop[s + i] : zero4;
                s_sn[i] = ok ? sop[N + s + i] : zero4;
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    R2 v;
                    v.x = v.y = R(0);
                    if (ok) v = q[(int64_t)(cb + c) * N + s + i];
                    if constexpr (MACC) {
                        s_q[i * 16 + c] = v.x;
                        s_q[CH * 16 + i * 16 + c] = v.y;
                    } else {
                        s_q[2 * (i * NR + c)] = v.x;
                        s_q[2 * (i * NR + c) + 1] = v.y;
                    }
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int j = 0; j < n16; j += 16) {
                const R a1 = ((const R *)s_sr)[(j + col) * 4 + kq];
                const R a2 = ((const R *)s_sn)[(j + col) * 4 + kq];
                if constexpr (!MACC) {
                    R qr[4][NR], qi[4][NR];
#pragma unroll
                    for (int v = 0; v < 4; ++v)
#pragma unroll
                        for (int c = 0; c < NR; ++c) {
                            const int ix = 2 * ((j + MfT<R>::row(kq, v)) * NR + c);
                            qr[v][c] = s_q[ix];
                            qi[v][c] = s_q[ix + 1];
                        }
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const V d1 = mfma_16x16x4(a1, bT[g], cR[g]);
                        const V d2 = mfma_16x16x4(a2, bT[g], zero4);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            R gr, gi;
                            kernel_value<R>(d1[v], d2[v], n0, etap, s_tab, gr, gi);
#pragma unroll
                            for (int c = 0; c < NR; ++c) {
                                ar[g][c] = fma(gr, qr[v][c], fma(-gi, qi[v][c], ar[g][c]));
                                ai[g][c] = fma(gr, qi[v][c], fma(gi, qr[v][c], ai[g][c]));
                            }
                        }
                    }
                } else {
                    // complex product with three real MFMAs (Gauss):
                    // K1 += Gr qr, K2 += Gi qi, K3 += (Gr + Gi)(qr + qi);
                    // Re = K1 - K2, Im = K3 - K1 - K2 after the last source
                    R bqr[4], bqi[4], bqs[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int src = j + MfT<R>::row(kq, v);
                        bqr[v] = s_q[src * 16 + col];
                        bqi[v] = s_q[CH * 16 + src * 16 + col];
                        bqs[v] = bqr[v] + bqi[v];
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const V d1 = mfma_16x16x4(a1, bT[g], cR[g]);
                        const V d2 = mfma_16x16x4(a2, bT[g], zero4);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            R gr, gi;
                            kernel_value<R>(d1[v], d2[v], n0, etap, s_tab, gr, gi);
                            kr[g] = mfma_16x16x4(gr, bqr[v], kr[g]);
                            ki[g] = mfma_16x16x4(gi, bqi[v], ki[g]);
                            ks[g] = mfma_16x16x4(gr + gi, bqs[v], ks[g]);
                        }
                    }
                }
            }
            s = e;
        }
    }

    if constexpr (!MACC) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int t = (wv * G + g) * 16 + col;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                R xr = ar[g][c], xi = ai[g][c];
                xr += __shfl_xor(xr, 16, 64);
                xi += __shfl_xor(xi, 16, 64);
                xr += __shfl_xor(xr, 32, 64);
                xi += __shfl_xor(xi, 32, 64);
                if (kq == 0 && t < w.tn) {
                    R2 o;
                    o.x = xr;
                    o.y = xi;
                    part[((int64_t)w.slot * nrhs + cb + c) * N + w.t0 + t] = o;
                }
            }
        }
    } else {
        // the lane holds target rows row(kq, v) of each group for right-hand side l%16
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = (wv * G + g) * 16 + MfT<R>::row(kq, v);
                if (t < w.tn) {
                    R2 o;
                    o.x = kr[g][v] - ki[g][v];
                    o.y = ks[g][v] - kr[g][v] - ki[g][v];
                    part[((int64_t)w.slot * nrhs + cb + col) * N + w.t0 + t] = o;
                }
            }
    }
}

// ---------------------------------------------------------------------------
// MFMA order with the complex multiply-accumulate on the FP16 matrix cores
// (FP32 results, 16 right-hand sides per group).  The geometry and the kernel
// values are those of the MFMA order above (FP32); each kernel value g and
// each density q is split into two FP16 numbers, g ~ g_hi + g_lo with g_hi =
// g rounded toward zero and g_lo the rounded remainder, and
//   g q ~ g_hi q_hi + g_hi q_lo + g_lo q_hi
// (the dropped g_lo q_lo and the rounding of the low parts are ~2^-20 of
// |g q|, below the FP32 rounding of the phase).  Four real products make the
// complex product (Re = Gr qr + Gi (-qi), Im = Gr qi + Gi qr), 12 MFMAs
// v_mfma_f32_16x16x32_f16 per 32 sources x 16 targets x 16 rhs, 16 cycles
// each, against 12 FP32 16x16x4 MFMAs of 32 cycles per 16 sources in the
// FP32 version.  FP16 has 5 exponent bits, so both factors are scaled by
// powers of two: G by S_G, chosen on the host from the bound
// |G| <= 1/d^2 + (|eta| + kappa)/d over pairs at least d apart (d = the
// smallest gap between the bodies' bounding balls), so that |G S_G| <= 8192;
// each rhs by S_q = 2^(13 - e) with 2^e <= max |q| (max over all nodes), so
// that |q S_q| < 16384.  The results are scaled back in FP32.
// Sources come in blocks of 32 nodes of one body (the last block of a body is
// padded with zero densities); lane (kq, col) computes the kernel values of
// target col for sources 4kq+v (v = 0..3) of each 16-source half of a block,
// which are exactly the eight k = 8kq + t entries of its A operand (t = v and
// 4 + v), so the MFMA operands need no exchange between lanes.  The densities
// are split once per application into six FP16 planes (q_r, q_i, -q_i, high
// and low) already in the B-operand order: [group][block][plane][rhs][k].
// ---------------------------------------------------------------------------
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
constexpr int MF16_CB = 4;           // 32-source blocks per LDS chunk
constexpr int MF16_BLK = 6 * 16 * 4; // h8 per block: 6 planes x 16 rhs x 4 k-slices

__device__ __forceinline__ f32x4 mfma_16x16x32h(h8 a, h8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// high and low FP16 parts of eight values: the high part rounded toward zero
// (v_cvt_pkrtz, two values per instruction), the low part the exact FP32
// remainder g - f32(high) rounded to nearest by the mixed-precision FMA, which
// reads the FP16 high part directly and writes one half of the packed result
// (v_fma_mixlo_f16 the low half, v_fma_mixhi_f16 the high half; each leaves
// the other half of its destination as it was)
__device__ __forceinline__ void split2(float a, float b, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(a, b));
    unsigned l;
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(l) : "v"(hi), "v"(a));
    asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(l) : "v"(hi), "v"(b));
    lo = l;
}
__device__ __forceinline__ void split8(const float *g, h8 &hi, h8 &lo) {
    unsigned h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) split2(g[2 * p], g[2 * p + 1], h[p], l[p]);
    hi = __builtin_bit_cast(h8, (uint4){h[0], h[1], h[2], h[3]});
    lo = __builtin_bit_cast(h8, (uint4){l[0], l[1], l[2], l[3]});
}
// 2^(13 - e) for the largest |q| of a rhs (bits of a non-negative float), 1 for 0
__device__ __forceinline__ int qscale_exp(unsigned bits) {
    if (bits == 0u) return 0;
    const int e = (int)(bits >> 23) - 127;       // floor(log2 max), normal numbers
    return 13 - (e < -100 ? -100 : e);
}

// Per-rhs max of max(|re|, |im|) of the staged densities, as the bits of a
// non-negative float (their integer order is the float order).  Two steps and
// no atomics (device-wide atomics on one address serialise across the chip):
// blocks (P, nrhs) reduce contiguous slices of a rhs into part[rhs][P], then
// one wavefront per rhs reduces the P partial maxima.
constexpr int QMAX_SLICES = 64;
__global__ __launch_bounds__(256) void qmax_part_kernel(const float2 *__restrict__ q, int64_t N,
                                                        unsigned *__restrict__ part) {
    __shared__ float s_m[4];
    const int c = blockIdx.y, P = gridDim.x;
    const int64_t per = (N + P - 1) / P;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(N, lo + per);
    float m = 0.f;
    for (int64_t j = lo + threadIdx.x; j < hi; j += 256) {
        const float2 v = q[(int64_t)c * N + j];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(int64_t)c * P + blockIdx.x] = __float_as_uint(fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3])));
}
__global__ __launch_bounds__(64) void qmax_final_kernel(const unsigned *__restrict__ part, int P,
                                                        unsigned *__restrict__ qmax) {
    const int c = blockIdx.x;
    unsigned m = 0u;
    for (int i = threadIdx.x; i < P; i += 64) m = max(m, part[(int64_t)c * P + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
    if (threadIdx.x == 0) qmax[c] = m;
}

// six FP16 planes per 32-source block and rhs group (B-operand order)
__global__ __launch_bounds__(256) void q16_kernel(const float2 *__restrict__ q, const unsigned *__restrict__ qmax,
                                                  const int64_t *__restrict__ boff, const int32_t *__restrict__ bblk,
                                                  int nbodies, int64_t N, int64_t nblk, int groups,
                                                  _Float16 *__restrict__ q16) {
    const int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x;   // ((grp * nblk + B) * 16 + c) * 32 + k
    if (item >= (int64_t)groups * nblk * 512) return;
    const int k = (int)(item & 31), c = (int)((item >> 5) & 15);
    const int64_t gb = item >> 9, B = gb % nblk;
    const int grp = (int)(gb / nblk);
    int lo = 0, hi = nbodies - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bblk[mid] <= B) lo = mid;
        else hi = mid - 1;
    }
    const int b = lo;
    const int t = k & 7, kq = k >> 3;
    const int r = (t < 4 ? 0 : 16) + 4 * kq + (t & 3);            // source of A-operand entry k
    const int64_t node = boff[b] + 32 * (B - bblk[b]) + r;
    const int rhs = grp * 16 + c;
    float2 v = make_float2(0.f, 0.f);
    if (node < boff[b + 1]) {
        v = q[(int64_t)rhs * N + node];
        const float s = ldexpf(1.f, qscale_exp(qmax[rhs]));
        v.x *= s;
        v.y *= s;
    }
    const h2 h = __builtin_bit_cast(h2, __builtin_amdgcn_cvt_pkrtz(v.x, v.y));
    const h2 l = __builtin_bit_cast(h2, __builtin_amdgcn_cvt_pkrtz(v.x - (float)h.x, v.y - (float)h.y));
    _Float16 *o = q16 + gb * (6 * 512) + c * 32 + k;
    o[0 * 512] = h.x;    // q_r high
    o[1 * 512] = l.x;    // q_r low
    o[2 * 512] = h.y;    // q_i high
    o[3 * 512] = l.y;    // q_i low
    o[4 * 512] = -h.y;   // -q_i high
    o[5 * 512] = -l.y;   // -q_i low
}

template <int G>
__global__ __launch_bounds__(256) void interbody_mfma16_kernel(
    const IBWork *__restrict__ work, const float *__restrict__ geo, const f32x4 *__restrict__ sop,
    const h8 *__restrict__ q16, const int64_t *__restrict__ boff, const int32_t *__restrict__ bblk, int nbodies,
    const float *__restrict__ frame, int64_t N, int nrhs, int64_t nblk, float s2, float etap_s, float gscale,
    int gexp, const unsigned *__restrict__ qmax, float2 *__restrict__ part) {
    __shared__ f32x4 s_sr[MF16_CB * 32], s_sn[MF16_CB * 32];
    __shared__ h8 s_q[MF16_CB * MF16_BLK];
    const IBWork w = work[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int grp = blockIdx.y, cb = grp * 16;
    const float *gx = geo, *gy = geo + N, *gz = geo + 2 * N;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    float tx[G], ty[G], tz[G], bT[G], n0 = 0.f;
    f32x4 cR[G], sumR[G], sumI[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = (wv * G + g) * 16 + col;
        const int64_t gi = w.t0 + (t < w.tn ? t : 0);
        tx[g] = gx[gi];
        ty[g] = gy[gi];
        tz[g] = gz[gi];
        bT[g] = 0.f;
        cR[g] = zero4;
        sumR[g] = sumI[g] = zero4;
    }
    int prev = -1;

#pragma unroll 1
    for (int rng = 0; rng < 2; ++rng) {
        const int64_t lo = rng == 0 ? w.s0 : w.s2;
        const int64_t hi = rng == 0 ? w.s1 : w.s3;
        int64_t B = lo;
#pragma unroll 1
        while (B < hi) {
            int b = 0;
            {
                int l2 = 0, h2_ = nbodies - 1;
                while (l2 < h2_) {
                    const int mid = (l2 + h2_ + 1) >> 1;
                    if (bblk[mid] <= B) l2 = mid;
                    else h2_ = mid - 1;
                }
                b = l2;
            }
            const int64_t e = min(hi, min((int64_t)bblk[b + 1], B + (int64_t)MF16_CB));
            const int nb = (int)(e - B);
            if (b != prev) {
                const float *f = frame + FRAME * b;
                const float k2pi = sqrtf(s2);
                float m = 1e30f;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const float dx = tx[g] - f[0], dy = ty[g] - f[1], dz = tz[g] - f[2];
                    const float px = fmaf(f[3], dx, fmaf(f[6], dy, f[9] * dz));
                    const float py = fmaf(f[4], dx, fmaf(f[7], dy, f[10] * dz));
                    const float pz = fmaf(f[5], dx, fmaf(f[8], dy, f[11] * dz));
                    bT[g] = kq == 0 ? px : kq == 1 ? py : kq == 2 ? pz : 1.f;
                    const float p2 = fmaf(px, px, fmaf(py, py, pz * pz));
                    const float c2 = s2 * p2;
                    cR[g] = (f32x4){c2, c2, c2, c2};
                    m = fminf(m, (sqrtf(p2) - f[12]) * k2pi);
                }
                n0 = wave_floor_min(m);
                prev = b;
            }
            __syncthreads();
            const int64_t first = boff[b] + 32 * (B - bblk[b]);
            for (int i = tid; i < nb * 32; i += 256) {
                const int64_t node = first + i;
                const bool ok = node < boff[b + 1];
                s_sr[i] = ok ? sop[node] : zero4;
                s_sn[i] = ok ? sop[N + node] * gscale : zero4;   // nd' scaled by S_G
            }
            const h8 *src = q16 + ((int64_t)grp * nblk + B) * MF16_BLK;
            for (int i = tid; i < nb * MF16_BLK; i += 256) s_q[i] = src[i];
            __syncthreads();
            // the matrix cores accumulate one chunk (at most 128 sources) from
            // zero; the chunk sums are added on the VALU, rounded to nearest
            f32x4 accR[G], accI[G];
#pragma unroll
            for (int g = 0; g < G; ++g) accR[g] = accI[g] = zero4;
#pragma unroll 1
            for (int jb = 0; jb < nb; ++jb) {
                const h8 *qb = s_q + jb * MF16_BLK;
                const h8 qrh = qb[(0 * 16 + col) * 4 + kq], qrl = qb[(1 * 16 + col) * 4 + kq];
                const h8 qih = qb[(2 * 16 + col) * 4 + kq], qil = qb[(3 * 16 + col) * 4 + kq];
                const h8 nqh = qb[(4 * 16 + col) * 4 + kq], nql = qb[(5 * 16 + col) * 4 + kq];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    float gr[8], gi[8];
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const int j = jb * 32 + half * 16 + col;
                        const float a1 = ((const float *)s_sr)[j * 4 + kq];
                        const float a2 = ((const float *)s_sn)[j * 4 + kq];
                        const f32x4 d1 = mfma_16x16x4(a1, bT[g], cR[g]);
                        const f32x4 d2 = mfma_16x16x4(a2, bT[g], zero4);
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            kernel_value<float>(d1[v], d2[v], n0, etap_s, nullptr, gr[half * 4 + v], gi[half * 4 + v]);
                    }
                    h8 grh, grl, gih, gil;
                    split8(gr, grh, grl);
                    split8(gi, gih, gil);
                    accR[g] = mfma_16x16x32h(grh, qrh, accR[g]);
                    accI[g] = mfma_16x16x32h(grh, qih, accI[g]);
                    accR[g] = mfma_16x16x32h(grh, qrl, accR[g]);
                    accI[g] = mfma_16x16x32h(grh, qil, accI[g]);
                    accR[g] = mfma_16x16x32h(grl, qrh, accR[g]);
                    accI[g] = mfma_16x16x32h(grl, qih, accI[g]);
                    accR[g] = mfma_16x16x32h(gih, nqh, accR[g]);
                    accI[g] = mfma_16x16x32h(gih, qrh, accI[g]);
                    accR[g] = mfma_16x16x32h(gih, nql, accR[g]);
                    accI[g] = mfma_16x16x32h(gih, qrl, accI[g]);
                    accR[g] = mfma_16x16x32h(gil, nqh, accR[g]);
                    accI[g] = mfma_16x16x32h(gil, qrh, accI[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                sumR[g] += accR[g];
                sumI[g] += accI[g];
            }
            B = e;
        }
    }
    // lane (kq, col) holds targets 4kq + v of each group for rhs cb + col
    const float inv = ldexpf(1.f, -(gexp + qscale_exp(qmax[cb + col])));
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = (wv * G + g) * 16 + 4 * kq + v;
            if (t < w.tn) {
                float2 o;
                o.x = sumR[g][v] * inv;
                o.y = sumI[g][v] * inv;
                part[((int64_t)w.slot * nrhs + cb + col) * N + w.t0 + t] = o;
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
                                    int64_t total, int add, double2 *__restrict__ y, int64_t N, int64_t row0,
                                    int64_t row1) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t row = i % N;
    if (row < row0 || row >= row1) {   // rows of bodies outside the target range
        if (!add) y[i] = make_double2(0.0, 0.0);
        return;
    }
    double re = 0, im = 0;
    if (add) {
        re = y[i].x;
        im = y[i].y;
    }
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
struct IBShape {
    int variant, tpt, bs, splits;
};

// targets per work item: TPT x block, or for the MFMA orders 16 x G x 4 waves
static int ib_tile(const IBShape &s) { return s.variant >= 3 ? 64 * s.tpt : s.tpt * s.bs; }

static IBShape launch_shape(Ctx &c, int prec, int nrhs) {
    const int pi = prec == AXS_FP32 ? 1 : 0;
    IBShape s;
    // Defaults from the launch-shape sweeps on MI355X (27-sphere lattice, one
    // rhs; 8 mixed bodies, 1-64 rhs; 64 mixed bodies, 16 rhs): below 16 rhs
    // the ring order (1 target per thread in FP32, 4 in FP64), from 16 rhs on
    // the MFMA order (2 groups of 16 targets per wavefront in FP32, with the
    // FP16 multiply-accumulate where the kernel values have a bound; 4 groups
    // in FP64); the point order where neither applies.
    s.bs = c.ib_block[pi] > 0 ? c.ib_block[pi] : 256;
    const bool ring_ok = !c.no_rings && c.max_nf / 2 + 1 <= s.bs && (c.kappa == 0 || c.near_phase_ok);
    const bool mf_ok = c.kappa > 0 && c.mf_src && c.near_phase_ok && s.bs == 256 &&
                       (c.ib_tpt[pi] == 0 || c.ib_tpt[pi] <= 4);
    const bool mf16_ok = mf_ok && prec == AXS_FP32 && c.mf16_ok;
    s.variant = c.ib_variant[pi] > 0 ? c.ib_variant[pi]
                : (nrhs >= 16 && mf16_ok) ? 4 : (nrhs >= 16 && mf_ok) ? 3 : ring_ok ? 2 : 1;
    const int dflt = prec == AXS_FP32 ? (s.variant == 2 ? 1 : 2) : 4;
    s.tpt = c.ib_tpt[pi] > 0 ? c.ib_tpt[pi] : dflt;
    AXS_REQUIRE(s.variant != 2 || ring_ok, AXS_EINVAL,
                "ring variant needs N_F/2 + 1 <= threads per block and bodies under 127 wavelengths across");
    if (s.variant == 4)
        AXS_REQUIRE(prec == AXS_FP32 && c.mf16_ok, AXS_EINVAL,
                    "FP16 multiply-accumulate: FP32 only, and bodies whose bounding balls do not overlap");
    if (s.variant >= 3) {
        AXS_REQUIRE(c.kappa > 0 && c.mf_src && c.near_phase_ok, AXS_EINVAL,
                    "MFMA variant needs kappa > 0 and bodies under 127 wavelengths across");
        AXS_REQUIRE(s.tpt == 1 || s.tpt == 2 || s.tpt == 4, AXS_EINVAL,
                    "MFMA variant: 1, 2 or 4 groups of 16 targets per wave");
        AXS_REQUIRE(s.bs == 256, AXS_EINVAL, "MFMA variant uses 256-thread blocks");
    }
    if (c.ib_splits[pi] > 0) {
        s.splits = c.ib_splits[pi];
    } else {
        // enough blocks to fill 256 CUs several times over; the FP32 ring order
        // (8 resident blocks per CU) takes 16K so that the last, partly filled
        // round of blocks is a small share of the launch
        int64_t tiles = 0;   // of the target rows computed (all bodies, or the set range)
        for (size_t bi = 0; bi < c.bodies.size(); ++bi)
            if (c.tgt_count < 0 || ((int)bi >= c.tgt_first && (int)bi < c.tgt_first + c.tgt_count))
                tiles += ceil_div(c.bodies[bi].n, (int64_t)ib_tile(s));
        const int64_t want = (prec == AXS_FP32 && s.variant == 2) ? 16384 : 4096;
        s.splits = 1;
        while (tiles * s.splits < want && s.splits < 64) s.splits *= 2;
    }
    return s;
}

int interbody_splits(Ctx &c, int prec, int nrhs) { return launch_shape(c, prec, nrhs).splits; }

void interbody_shape(Ctx &c, int prec, int nrhs, int out[4]) {
    const IBShape s = launch_shape(c, prec, nrhs);
    out[0] = s.variant;
    out[1] = s.tpt;
    out[2] = s.bs;
    out[3] = s.splits;
}

// Work items (worktable.h) in units of nodes, rings or 32-node blocks
enum class Units { nodes, rings, blocks };
static std::vector<IBWork> build_work(Ctx &c, int tile, int splits, Units units) {
    std::vector<WorkBody> wb;
    int64_t boff = 0;
    for (size_t bi = 0; bi < c.bodies.size(); ++bi) {
        const auto &b = c.bodies[bi];
        const int64_t nbk = ceil_div(b.n, (int64_t)32);
        const int64_t uoff = units == Units::rings ? c.ring_base[bi] : units == Units::blocks ? boff : b.offset;
        const int64_t un = units == Units::rings ? c.shapes[b.shape].NG : units == Units::blocks ? nbk : b.n;
        boff += nbk;
        // bodies outside the target range keep their sources, lose their targets
        const bool own = c.tgt_count < 0 || ((int)bi >= c.tgt_first && (int)bi < c.tgt_first + c.tgt_count);
        wb.push_back(WorkBody{b.offset, own ? b.n : 0, uoff, un});
    }
    const int64_t U = units == Units::rings ? c.nrings : units == Units::blocks ? c.nblk : c.N;
    return build_work_table(wb, U, tile, splits);
}

// ring tables, body frames and per-node azimuth cos/sin (built once)
void build_ring_tables(Ctx &c) {
    const int64_t N = c.N;
    std::vector<int32_t> ri;
    std::vector<double> rg, fr, csv(2 * N);
    c.ring_base.clear();
    int nr = 0;
    c.max_nf = 0;
    for (size_t bi = 0; bi < c.bodies.size(); ++bi) {
        const auto &b = c.bodies[bi];
        const Shape &s = c.shapes[b.shape];
        c.ring_base.push_back(nr);
        nr += s.NG;
        c.max_nf = std::max(c.max_nf, s.NF);
        for (int a = 0; a < 3; ++a) fr.push_back(b.centre[a]);
        for (int a = 0; a < 9; ++a) fr.push_back(b.rot[a]);
        fr.push_back(b.bound_radius);
        for (int a = 13; a < FRAME; ++a) fr.push_back(0.0);
        for (int l = 0; l < s.NF; ++l) {
            const double th = 2.0 * M_PI * l / s.NF;
            for (int i = 0; i < s.NG; ++i) {
                const int64_t j = b.offset + (int64_t)i * s.NF + l;
                csv[j] = std::cos(th);
                csv[N + j] = std::sin(th);
            }
        }
    }
    c.nrings = nr;
    // phases less whole revolutions stay below 2 (r_t + r_s) k/2pi + 1 revolutions
    double rmax = 0;
    for (auto &b : c.bodies) rmax = std::max(rmax, b.bound_radius);
    c.near_phase_ok = 4.0 * rmax * c.kappa / (2.0 * M_PI) + 2.0 < 256.0;
    // every pair of nodes closer than 255 wavelengths: the point order's FP32
    // phase stays inside the hardware sin/cos input range
    double dmax = 0;
    for (size_t a = 0; a < c.bodies.size(); ++a)
        for (size_t b = a; b < c.bodies.size(); ++b) {
            const auto &A = c.bodies[a], &B = c.bodies[b];
            const double dx = A.centre[0] - B.centre[0], dy = A.centre[1] - B.centre[1], dz = A.centre[2] - B.centre[2];
            dmax = std::max(dmax, std::sqrt(dx * dx + dy * dy + dz * dz) + A.bound_radius + B.bound_radius);
        }
    c.scene_phase_ok = dmax * c.kappa / (2.0 * M_PI) < 255.0;
    std::vector<int32_t> off(nr), nf(nr), body(nr), eoff(nr + 1, 0);
    std::vector<int2> pairs;
    std::vector<double> g(5 * (size_t)nr);
    AXS_REQUIRE(N < (int64_t)INT32_MAX, AXS_EINVAL, "node count beyond 32-bit ring tables");
    for (size_t bi = 0; bi < c.bodies.size(); ++bi) {
        const auto &b = c.bodies[bi];
        const Shape &s = c.shapes[b.shape];
        for (int i = 0; i < s.NG; ++i) {
            const int id = (int)c.ring_base[bi] + i;
            off[id] = (int32_t)(b.offset + (int64_t)i * s.NF);
            nf[id] = s.NF;
            body[id] = (int32_t)bi;
            // mirror-pair entries e = 0 .. N_F/2: azimuth e and N_F - e
            eoff[id] = (int32_t)pairs.size();
            for (int e = 0; e <= s.NF / 2; ++e) {
                const int mir = (e == 0 || 2 * e == s.NF) ? -1 : off[id] + s.NF - e;
                pairs.push_back(make_int2(off[id] + e, mir));
            }
            const double sp = std::hypot(s.dr[i], s.dz[i]);
            g[id] = s.r[i];
            g[nr + id] = s.z[i];
            g[2 * nr + id] = -s.dz[i] / sp;
            g[3 * nr + id] = s.dr[i] / sp;
            g[4 * nr + id] = s.r[i] > 0 ? -0.5 * g[2 * nr + id] / s.r[i] : 0.0;
        }
    }
    ri.insert(ri.end(), off.begin(), off.end());
    ri.insert(ri.end(), nf.begin(), nf.end());
    ri.insert(ri.end(), body.begin(), body.end());
    eoff[nr] = (int32_t)pairs.size();
    ri.insert(ri.end(), eoff.begin(), eoff.end());
    c.ring_i = (int32_t *)c.dalloc(ri.size() * sizeof(int32_t));
    AXS_HIP(hipMemcpy(c.ring_i, ri.data(), ri.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    c.ring_pair = (int2 *)c.dalloc(pairs.size() * sizeof(int2));
    AXS_HIP(hipMemcpy(c.ring_pair, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice));
    auto up = [&](const std::vector<double> &h, double *&d64, float *&d32) {
        std::vector<float> f(h.begin(), h.end());
        d64 = (double *)c.dalloc(h.size() * sizeof(double));
        d32 = (float *)c.dalloc(h.size() * sizeof(float));
        AXS_HIP(hipMemcpy(d64, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
        AXS_HIP(hipMemcpy(d32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    };
    up(g, c.ring_g64, c.ring_g32);
    up(fr, c.frame64, c.frame32);
    up(csv, c.cs64, c.cs32);

    // (cos, sin)(2 pi k / 1024) for the FP64 sin/cos of the inter-body kernels
    std::vector<double> tab(2 * SC_N);
    for (int k = 0; k < SC_N; ++k) {
        tab[2 * k] = std::cos(2.0 * M_PI * k / SC_N);
        tab[2 * k + 1] = std::sin(2.0 * M_PI * k / SC_N);
    }
    c.sctab = (double2 *)c.dalloc(tab.size() * sizeof(double));
    AXS_HIP(hipMemcpy(c.sctab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));

    std::vector<int64_t> bo;
    for (auto &b : c.bodies) bo.push_back(b.offset);
    bo.push_back(N);
    c.body_off = (int64_t *)c.dalloc(bo.size() * sizeof(int64_t));
    AXS_HIP(hipMemcpy(c.body_off, bo.data(), bo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    std::vector<int32_t> bk(1, 0);
    for (auto &b : c.bodies) bk.push_back(bk.back() + (int32_t)ceil_div(b.n, (int64_t)32));
    c.nblk = bk.back();
    c.blk_off = (int32_t *)c.dalloc(bk.size() * sizeof(int32_t));
    AXS_HIP(hipMemcpy(c.blk_off, bk.data(), bk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    // FP16 multiply-accumulate: every inter-body pair is at least dmin apart
    // (the smallest gap between bounding balls), so |4 pi G| <= 1/dmin^2 +
    // (|eta| + kappa)/dmin; S_G = 2^gexp brings that bound to at most 8192
    double dmin = 1e300;
    for (size_t a = 0; a < c.bodies.size(); ++a)
        for (size_t b2 = a + 1; b2 < c.bodies.size(); ++b2) {
            const auto &A = c.bodies[a], &Bb = c.bodies[b2];
            const double dx = A.centre[0] - Bb.centre[0], dy = A.centre[1] - Bb.centre[1],
                         dz = A.centre[2] - Bb.centre[2];
            dmin = std::min(dmin, std::sqrt(dx * dx + dy * dy + dz * dz) - A.bound_radius - Bb.bound_radius);
        }
    c.mf16_ok = false;
    if (c.bodies.size() > 1 && dmin > 1e-3) {
        const double gb = 1.0 / (dmin * dmin) + (std::fabs(c.eta) + c.kappa) / dmin;
        c.mf16_gexp = (int)std::floor(std::log2(8192.0 / gb));
        c.mf16_ok = c.mf16_gexp > -60 && c.mf16_gexp < 60;
    }
    if (c.kappa > 0) {
        // MFMA source operands in each body's frame, scaled so that the
        // products give R'^2 and nd' of the ring order directly
        const double k2pi = c.kappa / (2.0 * M_PI), s2 = k2pi * k2pi, c1 = s2 * k2pi;
        std::vector<double> mf64(8 * (size_t)N);
        for (size_t bi = 0; bi < c.bodies.size(); ++bi) {
            const auto &b = c.bodies[bi];
            const Shape &s = c.shapes[b.shape];
            for (int i = 0; i < s.NG; ++i) {
                const double sp = std::hypot(s.dr[i], s.dz[i]);
                const double nr = -s.dz[i] / sp, nz = s.dr[i] / sp;
                for (int l = 0; l < s.NF; ++l) {
                    const double th = 2.0 * M_PI * l / s.NF, ct = std::cos(th), st = std::sin(th);
                    const double y[3] = {s.r[i] * ct, s.r[i] * st, s.z[i]};
                    const double n[3] = {nr * ct, nr * st, nz};
                    const int64_t j = b.offset + (int64_t)i * s.NF + l;
                    double *a = &mf64[4 * j], *d = &mf64[4 * (N + j)];
                    for (int k = 0; k < 3; ++k) {
                        a[k] = -2.0 * s2 * y[k];
                        d[k] = c1 * n[k];
                    }
                    a[3] = s2 * (y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                    d[3] = -c1 * (n[0] * y[0] + n[1] * y[1] + n[2] * y[2]);
                }
            }
        }
        const std::vector<float> mf(mf64.begin(), mf64.end());
        c.mf_src = (float *)c.dalloc(mf.size() * sizeof(float));
        AXS_HIP(hipMemcpy(c.mf_src, mf.data(), mf.size() * sizeof(float), hipMemcpyHostToDevice));
        c.mf_src64 = (double *)c.dalloc(mf64.size() * sizeof(double));
        AXS_HIP(hipMemcpy(c.mf_src64, mf64.data(), mf64.size() * sizeof(double), hipMemcpyHostToDevice));
    }
}

template <typename R, int TPT, int BS, bool LAP>
static void launch_ib(Ctx &c, int variant, const IBWork *work, int nwork, const R *geo, const R *cs,
                      const R *rg, const R *frame, const typename C2T<R>::T *q, int nrhs,
                      typename C2T<R>::T *part) {
    // at kappa = 0 the ring order runs unscaled (k/2pi replaced by 1, no phase)
    const R kappa = (R)c.kappa, k2pi = LAP ? R(1) : (R)(c.kappa / (2.0 * M_PI)), eta = (R)c.eta;
    const RingTabs rt{c.ring_i, c.ring_i + c.nrings, c.ring_i + 2 * c.nrings, c.ring_i + 3 * c.nrings,
                      c.ring_pair};
    // one launch covers every body and every full group of NR right-hand sides
    // (grid.y = groups); a remainder group gets one more launch.  Groups stop
    // at 8: with mirror pairs a 16- or 32-wide group doubles the LDS tile and
    // the registers of the densities, and ran slower than groups of 8 (64 rhs
    // beyond 16 take the MFMA order anyway).
    int c0 = 0;
    while (c0 < nrhs) {
        const int left = nrhs - c0;
        const int nr = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        const int groups = left / nr;
#define AXS_IB_NR(NR_)                                                                                     \
    if (nr == NR_) {                                                                                       \
        if (variant == 2)                                                                                  \
            hipLaunchKernelGGL((interbody_ring_kernel<R, TPT, NR_, BS, LAP>), dim3(nwork, groups), dim3(BS), 0, \
                               c.stream, work, geo, cs, q, rt, rg, c.nrings, frame, c.N, nrhs, c0, k2pi, eta, \
                               c.sctab, part);                                                             \
        else                                                                                               \
            hipLaunchKernelGGL((interbody_kernel<R, TPT, NR_, BS, LAP>), dim3(nwork, groups), dim3(BS), 0, \
                               c.stream, work, geo, q, c.N, nrhs, c0, kappa, k2pi, eta, c.sctab,        \
                               c.scene_phase_ok ? 1 : 0, part);                                       \
    }
        AXS_IB_NR(8)
        AXS_IB_NR(4)
        AXS_IB_NR(2)
        AXS_IB_NR(1)
#undef AXS_IB_NR
        AXS_HIP(hipGetLastError());
        c0 += nr * groups;
    }
}

// MFMA order: full groups of 16 right-hand sides use MFMA accumulation, the
// remainder groups of 8, 4, 2, 1 the VALU one.
template <typename R, int G>
static void launch_mf(Ctx &c, const IBWork *work, int nwork, const typename C2T<R>::T *q, int nrhs,
                      typename C2T<R>::T *part, int c_begin = 0) {
    const R k2pi = (R)(c.kappa / (2.0 * M_PI));
    const R s2 = k2pi * k2pi, etap = (R)c.eta * k2pi;
    const R *geo = sizeof(R) == 4 ? (const R *)c.g32 : (const R *)c.g64;
    const R *frame = sizeof(R) == 4 ? (const R *)c.frame32 : (const R *)c.frame64;
    const auto *sop = (const typename MfT<R>::V *)(sizeof(R) == 4 ? (const void *)c.mf_src : (const void *)c.mf_src64);
    const int nb = (int)c.bodies.size();
    int c0 = c_begin;
    while (c0 < nrhs) {
        const int left = nrhs - c0;
        const int nr = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        const int groups = left / nr;
#define AXS_MF_NR(NR_)                                                                                      \
    if (nr == NR_)                                                                                         \
        hipLaunchKernelGGL((interbody_mfma_kernel<R, G, NR_>), dim3(nwork, groups), dim3(256), 0, c.stream, \
                           work, geo, sop, q, c.body_off, nb, frame, c.N, nrhs, c0, s2, etap, c.sctab, part);
        AXS_MF_NR(16)
        AXS_MF_NR(8)
        AXS_MF_NR(4)
        AXS_MF_NR(2)
        AXS_MF_NR(1)
#undef AXS_MF_NR
        AXS_HIP(hipGetLastError());
        c0 += nr * groups;
    }
}

template <typename R>
static void dispatch_ib(Ctx &c, const IBShape &s, const IBWork *work, int nwork, const R *geo, const R *cs,
                        const R *rg, const R *frame, const typename C2T<R>::T *q, int nrhs,
                        typename C2T<R>::T *part) {
    if (s.variant == 3) {
        if (s.tpt == 1) launch_mf<R, 1>(c, work, nwork, q, nrhs, part);
        else if (s.tpt == 2) launch_mf<R, 2>(c, work, nwork, q, nrhs, part);
        else launch_mf<R, 4>(c, work, nwork, q, nrhs, part);
        return;
    }
#define AXS_IB_CASE(T_, B_)                                                             \
    if (s.tpt == T_ && s.bs == B_) {                                                    \
        if (c.kappa > 0)                                                                \
            launch_ib<R, T_, B_, false>(c, s.variant, work, nwork, geo, cs, rg, frame, q, nrhs, part); \
        else                                                                            \
            launch_ib<R, T_, B_, true>(c, s.variant, work, nwork, geo, cs, rg, frame, q, nrhs, part); \
        return;                                                                         \
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

// cached work table [precision][wi] for a launch shape
static const IBWork *get_work(Ctx &c, int pi, int wi, const IBShape &s, Units units, int &nwork) {
    int *key = c.ib_key[pi][wi];
    if (!c.ib_work[pi][wi] || key[0] != s.tpt || key[1] != s.bs || key[2] != s.splits || key[3] != s.variant ||
        key[4] != c.tgt_first || key[5] != c.tgt_count) {
        // work tables are cached per launch shape; rebuilt only when it changes
        std::vector<IBWork> work = build_work(c, ib_tile(s), s.splits, units);
        if (c.arena) {
            // no allocation: the table goes to the caller's region for this call
            // only (the cache is left as it is)
            IBWork *t = (IBWork *)c.scratch(WS_WORK, work.size() * sizeof(IBWork));
            AXS_HIP(hipMemcpyAsync(t, work.data(), work.size() * sizeof(IBWork), hipMemcpyHostToDevice, c.stream));
            AXS_HIP(hipStreamSynchronize(c.stream));   // work is pageable host memory
            nwork = (int)work.size();
            return t;
        }
        if (c.ib_work[pi][wi]) {
            AXS_HIP(hipStreamSynchronize(c.stream));
            c.dfree(c.ib_work[pi][wi]);
        }
        c.ib_work[pi][wi] = (IBWork *)c.dalloc(work.size() * sizeof(IBWork));
        AXS_HIP(hipMemcpy(c.ib_work[pi][wi], work.data(), work.size() * sizeof(IBWork), hipMemcpyHostToDevice));
        c.ib_nwork[pi][wi] = (int)work.size();
        key[0] = s.tpt;
        key[1] = s.bs;
        key[2] = s.splits;
        key[3] = s.variant;
        key[4] = c.tgt_first;
        key[5] = c.tgt_count;
    }
    nwork = c.ib_nwork[pi][wi];
    return c.ib_work[pi][wi];
}

// MFMA order with the FP16 multiply-accumulate: full groups of 16 rhs over
// 32-node source blocks; a remainder of fewer than 16 rhs takes the FP32 MFMA
// order (node units).  Both write the same [splits][nrhs][N] partial sums.
static void launch_mf16(Ctx &c, const IBShape &s, const float2 *q, int nrhs, float2 *part) {
    const int groups = nrhs / 16;
    if (groups > 0) {
        int nwork = 0;
        const IBWork *work = get_work(c, 1, 2, s, Units::blocks, nwork);
        // slices of at least 16K nodes per block, at most QMAX_SLICES per rhs
        const int P = (int)std::min<int64_t>(QMAX_SLICES, std::max<int64_t>(1, c.N / 16384));
        unsigned *qmax = (unsigned *)c.scratch(WS_QMAX, (size_t)nrhs * (P + 1) * sizeof(unsigned));
        unsigned *qpart = qmax + nrhs;
        hipLaunchKernelGGL(qmax_part_kernel, dim3(P, nrhs), dim3(256), 0, c.stream, q, c.N, qpart);
        hipLaunchKernelGGL(qmax_final_kernel, dim3(nrhs), dim3(64), 0, c.stream, qpart, P, qmax);
        const int64_t items = (int64_t)groups * c.nblk * 512;
        _Float16 *q16 = (_Float16 *)c.scratch(WS_Q16, (size_t)items * 6 * sizeof(_Float16));
        hipLaunchKernelGGL(q16_kernel, dim3(ceil_div(items, (int64_t)256)), dim3(256), 0, c.stream, q, qmax,
                           c.body_off, c.blk_off, (int)c.bodies.size(), c.N, c.nblk, groups, q16);
        AXS_HIP(hipGetLastError());
        const float k2pi = (float)(c.kappa / (2.0 * M_PI));
        const float s2 = k2pi * k2pi;
        const float gscale = std::ldexp(1.0f, c.mf16_gexp);
        const float etap_s = (float)(c.eta * c.kappa / (2.0 * M_PI)) * gscale;
        const auto *sop = (const f32x4 *)c.mf_src;
        const auto *q16v = (const h8 *)q16;
#define AXS_MF16(G_)                                                                                         \
    if (s.tpt == G_)                                                                                        \
        hipLaunchKernelGGL((interbody_mfma16_kernel<G_>), dim3(nwork, groups), dim3(256), 0, c.stream, work, \
                           c.g32, sop, q16v, c.body_off, c.blk_off, (int)c.bodies.size(), c.frame32, c.N,    \
                           nrhs, c.nblk, s2, etap_s, gscale, c.mf16_gexp, qmax, part);
        AXS_MF16(1)
        AXS_MF16(2)
        AXS_MF16(4)
#undef AXS_MF16
        AXS_HIP(hipGetLastError());
    }
    if (16 * groups < nrhs) {
        int nwork = 0;
        IBShape s3 = s;
        s3.variant = 3;
        const IBWork *work = get_work(c, 1, 1, s3, Units::nodes, nwork);
        if (s.tpt == 1) launch_mf<float, 1>(c, work, nwork, q, nrhs, part, 16 * groups);
        else if (s.tpt == 2) launch_mf<float, 2>(c, work, nwork, q, nrhs, part, 16 * groups);
        else launch_mf<float, 4>(c, work, nwork, q, nrhs, part, 16 * groups);
    }
}

int64_t interbody_scratch_bytes(Ctx &c, int prec, int nrhs) {
    const int pi = prec == AXS_FP32 ? 1 : 0;
    const IBShape s = launch_shape(c, prec, nrhs);
    if (s.variant != 1 && s.variant != 2) return -1;
    auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t total = (int64_t)nrhs * c.N, e2 = prec == AXS_FP32 ? 8 : 16;
    int64_t bytes = r256(total * e2) + r256((int64_t)s.splits * total * e2);
    const int *key = c.ib_key[pi][0];
    const bool cached = c.ib_work[pi][0] && key[0] == s.tpt && key[1] == s.bs && key[2] == s.splits &&
                        key[3] == s.variant && key[4] == c.tgt_first && key[5] == c.tgt_count;
    if (!cached)
        bytes += r256((int64_t)build_work(c, ib_tile(s), s.splits, s.variant == 2 ? Units::rings : Units::nodes).size() *
                      (int64_t)sizeof(IBWork));
    return bytes;
}

void interbody_partials(Ctx &c, const void *sigma, int nrhs, int prec) {
    const int pi = prec == AXS_FP32 ? 1 : 0;
    const IBShape s = launch_shape(c, prec, nrhs);
    const int64_t total = (int64_t)nrhs * c.N;
    const int thr = 256;
    if (s.variant == 4) {
        float2 *q = (float2 *)c.scratch(WS_Q, total * sizeof(float2));
        float2 *part = (float2 *)c.scratch(WS_PART, (size_t)s.splits * total * sizeof(float2));
        hipLaunchKernelGGL(stage_density_kernel<float>, dim3(ceil_div(total, thr)), dim3(thr), 0,
                           c.stream, (const double2 *)sigma, c.g64 + 6 * c.N, c.N, total, q);
        AXS_HIP(hipGetLastError());
        launch_mf16(c, s, q, nrhs, part);
        return;
    }
    int nwork = 0;
    const IBWork *dwork = get_work(c, pi, s.variant == 3 ? 1 : 0, s,
                                   s.variant == 2 ? Units::rings : Units::nodes, nwork);
    if (prec == AXS_FP32) {
        float2 *q = (float2 *)c.scratch(WS_Q, total * sizeof(float2));
        float2 *part = (float2 *)c.scratch(WS_PART, (size_t)s.splits * total * sizeof(float2));
        hipLaunchKernelGGL(stage_density_kernel<float>, dim3(ceil_div(total, thr)), dim3(thr), 0,
                           c.stream, (const double2 *)sigma, c.g64 + 6 * c.N, c.N, total, q);
        AXS_HIP(hipGetLastError());
        dispatch_ib<float>(c, s, dwork, nwork, c.g32, c.cs32, c.ring_g32, c.frame32, q, nrhs, part);
    } else {
        double2 *q = (double2 *)c.scratch(WS_Q, total * sizeof(double2));
        double2 *part = (double2 *)c.scratch(WS_PART, (size_t)s.splits * total * sizeof(double2));
        hipLaunchKernelGGL(stage_density_kernel<double>, dim3(ceil_div(total, thr)), dim3(thr), 0,
                           c.stream, (const double2 *)sigma, c.g64 + 6 * c.N, c.N, total, q);
        AXS_HIP(hipGetLastError());
        dispatch_ib<double>(c, s, dwork, nwork, c.g64, c.cs64, c.ring_g64, c.frame64, q, nrhs, part);
    }
}

void interbody_reduce_to_c128(Ctx &c, void *y, int nrhs, int prec, bool add) {
    const int splits = interbody_splits(c, prec, nrhs);
    const int64_t total = (int64_t)nrhs * c.N;
    const int thr = 256;
    int64_t row0 = 0, row1 = c.N;
    if (c.tgt_count >= 0) {
        const auto &f = c.bodies[c.tgt_first], &l = c.bodies[c.tgt_first + c.tgt_count - 1];
        row0 = f.offset;
        row1 = l.offset + l.n;
    }
    if (prec == AXS_FP32)
        hipLaunchKernelGGL(reduce_parts_kernel<float>, dim3(ceil_div(total, thr)), dim3(thr), 0, c.stream,
                           (const float2 *)c.scratch(WS_PART, 0), splits, total, add ? 1 : 0, (double2 *)y, c.N,
                           row0, row1);
    else
        hipLaunchKernelGGL(reduce_parts_kernel<double>, dim3(ceil_div(total, thr)), dim3(thr), 0, c.stream,
                           (const double2 *)c.scratch(WS_PART, 0), splits, total, add ? 1 : 0, (double2 *)y, c.N,
                           row0, row1);
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
                                                        double kappa, double gam_re, double gam_im,
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
        // 4 pi G = e^{ikR}/R [a (1 - i k R) + gamma], a = n.d / R^2
        const double a = nd / r2, are = a + gam_re, bim = gam_im - a * kappa * R;
        const double er = cs / R, ei = s / R;
        const double gr = er * are - ei * bim, gi = er * bim + ei * are;
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
                       (const double2 *)sigma, tgt_dev, nt, c.kappa, c.gam_re, c.gam_im, (double2 *)u);
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
