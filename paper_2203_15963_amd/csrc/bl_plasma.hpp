// bl_plasma.hpp -- grid sampling, plasma state, thermal synchrotron
// coefficients and the fluid-frame tetrad on the device.
//
// Paper section 2.5 (Sampling): primitives rho, p, normal-frame velocity and
// B^a are interpolated, nearest-cell or trilinear within one block (blocks
// carry no ghost zones, so corner indices are clamped to the block: values are
// held constant within half a cell of a block face).  Section 2.6
// (Coefficients): n_e = rho/(mu m_p) (1 + 1/(n_e/n_i))^-1, T_i/T_e from
// R_high/R_low and beta, sigma > sigma_max is vacuum, U coefficients vanish in
// the rotated frame.  The thermal fitting formulas the paper takes from
// Marszewski et al. (2021) are not printed there; this file uses the thermal
// set of Dexter (2016) for the emissivities and of Shcherbakov (2008) for the
// rotativities, with absorptivities from Kirchhoff's law alpha = j / B_nu.
//
// Everything after the block lookup is a template on the real type R (double
// for the plain form, float for the mixed form); constants are grouped so
// that no intermediate leaves the float range.
#pragma once

#include "bl_kerr.hpp"

namespace bl {

// ---------------------------------------------------------------- lookup
// Index of the block lattice cell holding x (half-open boxes, so faces
// belong to the upper block), or -1 outside the lattice.
__device__ __forceinline__ long long lattice_cell(const DevGrid &g, const double x[3]) {
    int idx[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = (x[d] - g.t0[d]) * g.itb[d];
        if (!(u >= 0.0) || u >= (double)g.tn[d]) return -1;
        idx[d] = (int)floor(u);
        if (idx[d] >= g.tn[d]) return -1;
    }
    return (long long)((idx[2] * g.tn[1] + idx[1]) * g.tn[0] + idx[0]);
}

// The table entry of the lattice cell of the previous sample, kept by the
// FP64 walk (one wave per SIMD, registers to spare): consecutive samples
// mostly share a lattice cell (a cell is a block of the finest level), and
// the entry's load is then one dependent round trip fewer.  Entries are a
// function of the cell alone, so the choice of block is the table's.
struct BlockCache {
    long long cell;   // lattice cell of the entry held, -1: none
    double o[3], is[3];
    long long cb;
};

// Cells hold 8 primitives (32 or 64 contiguous bytes, 16-byte aligned) and
// are read with 16-byte vector loads.
typedef float gf4 __attribute__((ext_vector_type(4)));
typedef double gd2 __attribute__((ext_vector_type(2)));

// A table entry: the block's origin, inverse cell sizes and first cell
// (negative: no block), in four 16-byte loads.
__device__ __forceinline__ long long block_meta(const double *e, double o[3], double is[3]) {
    const gd2 *p = reinterpret_cast<const gd2 *>(e);
    const gd2 m0 = p[0], m1 = p[1], m2 = p[2], m3 = p[3];
    o[0] = m0[0];
    o[1] = m0[1];
    o[2] = m1[0];
    is[0] = m1[1];
    is[1] = m2[0];
    is[2] = m2[1];
    return (long long)m3[0];
}

// Trilinear weights of the eight corners, corner q = (di, dj, dk) = (q & 1, (q >> 1) & 1, q >> 2).
template <typename R>
__device__ __forceinline__ void corner_weights(const R w[3], R wt[8]) {
    const R x0 = R(1) - w[0], y0 = R(1) - w[1], z0 = R(1) - w[2];
    const R wxy[4] = {x0 * y0, w[0] * y0, x0 * w[1], w[0] * w[1]};
#pragma unroll
    for (int q = 0; q < 8; ++q) wt[q] = wxy[q & 3] * ((q >> 2) ? w[2] : z0);
}

// Weighted sum of the eight corner cells of cell c0 (strides 1, sy, sz).  The
// corners are read in groups of G whose loads are all issued before any is
// used, so a lane waits for one round trip per group instead of one per
// corner (G = 4 for the FP32 grid, 2 for the FP64 grid in the mixed form: 32
// registers of cell data in flight either way; 4 for the FP64 grid in the
// all-FP64 form, and all 8 in its polarized walk, which runs one wave per SIMD
// with registers to spare and has round trips to hide).
template <int G, typename T, typename R>
__device__ __forceinline__ void trilerp(const T *base, long long c0, long long sy, long long sz, const R w[3],
                                        R prim[8]) {
    typedef T tv __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int NV = 8 * sizeof(T) / 16;   // vectors per cell
    constexpr int NE = 16 / sizeof(T);       // elements per vector
    R wt[8];
    corner_weights(w, wt);
#pragma unroll
    for (int g0 = 0; g0 < 8; g0 += G) {
        tv v[G][NV];
#pragma unroll
        for (int qq = 0; qq < G; ++qq) {
            const int q = g0 + qq;
            const tv *p = reinterpret_cast<const tv *>(base + (c0 + (q >> 2) * sz + ((q >> 1) & 1) * sy + (q & 1)) * 8);
#pragma unroll
            for (int k = 0; k < NV; ++k) v[qq][k] = p[k];
        }
#pragma unroll
        for (int qq = 0; qq < G; ++qq)
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int e = 0; e < NE; ++e) prim[k * NE + e] += wt[g0 + qq] * (R)v[qq][k][e];
    }
}

// Interpolated primitives at x; returns false outside every block (vacuum).
// Block search and cell location in double, weights and accumulation in R.  Blocks
// have at least two cells per axis (checked when the grid is made), so the
// clamped corner indices i0, i0 + 1 always lie inside the block and all eight
// corners are read, those of weight zero included.
// WIDE: the one-wave-per-SIMD FP64 polarized walk (all eight corners at once,
// block entry from bc when the lattice cell is the previous sample's).
template <typename R, bool WIDE = false>
__device__ __forceinline__ bool sample_grid(const DevGrid &g, int interp, const double x[3], R prim[8],
                                            BlockCache *bc = nullptr) {
    const long long cell = lattice_cell(g, x);
    if (cell < 0) return false;
    double o[3], is[3];
    long long cb;
    if (WIDE && bc->cell == cell) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[d] = bc->o[d];
            is[d] = bc->is[d];
        }
        cb = bc->cb;
    } else {
        cb = block_meta(g.table + 8 * cell, o, is);
        if (WIDE) {
            bc->cell = cell;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                bc->o[d] = o[d];
                bc->is[d] = is[d];
            }
            bc->cb = cb;
        }
    }
    if (cb < 0) return false;
    const int nn[3] = {g.bnx, g.bny, g.bnz};
#pragma unroll
    for (int m = 0; m < 8; ++m) prim[m] = R(0);
    const long long sy = g.bnx, sz = (long long)g.bny * g.bnx;
    if (!interp) {
        int i0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int ii = (int)floor((x[d] - o[d]) * is[d]);
            i0[d] = ii < 0 ? 0 : (ii > nn[d] - 1 ? nn[d] - 1 : ii);
        }
        const long long c0 = cb + i0[2] * sz + i0[1] * sy + i0[0];
        if (g.dtype != 0) {
            const gf4 *p = reinterpret_cast<const gf4 *>((const float *)g.prims + c0 * 8);
            const gf4 v0 = p[0], v1 = p[1];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                prim[m] = (R)v0[m];
                prim[4 + m] = (R)v1[m];
            }
        } else {
            const gd2 *p = reinterpret_cast<const gd2 *>((const double *)g.prims + c0 * 8);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const gd2 v = p[k];
                prim[2 * k] = (R)v[0];
                prim[2 * k + 1] = (R)v[1];
            }
        }
        return true;
    }
    int i0[3];
    R w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = (x[d] - o[d]) * is[d] - 0.5;
        const double fl = floor(u);
        const int i = (int)fl;
        const R wd = (R)(u - fl);
        const bool lo = i < 0, hi = i > nn[d] - 2;
        i0[d] = lo ? 0 : (hi ? nn[d] - 2 : i);
        w[d] = lo ? R(0) : (hi ? R(1) : wd);
    }
    const long long c0 = cb + i0[2] * sz + i0[1] * sy + i0[0];
    if (g.dtype != 0)
        trilerp<4>((const float *)g.prims, c0, sy, sz, w, prim);
    else
        trilerp<sizeof(R) == 8 ? (WIDE ? 8 : 4) : 2>((const double *)g.prims, c0, sy, sz, w, prim);
    return true;
}

// ---------------------------------------------------------------- Bessel
// Ratios K0(x)/K2(x) and K1(x)/K2(x).  For x <= 2 the ascending series
// K0 = -(ln(x/2) + gamma) I0 + sum_k H_k y^k/(k!)^2 and
// K1 = 1/x + (x/2) [(ln(x/2) + gamma) sum_k y^k/(k!(k+1)!) - 1/2 sum_k (H_k + H_k+1) y^k/(k!(k+1)!)]
// with y = x^2/4 (Abramowitz & Stegun 9.6.11, 9.6.13), K2 = K0 + (2/x) K1;
// for x > 2 in FP64 the trapezoid rule on e^x K_n(x) = int_0^inf
// exp(-x (cosh t - 1)) cosh(n t) dt, exponentially convergent in the step; for
// x > 2 in FP32 the polynomials in 2/x for sqrt(x) e^x K0(x) and
// sqrt(x) e^x K1(x) of Abramowitz & Stegun 9.8.6 and 9.8.8 (absolute errors
// below 1.9e-7 and 2.2e-7 on values near 1.25, a few FP32 ulp; the factor
// sqrt(x) e^x cancels in the ratios), with K2 again from the recurrence.
// Terms and steps are sized for the precision of R.
template <typename R>
__device__ __forceinline__ void bessel_ratios(R x, R ix, R &r0, R &r1) {   // ix = 1/x
    constexpr bool dbl = sizeof(R) == 8;
    constexpr int nterms = dbl ? 16 : 9;
    R K0, K1, K2;
    if (x <= R(2)) {
        R y = R(0.25) * x * x;
        R L = flog(R(0.5) * x) + R(kEulerGamma);
        R t0 = R(1), t1 = R(1), H = R(0);
        R I0 = R(1), S0 = R(0), A = R(1), S1 = R(1);   // k = 0 terms (H_0 = 0, H_1 = 1)
#pragma unroll
        for (int kk = 1; kk < nterms; ++kk) {
            // 1/k^2, 1/(k(k+1)), 1/k, 1/(k+1) fold to constants after unrolling
            const double k = (double)kk;
            t0 *= y * R(1.0 / (k * k));
            t1 *= y * R(1.0 / (k * (k + 1.0)));
            H += R(1.0 / k);
            R Hn = H + R(1.0 / (k + 1.0));
            I0 += t0;
            S0 += H * t0;
            A += t1;
            S1 += (H + Hn) * t1;
        }
        K0 = -L * I0 + S0;
        K1 = ix + R(0.5) * x * (L * A - R(0.5) * S1);
        K2 = K0 + R(2) * ix * K1;
    } else if constexpr (!dbl) {
        const R t = R(2) * ix;
        K0 = R(1.25331414) +
             t * (R(-0.07832358) +
                  t * (R(0.02189568) +
                       t * (R(-0.01062446) + t * (R(0.00587872) + t * (R(-0.00251540) + t * R(0.00053208))))));
        K1 = R(1.25331414) +
             t * (R(0.23498619) +
                  t * (R(-0.03655620) +
                       t * (R(0.01504268) + t * (R(-0.00780353) + t * (R(0.00325614) + t * R(-0.00068245))))));
        K2 = K0 + ix * R(2) * K1;
    } else {
        R hq = fmin(R(0.15), R(0.5) * rsqrt_r(x));
        const R stop = R(40);
        R s0 = R(0.5), s1 = R(0.5), s2 = R(0.5);
        for (int i = 1; i < 400; ++i) {
            R t = (R)i * hq;
            R em = fexpm1(t);
            R cm = fdiv(em * em, R(2) * (R(1) + em));   // cosh t - 1
            R c = R(1) + cm;
            R wgt = fexp(-x * cm);
            s0 += wgt;
            s1 += wgt * c;
            s2 += wgt * (R(2) * c * c - R(1));
            if (x * cm - R(2) * t > stop && t > R(1)) break;
        }
        K0 = s0;
        K1 = s1;
        K2 = s2;
    }
    const R iK2 = fdiv(R(1), K2);
    r0 = K0 * iK2;
    r1 = K1 * iK2;
}

// ------------------------------------------------------- thermal coefficients
// Constants of the fits, grouped so that no intermediate leaves float range.
constexpr double kNuB = kQe / (2.0 * kPi * kMe * kC);            // nu_B per gauss
constexpr double kPreI = kQe * kQe / (2.0 * 1.7320508075688772 * kC);
constexpr double kPreV = 2.0 * kQe * kQe / (3.0 * 1.7320508075688772 * kC);
constexpr double kPlanck9 = 2.0 * kH / (kC * kC) * 1e27;         // 2h/c^2 (1e9 Hz)^3
constexpr double kHoverMec2 = kH / (kMe * kC * kC);
constexpr double kRotBase = kQe * kQe / (kMe * kC);

// Fluid-frame coefficients at frequency nu (Hz) for electron density ne,
// temperature Theta_e, field B (gauss), and cos(theta_B):
// out = jI, jQ, jV, aI, aQ, aV, rQ, rV (CGS).
// The reciprocals 1/nu, 1/Theta_e, 1/sin(theta_B) and the powers of
// x = nu/nu_c are formed once (x^1/3 from one logarithm and exponential, its
// reciprocal and 1/sqrt(x) without further transcendentals).
template <typename R>
__device__ __forceinline__ void thermal_coeffs(R ne, R th, R B, R nu, R cth, int polarized, R out[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) out[m] = R(0);
    cth = fmin(R(1), fmax(R(-1), cth));
    R sth = sqrt(R(1) - cth * cth);
    if (!(ne > R(0)) || !(th > R(0)) || !(B > R(0)) || !(sth > R(0))) return;
    const R inu = fdiv(R(1), nu), ith = fdiv(R(1), th);
    const R nuB = R(kNuB) * B;
    const R x = fdiv(nu, R(1.5) * nuB * sth * th * th);
    const R x13 = fexp(flog(x) * R(1.0 / 3.0));
    const R xm13 = fdiv(R(1), x13);
    const R xm23 = xm13 * xm13;
    const R E = fexp(R(-1.8899) * x13);
    const R pre = (ne * R(kPreI)) * nu * (ith * ith);
    const R jI = pre * R(2.5651) * (R(1) + R(1.92) * xm13 + R(0.9977) * xm23) * E;
    // 1/B_nu = (e^{h nu/kT} - 1) / (2 h nu^3/c^2), nu in units of 1e9 Hz
    const R inu9 = R(1e9) * inu;
    const R iB = fexpm1(R(kHoverMec2) * nu * ith) * (R(1.0 / kPlanck9) * inu9 * inu9 * inu9);
    out[0] = jI;
    out[3] = jI * iB;
    if (!polarized) return;
    const R jQ = pre * R(2.5651) * (R(1) + R(0.932) * xm13 + R(0.4998) * xm23) * E;
    const R ix = xm13 * xm13 * xm13, isx = rsqrt_r(x);
    const R jV = (ne * R(kPreV)) * nu * fdiv(cth, sth) * (ith * ith * ith) *
                 (R(1.8138) * ix + R(3.423) * xm23 + R(0.02955) * isx + R(2.0377) * xm13) * E;
    out[1] = jQ;
    out[2] = jV;
    out[4] = jQ * iB;
    out[5] = jV * iB;
    const R Xr = th * sqrt(R(1.4142135623730951) * sth * R(1e3) * nuB * inu);
    R r0, r1;
    bessel_ratios(ith, th, r0, r1);
    // powers of X through one logarithm: X^-1/2, X^-0.5175, X^-0.6, X^4/3
    const R lX = flog(Xr);
    const R ism = rsqrt_r(Xr);
    const R e169 = R(0.011) * fexp(R(-1.69) * ism);
    const R f0 = R(2.011) * fexp(R(-19.78) * fexp(R(-0.5175) * lX)) -
                 fcos(R(39.89) * ism) * fexp(R(-70.16) * fexp(R(-0.6) * lX)) - e169;
    // (1 + tanh y) / 2 = 1 / (1 + e^{-2y}), y = 10 (ln 0.6648 - lX / 2)
    const R fm = f0 + (e169 - R(0.003135) * fexp(R(4.0 / 3.0) * lX)) /
                          (R(1) + fexp(R(-20) * (R(-0.4082690354408987) - R(0.5) * lX)));
    const R gX = R(1) - R(0.11) * flog1p_abs(R(0.035) * Xr);
    const R base = ne * R(kRotBase);
    const R rb = nuB * inu;
    out[6] = base * rb * rb * sth * sth * inu * fm * (r1 + R(6) * th);
    out[7] = R(2) * base * rb * inu * r0 * cth * gX;
}

// ------------------------------------------------ nonthermal populations
// Synchrotron coefficients of the power-law and kappa electrons (paper
// sections 2.6 and 4.5; constants in NthParams), added to out.  The circular
// and rotative coefficients of these populations are zero.  The powers of X
// come from one logarithm; a bridge (low^-b + high^-b)^(-1/b) is evaluated
// on the logarithms of its two terms, scaled by the smaller one.
template <typename R>
__device__ __forceinline__ R nth_bridge(R ll, R lh, R b) {   // ll, lh: logs of low, high
    const R m = fmin(ll, lh);
    return fexp(m - flog(fexp(-b * (ll - m)) + fexp(-b * (lh - m))) * fdiv(R(1), b));
}

template <typename R>
__device__ __forceinline__ void nonthermal_coeffs(const NthParams &q, R ne, R B, R nu, R cth, int polarized,
                                                  R out[8]) {
    cth = fmin(R(1), fmax(R(-1), cth));
    const R sth = sqrt(R(1) - cth * cth);
    if (!(ne > R(0)) || !(B > R(0)) || !(sth > R(0))) return;
    const R nuc = R(kNuB) * B;
    const R lX = flog(fdiv(nu, nuc * sth));
    const R lsth = flog(sth);
    const R jn = ne * R(kQe * kQe / kC) * nuc;             // n_e e^2 nu_c / c
    const R an = fdiv(ne * R(kQe * kQe / (kMe * kC)), nu);   // n_e e^2 / (nu m c)
    for (int k = 0; k < 2; ++k) {
        const R f = (R)q.frac[1 + k];
        if (!(f > R(0))) continue;
        // power-law terms, as logarithms
        const R lhj = (R)q.lhj[k] + lsth + (R)q.ej[k] * lX;
        const R lha = (R)q.lha[k] + (R)q.ea[k] * lX;
        R jI, jQ, aI, aQ;
        if (k == 0) {
            jI = fexp(lhj);
            aI = fexp(lha);
            jQ = fexp(lhj + (R)q.lhjq[k]);
            aQ = fexp(lha + (R)q.lhaq[k]);
        } else {
            const R llj = (R)q.llj + lsth + lX * R(1.0 / 3.0);
            const R lla = (R)q.lla - lX * R(2.0 / 3.0);
            const R ln2 = R(0.6931471805599453);
            jI = nth_bridge(llj, lhj, R(0.5));
            aI = nth_bridge(lla, lha, R(3.0 / 7.0));
            jQ = nth_bridge(llj - ln2, lhj + (R)q.lhjq[k], R(0.5));
            aQ = nth_bridge(lla - ln2, lha + (R)q.lhaq[k], R(0.5));
        }
        out[0] += f * jn * jI;
        out[3] += f * an * aI;
        if (polarized) {
            out[1] += f * jn * jQ;
            out[4] += f * an * aQ;
        }
    }
}

// -------------------------------------------------------------- plasma
template <typename R>
struct Sample {
    bool plasma;          // emitting plasma (else vacuum)
    KS<R> k;              // metric functions at the sample point (set when the cell holds matter)
    R co[8];              // fluid-frame jI, jQ, jV, aI, aQ, aV, rQ, rV (CGS)
    R u[4], b[4];         // fluid 4-velocity and magnetic 4-vector (contravariant)
    R omega;              // -k.u for the unnormalised k
    R ne, th, B, nu_fl, sigma;
    R rho, p, binv;       // density and pressure (code units), beta^-1
};

// Plasma state and fluid-frame coefficients at state y = (x^mu, k_mu) for a
// ray of normalisation n (paper sections 2.5, 2.6):
//   u^t = gamma/alpha, u^a = u~^a - gamma beta^a/alpha,
//   b^t = B^a u_a, b^a = (B^a + b^t u^a)/u^t, sigma = b^2/rho,
//   beta^-1 = b^2/(2p), nu_fl = n (-k.u), cos(theta_B) = k.b/((-k.u)|b|).
// A quantity outside its cut limits (paper section 4.1, Data Cuts), compared
// in the arithmetic's own precision.
template <typename R>
__device__ __forceinline__ bool cut_out(const CutParams &c, int k, R q) {
    if constexpr (sizeof(R) == 4) return q < c.lo_f[k] || q > c.hi_f[k];
    else return q < c.lo[k] || q > c.hi[k];
}

// CUTS: compiled with the data-cut checks (renders with cuts installed use
// that instantiation, so the others carry no trace of them); NTH: with the
// nonthermal electron populations (likewise).
template <typename R, bool CUTS = false, bool NTH = false, bool WIDE = false>
__device__ __forceinline__ void sample_point(double a, int flat, const DevGrid &g, const PlasmaParams &pp,
                                             const double yd[8], double n_norm, Sample<R> &s,
                                             BlockCache *bc = nullptr) {
    s.plasma = false;
    s.sigma = R(0);
    s.ne = s.th = s.B = s.nu_fl = s.omega = R(0);
#pragma unroll
    for (int m = 0; m < 8; ++m) s.co[m] = R(0);
    R prim[8];
    if (!sample_grid<R, WIDE>(g, pp.interp, yd + 1, prim, bc)) return;
    R rho = prim[0], p = prim[1];
    if (!(rho > R(0))) return;
    s.k = ks_point<R>((R)a, flat, (R)yd[1], (R)yd[2], (R)yd[3]);
    const KS<R> &k = s.k;
    R ut[3] = {prim[2], prim[3], prim[4]};
    velocity_from_normal(k, ut, s.u);
    R ul[4];
    lower(k, s.u, ul);
    R bt = prim[5] * ul[1] + prim[6] * ul[2] + prim[7] * ul[3];
    s.b[0] = bt;
    R iut = fdiv(R(1), s.u[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c) s.b[1 + c] = (prim[5 + c] + bt * s.u[1 + c]) * iut;
    R b2 = gdot(k, s.b, s.b);
    s.sigma = fdiv(b2, rho);
    if (s.sigma > (R)pp.sigma_max) return;
    R binv = fdiv(b2, R(2) * p);
    R ne = rho * (R)pp.ne_per_rho;
    R tr = fdiv((R)pp.r_high + binv * binv * (R)pp.r_low, R(1) + binv * binv);
    R th = (R)pp.th_per_pr * fdiv(p, rho) * fdiv((R)(pp.ne_ni + 1.0), (R)pp.ne_ni + tr);
    R Bg = sqrt(b2) * (R)pp.gauss_per_b;
    if (CUTS && pp.cuts) {
        // an opaque copy of the pointer keeps the limit loads here: hoisted out
        // of the transfer's loop they would hold scalar registers throughout
        const CutParams *cp = pp.cut;
        asm volatile("" : "+s"(cp));
        const CutParams &c = *cp;
        const double d = (yd[1] - c.x0[0]) * c.n[0] + (yd[2] - c.x0[1]) * c.n[1] + (yd[3] - c.x0[2]) * c.n[2];
        if (cut_out<R>(c, kCutRho, rho) || cut_out<R>(c, kCutP, p) || cut_out<R>(c, kCutR, k.r) ||
            cut_out<R>(c, kCutNe, ne) || cut_out<R>(c, kCutThetaE, th) || cut_out<R>(c, kCutB, Bg) ||
            cut_out<R>(c, kCutSigma, s.sigma) || cut_out<R>(c, kCutBetaInv, binv) || (c.plane > 0 && d < 0.0) ||
            (c.plane < 0 && d > 0.0))
            return;
    }
    R kc[4] = {(R)yd[4], (R)yd[5], (R)yd[6], (R)yd[7]};
    R omega = -(kc[0] * s.u[0] + kc[1] * s.u[1] + kc[2] * s.u[2] + kc[3] * s.u[3]);
    R kb = kc[0] * s.b[0] + kc[1] * s.b[1] + kc[2] * s.b[2] + kc[3] * s.b[3];
    R nu = (R)n_norm * omega;
    R cth = (b2 > R(0)) ? fdiv(kb, omega * sqrt(b2)) : R(0);
    if (NTH && pp.nonthermal) {
        const NthParams *np = pp.nth;
        asm volatile("" : "+s"(np));
        thermal_coeffs<R>(ne * (R)np->frac[0], th, Bg, nu, cth, pp.polarized, s.co);
        nonthermal_coeffs<R>(*np, ne, Bg, nu, cth, pp.polarized, s.co);
    } else {
        thermal_coeffs<R>(ne, th, Bg, nu, cth, pp.polarized, s.co);
    }
    s.omega = omega;
    s.ne = ne;
    s.th = th;
    s.B = Bg;
    s.nu_fl = nu;
    s.rho = rho;
    s.p = p;
    s.binv = binv;
    s.plasma = true;
}

// Orthonormal tetrad of observer u with photon momentum k (covariant kc):
// e0 = u, e3 = (k - omega u)/omega with omega = -k.u, e2 along w projected
// orthogonal to u and e3 (falling back to z, then x, when w is degenerate),
// e1^a = [abcd] u_b e2_c e3_d (sqrt(-g) = 1 in CKS): e1 x e2 = e3.  Lowering
// every index of the alternating symbol multiplies it by det g = -1, so the
// covariant e1 is p_a = -[abcd] u^b e2^c e3^d, formed here from the
// contravariant vectors and raised once.  Returns the screen vectors e1, e2
// contravariant and p = e1_a, q = e2_a covariant, and e3.
// Every Stokes readout and repacking of the polarization state goes through
// e1 and e2, so a scale error of their norms compounds over the samples of a
// ray.  In FP32 the reciprocal of omega and the normalisation of e2 are
// therefore refined (rcp_acc, rsqrt_acc), and e1, which inherits the rounding
// of u, e2 and e3 through the cofactors, is normalised explicitly by
// (p.e1)^-1/2.  In FP64 the construction is exact to rounding as it stands.
template <typename R>
__device__ __forceinline__ void screen_basis(const KS<R> &k, const R u[4], const R kc[4], const R w[4], R e1[4],
                                             R e2[4], R p[4], R q[4], R e3[4]) {
    R ku[4];
    raise(k, kc, ku);
    const R omega = -(kc[0] * u[0] + kc[1] * u[1] + kc[2] * u[2] + kc[3] * u[3]);
    const R iom = sizeof(R) == 4 ? rcp_acc(omega) : fdiv(R(1), omega);
#pragma unroll
    for (int m = 0; m < 4; ++m) e3[m] = (ku[m] - omega * u[m]) * iom;
    R t[4], nrm2 = R(0);
    for (int attempt = 0; attempt < 3; ++attempt) {
        R v[4];
        if (attempt == 0) {
            v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; v[3] = w[3];
        } else if (attempt == 1) {
            v[0] = R(0); v[1] = R(0); v[2] = R(0); v[3] = R(1);
        } else {
            v[0] = R(0); v[1] = R(1); v[2] = R(0); v[3] = R(0);
        }
        R V[4];
        lower(k, v, V);
        const R vv = fabs(V[0] * v[0] + V[1] * v[1] + V[2] * v[2] + V[3] * v[3]);
        const R wu = V[0] * u[0] + V[1] * u[1] + V[2] * u[2] + V[3] * u[3];
        const R we3 = V[0] * e3[0] + V[1] * e3[1] + V[2] * e3[2] + V[3] * e3[3];
#pragma unroll
        for (int m = 0; m < 4; ++m) t[m] = v[m] + wu * u[m] - we3 * e3[m];
        nrm2 = fabs(gdot(k, t, t));
        if (vv > R(0) && nrm2 > R(1e-20) * vv) break;
    }
    const R inrm = sizeof(R) == 4 ? rsqrt_acc(nrm2) : rsqrt_r(nrm2);
#pragma unroll
    for (int m = 0; m < 4; ++m) e2[m] = t[m] * inrm;
    lower(k, e2, q);
    // the four 3x3 cofactors from the six 2x2 minors of (e2, e3)
    const R m01 = e2[0] * e3[1] - e2[1] * e3[0], m02 = e2[0] * e3[2] - e2[2] * e3[0];
    const R m03 = e2[0] * e3[3] - e2[3] * e3[0], m12 = e2[1] * e3[2] - e2[2] * e3[1];
    const R m13 = e2[1] * e3[3] - e2[3] * e3[1], m23 = e2[2] * e3[3] - e2[3] * e3[2];
    p[0] = -(u[1] * m23 - u[2] * m13 + u[3] * m12);
    p[1] = u[0] * m23 - u[2] * m03 + u[3] * m02;
    p[2] = -(u[0] * m13 - u[1] * m03 + u[3] * m01);
    p[3] = u[0] * m12 - u[1] * m02 + u[2] * m01;
    raise(k, p, e1);
    if constexpr (sizeof(R) == 4) {
        const R s1 = rsqrt_acc(fabs(p[0] * e1[0] + p[1] * e1[1] + p[2] * e1[2] + p[3] * e1[3]));
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            e1[m] *= s1;
            p[m] *= s1;
        }
    }
}

// The whole tetrad (rows e0..e3, contravariant).
template <typename R>
__device__ __forceinline__ void tetrad(const KS<R> &k, const R u[4], const R kc[4], const R w[4], R e[4][4]) {
    R p[4], q[4];
    screen_basis(k, u, kc, w, e[1], e[2], p, q, e[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m) e[0][m] = u[m];
}

}  // namespace bl
