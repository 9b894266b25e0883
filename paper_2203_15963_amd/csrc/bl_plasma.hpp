// bl_plasma.hpp -- grid sampling, plasma state, thermal synchrotron
// coefficients and the fluid-frame tetrad on the device.
//
// Paper section 2.4 (Sampling): primitives rho, p, normal-frame velocity and
// B^a are interpolated, nearest-cell or trilinear within one block (blocks
// carry no ghost zones, so corner indices are clamped to the block: values are
// held constant within half a cell of a block face).  Section 2.5
// (Coefficients): n_e = rho/(mu m_p) (1 + 1/(n_e/n_i))^-1, T_i/T_e from
// R_high/R_low and beta, sigma > sigma_max is vacuum, U coefficients vanish in
// the rotated frame.  The thermal fitting formulas the paper takes from
// Marszewski et al. (2021) are not printed there; this file uses the thermal
// set of Dexter (2016) for the emissivities and of Shcherbakov (2008) for the
// rotativities, with absorptivities from Kirchhoff's law alpha = j / B_nu.
#pragma once

#include "bl_kerr.hpp"

namespace bl {

// ---------------------------------------------------------------- lookup
// Block holding x: the table maps a cell of the finest block lattice to the
// leaf block covering it (half-open boxes, so faces belong to the upper block).
__device__ __forceinline__ int find_block(const DevGrid &g, const double x[3]) {
    int idx[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = (x[d] - g.t0[d]) / g.tb[d];
        if (!(u >= 0.0) || u >= (double)g.tn[d]) return -1;
        idx[d] = (int)floor(u);
        if (idx[d] >= g.tn[d]) return -1;
    }
    return g.table[(idx[2] * g.tn[1] + idx[1]) * g.tn[0] + idx[0]];
}

template <typename T>
__device__ __forceinline__ void load_cell(const T *base, long long off, double acc[8], double wt) {
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] += wt * (double)base[off * 8 + m];
}

// Interpolated primitives at x; returns the block id or -1 (vacuum).
__device__ __forceinline__ int sample_grid(const DevGrid &g, int interp, const double x[3], double prim[8]) {
    int b = find_block(g, x);
    if (b < 0) return -1;
    const double *bm = g.bmeta + 6 * b;
    int nn[3] = {g.bnx, g.bny, g.bnz};
    int i0[3];
    double w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (interp) {
            double u = (x[d] - bm[d]) / bm[3 + d] - 0.5;
            double fl = floor(u);
            i0[d] = (int)fl;
            w[d] = u - fl;
            if (i0[d] < 0) { i0[d] = 0; w[d] = 0.0; }
            if (i0[d] > nn[d] - 2) { i0[d] = nn[d] - 2; w[d] = 1.0; }
        } else {
            int ii = (int)floor((x[d] - bm[d]) / bm[3 + d]);
            ii = ii < 0 ? 0 : (ii > nn[d] - 1 ? nn[d] - 1 : ii);
            i0[d] = ii;
            w[d] = 0.0;
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) prim[m] = 0.0;
    long long bbase = (long long)b * g.bnx * g.bny * g.bnz;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                double wt = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                if (wt == 0.0) continue;
                long long off = bbase + ((long long)(i0[2] + dk) * g.bny + (i0[1] + dj)) * g.bnx + (i0[0] + di);
                if (g.dtype == 0)
                    load_cell((const double *)g.prims, off, prim, wt);
                else
                    load_cell((const float *)g.prims, off, prim, wt);
            }
    return b;
}

// Does the chord from p to q (spatial components 1..3) meet the closed box?
__device__ __forceinline__ bool chord_meets_box(const double bb[6], const double *p, const double *q) {
    double t0 = 0.0, t1 = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double a0 = p[1 + d], dd = q[1 + d] - p[1 + d];
        if (dd == 0.0) {
            if (a0 < bb[2 * d] || a0 > bb[2 * d + 1]) return false;
        } else {
            double ta = (bb[2 * d] - a0) / dd, tb = (bb[2 * d + 1] - a0) / dd;
            double lo = fmin(ta, tb), hi = fmax(ta, tb);
            t0 = fmax(t0, lo);
            t1 = fmin(t1, hi);
            if (t0 > t1) return false;
        }
    }
    return true;
}

// ---------------------------------------------------------------- Bessel
// Ratios K0(x)/K2(x) and K1(x)/K2(x).  For x <= 2 the ascending series
// K0 = -(ln(x/2) + gamma) I0 + sum_k H_k y^k/(k!)^2 and
// K1 = 1/x + (x/2) [(ln(x/2) + gamma) sum_k y^k/(k!(k+1)!) - 1/2 sum_k (H_k + H_k+1) y^k/(k!(k+1)!)]
// with y = x^2/4 (Abramowitz & Stegun 9.6.11, 9.6.13); for x > 2 the
// trapezoid rule on e^x K_n(x) = int_0^inf exp(-x (cosh t - 1)) cosh(n t) dt
// with step min(0.15, 0.5/sqrt(x)), exponentially convergent.
// K2 = K0 + (2/x) K1 in the series branch.
__device__ __forceinline__ void bessel_ratios(double x, double &r0, double &r1) {
    double K0, K1, K2;
    if (x <= 2.0) {
        double y = 0.25 * x * x;
        double L = log(0.5 * x) + kEulerGamma;
        double t0 = 1.0, t1 = 1.0, H = 0.0;
        double I0 = 1.0, S0 = 0.0, A = 1.0, S1 = 1.0;   // k = 0 terms (H_0 = 0, H_1 = 1)
#pragma unroll
        for (int kk = 1; kk < 16; ++kk) {
            // 1/k^2, 1/(k(k+1)), 1/k, 1/(k+1) fold to constants after unrolling
            const double k = (double)kk;
            t0 *= y * (1.0 / (k * k));
            t1 *= y * (1.0 / (k * (k + 1.0)));
            H += 1.0 / k;
            double Hn = H + 1.0 / (k + 1.0);
            I0 += t0;
            S0 += H * t0;
            A += t1;
            S1 += (H + Hn) * t1;
        }
        K0 = -L * I0 + S0;
        K1 = 1.0 / x + 0.5 * x * (L * A - 0.5 * S1);
        K2 = K0 + 2.0 / x * K1;
    } else {
        double hq = fmin(0.15, 0.5 / sqrt(x));
        double s0 = 0.5, s1 = 0.5, s2 = 0.5;
        for (int i = 1; i < 400; ++i) {
            double t = i * hq;
            double em = expm1(t);
            double cm = em * em / (2.0 * (1.0 + em));   // cosh t - 1
            double c = 1.0 + cm;
            double wgt = exp(-x * cm);
            s0 += wgt;
            s1 += wgt * c;
            s2 += wgt * (2.0 * c * c - 1.0);
            if (x * cm - 2.0 * t > 40.0 && t > 1.0) break;
        }
        K0 = s0;
        K1 = s1;
        K2 = s2;
    }
    r0 = K0 / K2;
    r1 = K1 / K2;
}

// ------------------------------------------------------- thermal coefficients
// Fluid-frame coefficients at frequency nu (Hz) for electron density ne,
// temperature Theta_e, field B (gauss), and cos(theta_B):
// out = jI, jQ, jV, aI, aQ, aV, rQ, rV.
__device__ __forceinline__ void thermal_coeffs(double ne, double th, double B, double nu, double cth,
                                               int polarized, double out[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) out[m] = 0.0;
    cth = fmin(1.0, fmax(-1.0, cth));
    double sth = sqrt(1.0 - cth * cth);
    if (!(ne > 0.0) || !(th > 0.0) || !(B > 0.0) || !(sth > 0.0)) return;
    const double e2 = kQe * kQe;
    double nuB = kQe * B / (2.0 * kPi * kMe * kC);
    double nuc = 1.5 * nuB * sth * th * th;
    double x = nu / nuc;
    double x13 = cbrt(x);
    double xm13 = 1.0 / x13;
    double xm23 = xm13 * xm13;
    double E = exp(-1.8899 * x13);
    double pre = ne * e2 * nu / (2.0 * sqrt(3.0) * kC * th * th);
    double jI = pre * 2.5651 * (1.0 + 1.92 * xm13 + 0.9977 * xm23) * E;
    double Bnu = 2.0 * kH * nu * nu * nu / (kC * kC) / expm1(kH * nu / (th * kMe * kC * kC));
    out[0] = jI;
    out[3] = jI / Bnu;
    if (!polarized) return;
    double jQ = pre * 2.5651 * (1.0 + 0.932 * xm13 + 0.4998 * xm23) * E;
    double jV = 2.0 * ne * e2 * nu * (cth / sth) / (3.0 * sqrt(3.0) * kC * th * th * th) *
                (1.8138 / x + 3.423 * xm23 + 0.02955 / sqrt(x) + 2.0377 * xm13) * E;
    out[1] = jQ;
    out[2] = jV;
    out[4] = jQ / Bnu;
    out[5] = jV / Bnu;
    double Xr = th * sqrt(sqrt(2.0) * sth * 1.0e3 * nuB / nu);
    double r0, r1;
    bessel_ratios(1.0 / th, r0, r1);
    // powers of X through one logarithm: X^-1/2, X^-0.5175, X^-0.6, X^4/3
    double lX = log(Xr);
    double ism = exp(-0.5 * lX);
    double e169 = 0.011 * exp(-1.69 * ism);
    double f0 = 2.011 * exp(-19.78 * exp(-0.5175 * lX)) - cos(39.89 * ism) * exp(-70.16 * exp(-0.6 * lX)) - e169;
    double fm = f0 + (e169 - 0.003135 * exp((4.0 / 3.0) * lX)) * 0.5 * (1.0 + tanh(10.0 * (log(0.6648) - 0.5 * lX)));
    double gX = 1.0 - 0.11 * log1p(0.035 * Xr);
    double base = ne * e2 / (kMe * kC);
    out[6] = base * nuB * nuB * sth * sth / (nu * nu * nu) * fm * (r1 + 6.0 * th);
    out[7] = 2.0 * base * nuB / (nu * nu) * r0 * cth * gX;
}

// -------------------------------------------------------------- plasma
struct Sample {
    bool plasma;          // emitting plasma (else vacuum)
    double c[8];          // invariant coefficients jI, jQ, jV, aI, aQ, aV, rQ, rV
    double u[4], b[4];    // fluid 4-velocity and magnetic 4-vector (contravariant)
    double ne, th, B, nu_fl, sigma;
};

// Plasma state and invariant coefficients at state y = (x^mu, k_mu) for a ray
// of normalisation n (paper sections 2.4, 2.5):
//   u^t = gamma/alpha, u^a = u~^a - gamma beta^a/alpha,
//   b^t = B^a u_a, b^a = (B^a + b^t u^a)/u^t, sigma = b^2/rho,
//   beta^-1 = b^2/(2p), nu_fl = n (-k.u), cos(theta_B) = k.b/((-k.u)|b|),
// invariants j/nu_fl^2, alpha nu_fl, rho nu_fl.
__device__ __forceinline__ void sample_point(double a, int flat, const DevGrid &g, const PlasmaParams &pp,
                                             const double y[8], double n_norm, Sample &s) {
    s.plasma = false;
    s.sigma = 0.0;
    s.ne = s.th = s.B = s.nu_fl = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) s.c[m] = 0.0;
    double prim[8];
    if (sample_grid(g, pp.interp, y + 1, prim) < 0) return;
    double rho = prim[0], p = prim[1];
    if (!(rho > 0.0)) return;
    KS k = ks_point(a, flat, y[1], y[2], y[3]);
    double ut[3] = {prim[2], prim[3], prim[4]};
    velocity_from_normal(k, ut, s.u);
    double ul[4];
    lower(k, s.u, ul);
    double bt = prim[5] * ul[1] + prim[6] * ul[2] + prim[7] * ul[3];
    s.b[0] = bt;
#pragma unroll
    for (int c = 0; c < 3; ++c) s.b[1 + c] = (prim[5 + c] + bt * s.u[1 + c]) / s.u[0];
    double b2 = gdot(k, s.b, s.b);
    s.sigma = b2 / rho;
    if (s.sigma > pp.sigma_max) return;
    double binv = b2 / (2.0 * p);
    double ne = rho * g.rho_unit / (pp.mu * kMp) / (1.0 + 1.0 / pp.ne_ni);
    double tr = (pp.r_high + binv * binv * pp.r_low) / (1.0 + binv * binv);
    double th = pp.mu * kMp / kMe * (p / rho) * (pp.ne_ni + 1.0) / (pp.ne_ni + tr);
    double Bg = sqrt(b2) * kC * sqrt(4.0 * kPi * g.rho_unit);
    double omega = -(y[4] * s.u[0] + y[5] * s.u[1] + y[6] * s.u[2] + y[7] * s.u[3]);
    double kb = y[4] * s.b[0] + y[5] * s.b[1] + y[6] * s.b[2] + y[7] * s.b[3];
    double nu = n_norm * omega;
    double cth = (b2 > 0.0) ? kb / (omega * sqrt(b2)) : 0.0;
    double co[8];
    thermal_coeffs(ne, th, Bg, nu, cth, pp.polarized, co);
    double inu2 = 1.0 / (nu * nu);
#pragma unroll
    for (int m = 0; m < 3; ++m) s.c[m] = co[m] * inu2;
#pragma unroll
    for (int m = 3; m < 8; ++m) s.c[m] = co[m] * nu;
    s.ne = ne;
    s.th = th;
    s.B = Bg;
    s.nu_fl = nu;
    s.plasma = true;
}

// 3x3 determinant of rows (a1 a2 a3), (b1 b2 b3), (c1 c2 c3)
__device__ __forceinline__ double det3(double a1, double a2, double a3, double b1, double b2, double b3,
                                       double c1, double c2, double c3) {
    return a1 * (b2 * c3 - b3 * c2) - a2 * (b1 * c3 - b3 * c1) + a3 * (b1 * c2 - b2 * c1);
}

// Orthonormal tetrad of observer u with photon momentum k (covariant kc):
// e0 = u, e3 = (k - omega u)/omega with omega = -k.u, e2 along w projected
// orthogonal to u and e3 (falling back to z, then x, when w is degenerate),
// e1^a = [a b c d] u_b e2_c e3_d (sqrt(-g) = 1 in CKS): e1 x e2 = e3.
__device__ __forceinline__ void tetrad(const KS &k, const double u[4], const double kc[4], const double w[4],
                                       double e[4][4]) {
    double ku[4];
    raise(k, kc, ku);
    double omega = -(kc[0] * u[0] + kc[1] * u[1] + kc[2] * u[2] + kc[3] * u[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        e[0][m] = u[m];
        e[3][m] = (ku[m] - omega * u[m]) / omega;
    }
    double t[4], nrm = 0.0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        double v[4];
        if (attempt == 0) {
            v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; v[3] = w[3];
        } else if (attempt == 1) {
            v[0] = 0.0; v[1] = 0.0; v[2] = 0.0; v[3] = 1.0;
        } else {
            v[0] = 0.0; v[1] = 1.0; v[2] = 0.0; v[3] = 0.0;
        }
        double vn = sqrt(fabs(gdot(k, v, v)));
        double wu = gdot(k, v, u), we3 = gdot(k, v, e[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) t[m] = v[m] + wu * u[m] - we3 * e[3][m];
        nrm = sqrt(fabs(gdot(k, t, t)));
        if (vn > 0.0 && nrm > 1e-10 * vn) break;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) e[2][m] = t[m] / nrm;
    double U[4], P[4], Q[4];
    lower(k, u, U);
    lower(k, e[2], P);
    lower(k, e[3], Q);
    e[1][0] = det3(U[1], U[2], U[3], P[1], P[2], P[3], Q[1], Q[2], Q[3]);
    e[1][1] = -det3(U[0], U[2], U[3], P[0], P[2], P[3], Q[0], Q[2], Q[3]);
    e[1][2] = det3(U[0], U[1], U[3], P[0], P[1], P[3], Q[0], Q[1], Q[3]);
    e[1][3] = -det3(U[0], U[1], U[2], P[0], P[1], P[2], Q[0], Q[1], Q[2]);
}

}  // namespace bl
