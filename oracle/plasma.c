/*
 * plasma.c -- grid sampling, plasma state and thermal synchrotron
 * coefficients (oracle).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper sections 2.5 (Sampling) and 2.6 (Coefficients):
 *  - primitives rho, p, normal-frame u~, B^a are interpolated (nearest cell
 *    or trilinear within a block) and everything else derives from them;
 *  - b^alpha = u_beta (*F)^{beta alpha}: b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t;
 *    B = (b.b)^1/2, sigma = B^2/rho, beta^-1 = B^2/(2p);
 *  - n_e = rho/(mu m_p) (1 + 1/(n_e/n_i))^-1;
 *  - T_i/T_e = (R_high + beta^-2 R_low)/(1 + beta^-2),
 *    T_e = (mu m_p p/(k_B rho)) (n_e/n_i + 1)/(n_e/n_i + T_i/T_e);
 *  - sigma > sigma_max is vacuum (used for every simulation image);
 *  - the frame is rotated so that the U coefficients vanish.
 *
 * Readings (formulas and conventions the paper does not print):
 *  - cells are cell-centred; trilinear weights use the 8 nearest centres in
 *    the block, with corner indices clamped to the block (constant within
 *    half a cell of a block face); a point belongs to the block whose
 *    half-open box [x0,x1) x [y0,y1) x [z0,z1) holds it; outside all blocks,
 *    or rho <= 0, is vacuum;
 *  - code units: p_unit = rho_unit c^2, B_gauss = B_code c sqrt(4 pi rho_unit);
 *  - thermal fitting formulas (the paper cites Marszewski et al. 2021, not
 *    reproduced in it): the Dexter (2016) / Shcherbakov (2008) thermal set
 *    written out in thermal_coeffs() below, with alpha_A = j_A / B_nu
 *    (Kirchhoff).  Physical values are parity-unpinned;
 *  - invariants j/nu^2, alpha*nu, rho*nu at the fluid-frame frequency
 *    nu_fl = n (-k.u);
 *  - tetrad: e0 = u, e3 = (k - omega u)/omega with omega = -k.u,
 *    e2 along b projected orthogonal to e3, e1^a = [a b c d] u_b e2_c e3_d
 *    (sqrt(-g) = 1 in CKS); Q > 0 along e1 (perpendicular to the field).
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

#define C_LIGHT 2.99792458e10
#define G_NEWTON 6.67430e-8
#define M_SUN 1.98841e33
#define M_ELECTRON 9.1093837015e-28
#define M_PROTON 1.67262192369e-24
#define Q_ELECTRON 4.80320471e-10
#define H_PLANCK 6.62607015e-27
#define K_BOLTZMANN 1.380649e-16

int or_grid_sample(const or_grid *gr, int interp, const double x[3], double prim[8])
{
    int b, found = -1, m;
    for (b = 0; b < gr->n_blocks; ++b) {
        const double *bd = gr->bounds + 6 * b;
        if (x[0] >= bd[0] && x[0] < bd[1] && x[1] >= bd[2] && x[1] < bd[3]
            && x[2] >= bd[4] && x[2] < bd[5]) { found = b; break; }
    }
    if (found < 0) return -1;
    {
        const double *bd = gr->bounds + 6 * found;
        int nn[3] = {gr->bnx, gr->bny, gr->bnz};
        double w[3];
        int i0[3], d;
        const double *base = gr->prims + (size_t)found * gr->bnx * gr->bny * gr->bnz * 8;
        for (d = 0; d < 3; ++d) {
            double dx = (bd[2 * d + 1] - bd[2 * d]) / nn[d];
            if (interp) {
                double u = (x[d] - bd[2 * d]) / dx - 0.5;
                double fl = floor(u);
                i0[d] = (int)fl;
                w[d] = u - fl;
                if (i0[d] < 0) { i0[d] = 0; w[d] = 0.0; }
                if (i0[d] > nn[d] - 2) { i0[d] = nn[d] - 2; w[d] = 1.0; }
                if (nn[d] == 1) { i0[d] = 0; w[d] = 0.0; }
            } else {
                int ii = (int)floor((x[d] - bd[2 * d]) / dx);
                if (ii < 0) ii = 0;
                if (ii > nn[d] - 1) ii = nn[d] - 1;
                i0[d] = ii;
                w[d] = 0.0;
            }
        }
        for (m = 0; m < 8; ++m) prim[m] = 0.0;
        {
            int di, dj, dk;
            for (dk = 0; dk < 2; ++dk)
                for (dj = 0; dj < 2; ++dj)
                    for (di = 0; di < 2; ++di) {
                        double wt = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1])
                                  * (dk ? w[2] : 1.0 - w[2]);
                        int ii = i0[0] + di, jj = i0[1] + dj, kk = i0[2] + dk;
                        const double *cell;
                        if (wt == 0.0) continue;
                        cell = base + (((size_t)kk * gr->bny + jj) * gr->bnx + ii) * 8;
                        for (m = 0; m < 8; ++m) prim[m] += wt * cell[m];
                    }
        }
    }
    return found;
}

/* e^x K_n(x) = int_0^inf exp(-x (cosh t - 1)) cosh(n t) dt by the trapezoid
   rule, which converges exponentially for this analytic integrand: the step
   min(1/16, 1/(4 sqrt(x))) keeps the discretisation error far below double
   precision also when the integrand narrows to width ~ x^-1/2; summed until
   the integrand is below e^-50 of its scale. */
double or_bessel_k_scaled(int n, double x)
{
    const double hq = fmin(1.0 / 16.0, 0.25 / sqrt(x));
    double sum = 0.5, t;
    int i;
    for (i = 1;; ++i) {
        double term;
        t = i * hq;
        term = exp(-x * (cosh(t) - 1.0)) * cosh(n * t);
        sum += term;
        if (x * (cosh(t) - 1.0) - n * t > 50.0 && t > 1.0) break;
    }
    return sum * hq;
}

/* Thermal synchrotron coefficients in the fluid frame (CGS), Dexter (2016)
   emissivity fits with x = nu/nu_c, nu_c = 3/2 nu_B sin(theta) Theta_e^2,
   nu_B = e B/(2 pi m_e c); Faraday rotativities after Shcherbakov (2008)
   with X = Theta_e (sqrt(2) sin(theta) 1e3 nu_B/nu)^(1/2).
   out = jI, jQ, jV, aI, aQ, aV, rQ, rV. */
void or_thermal_coeffs(double ne, double thetae, double B, double nu,
                       double cos_theta, int polarized, double out[8])
{
    double sin_theta, nuB, nuc, x, E, pre, jI, jQ = 0, jV = 0, Bnu;
    int m;
    for (m = 0; m < 8; ++m) out[m] = 0.0;
    if (cos_theta > 1.0) cos_theta = 1.0;
    if (cos_theta < -1.0) cos_theta = -1.0;
    sin_theta = sqrt(1.0 - cos_theta * cos_theta);
    if (!(ne > 0.0) || !(thetae > 0.0) || !(B > 0.0) || !(sin_theta > 0.0)) return;
    nuB = Q_ELECTRON * B / (2.0 * M_PI * M_ELECTRON * C_LIGHT);
    nuc = 1.5 * nuB * sin_theta * thetae * thetae;
    x = nu / nuc;
    E = exp(-1.8899 * pow(x, 1.0 / 3.0));
    pre = ne * Q_ELECTRON * Q_ELECTRON * nu / (2.0 * sqrt(3.0) * C_LIGHT * thetae * thetae);
    jI = pre * 2.5651 * (1.0 + 1.92 * pow(x, -1.0 / 3.0) + 0.9977 * pow(x, -2.0 / 3.0)) * E;
    Bnu = 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT)
        / expm1(H_PLANCK * nu / (thetae * M_ELECTRON * C_LIGHT * C_LIGHT));
    out[0] = jI;
    out[3] = jI / Bnu;
    if (!polarized) return;
    jQ = pre * 2.5651 * (1.0 + 0.932 * pow(x, -1.0 / 3.0) + 0.4998 * pow(x, -2.0 / 3.0)) * E;
    jV = 2.0 * ne * Q_ELECTRON * Q_ELECTRON * nu * (cos_theta / sin_theta)
       / (3.0 * sqrt(3.0) * C_LIGHT * thetae * thetae * thetae)
       * (1.8138 / x + 3.423 * pow(x, -2.0 / 3.0) + 0.02955 * pow(x, -0.5)
          + 2.0377 * pow(x, -1.0 / 3.0)) * E;
    out[1] = jQ;
    out[2] = jV;
    out[4] = jQ / Bnu;
    out[5] = jV / Bnu;
    {
        double Xr = thetae * sqrt(sqrt(2.0) * sin_theta * 1.0e3 * nuB / nu);
        double k0 = or_bessel_k_scaled(0, 1.0 / thetae);
        double k1 = or_bessel_k_scaled(1, 1.0 / thetae);
        double k2 = or_bessel_k_scaled(2, 1.0 / thetae);
        double ism = pow(Xr, -0.5);
        double f0 = 2.011 * exp(-19.78 * pow(Xr, -0.5175))
                  - cos(39.89 * ism) * exp(-70.16 * pow(Xr, -0.6))
                  - 0.011 * exp(-1.69 * ism);
        double fm = f0 + (0.011 * exp(-1.69 * ism) - 0.003135 * pow(Xr, 4.0 / 3.0))
                  * 0.5 * (1.0 + tanh(10.0 * log(0.6648 * ism)));
        double gX = 1.0 - 0.11 * log(1.0 + 0.035 * Xr);
        double base = ne * Q_ELECTRON * Q_ELECTRON / (M_ELECTRON * C_LIGHT);
        out[6] = base * nuB * nuB * sin_theta * sin_theta / (nu * nu * nu) * fm
               * (k1 / k2 + 6.0 * thetae);
        out[7] = 2.0 * base * nuB / (nu * nu) * (k0 / k2) * cos_theta * gX;
    }
}

/* ------------------------------------------------ nonthermal electrons
 * Power-law and kappa distributions as defined in the paper (section 2.6):
 *   power law: dn/dgamma prop. gamma^-p on gmin <= gamma <= gmax;
 *   kappa:     dn/dgamma prop. gamma sqrt(gamma^2 - 1) (1 + (gamma - 1)/(kappa w))^(-kappa-1).
 * The paper takes their coefficients from fitting formulas it does not print.
 * Reading used here: the ultrarelativistic synchrotron coefficients of the
 * distribution, i.e. the emissivities j = (sqrt3 e^3 B sin(theta)/(4 pi m c^2))
 * int dn F(x) (I) and G(x) (Q, perpendicular to the projected field), and the
 * absorptivities from alpha = -(1/(8 pi m nu^2)) int P gamma^2 d/dgamma(dn/gamma^2)
 * (Rybicki and Lightman, synchrotron chapter), with x = nu/nu_crit,
 * nu_crit = 3/2 gamma^2 nu_c sin(theta), nu_c = e B/(2 pi m c), F(x) = x
 * int_x^inf K5/3, G(x) = x K2/3(x), in closed forms:
 *  - power law: the classical results for gmin^2 << X << gmax^2, X =
 *    nu/(nu_c sin theta) (the band that contains the paper's 230 GHz
 *    images), used at every X;
 *  - kappa: the exact low-frequency asymptotes (F and G at small x: the
 *    moments <gamma^-2/3> and <gamma^-5/3> of the distribution) and
 *    high-frequency asymptotes (the power-law tail gamma^(1-kappa) of the
 *    normalised distribution), joined as (low^-b + high^-b)^(-1/b) with b =
 *    3/7 for alpha_I and 1/2 for the others (chosen against the full
 *    integrals at kappa = 3.5..4, w = 1/2..1: within a factor 1.23 of them
 *    for the emissivities and 1.48 for the absorptivities over the
 *    transition, exact in both limits).
 * The circular and rotative terms (jV, aV, rQ, rV) of these populations are
 * taken as zero.  Physical values of the bridge: parity unpinned beyond the
 * stated accuracy. */

/* int_0^inf g(t) dt for a smooth g on (0, inf) by the trapezoid rule in
   v = ln t, the integrand g(t) t decaying exponentially in |v| at both ends */
static double kappa_dist_moment(double kappa, double w, double s)
{
    const double h = 0.005, kw = kappa * w;
    double sum = 0.0, v;
    for (v = -60.0; v <= 80.0; v += h) {
        double t = exp(v), gam = 1.0 + t;
        double f = gam * sqrt(t * (2.0 + t)) * pow(1.0 + t / kw, -kappa - 1.0) * pow(gam, s);
        sum += f * t;
    }
    return sum * h;
}

double or_kappa_integral(double kappa, double w, double s)
{
    return kappa_dist_moment(kappa, w, s);
}

void or_nonthermal_prepare(or_plasma *pl)
{
    double p = pl->pl_p, z;
    pl->pl_norm = (p - 1.0) / (pow(pl->pl_gmin, 1.0 - p) - pow(pl->pl_gmax, 1.0 - p));
    pl->kap_norm = pl->kap_m23 = pl->kap_m53 = 0.0;
    if (pl->kappa > 2.0 && pl->kappa_w > 0.0) {
        z = kappa_dist_moment(pl->kappa, pl->kappa_w, 0.0);
        pl->kap_norm = 1.0 / z;
        pl->kap_m23 = kappa_dist_moment(pl->kappa, pl->kappa_w, -2.0 / 3.0) / z;
        pl->kap_m53 = kappa_dist_moment(pl->kappa, pl->kappa_w, -5.0 / 3.0) / z;
    }
}

/* classical power-law coefficients in units of ne e^2 nu_c/c (j) and
   ne e^2/(nu m c) (alpha) for dn/dgamma = ne C gamma^-p at X = nu/(nu_c sin) */
static void powerlaw_reduced(double p, double C, double X, double sin_theta, double r[4])
{
    r[0] = pow(3.0, p / 2.0) * C * sin_theta / (2.0 * (p + 1.0))
         * tgamma((3.0 * p - 1.0) / 12.0) * tgamma((3.0 * p + 19.0) / 12.0) * pow(X, -(p - 1.0) / 2.0);
    r[1] = r[0] * (p + 1.0) / (p + 7.0 / 3.0);
    r[2] = pow(3.0, (p + 1.0) / 2.0) * C / 4.0
         * tgamma((3.0 * p + 2.0) / 12.0) * tgamma((3.0 * p + 22.0) / 12.0) * pow(X, -(p + 2.0) / 2.0);
    r[3] = r[2] * (p + 2.0) / (p + 10.0 / 3.0);
}

void or_nonthermal_coeffs(int kind, const or_plasma *pl, double ne, double B, double nu,
                          double cos_theta, int polarized, double out[8])
{
    double sin_theta, nuc, X, jn, an, r[4];
    int m;
    for (m = 0; m < 8; ++m) out[m] = 0.0;
    if (cos_theta > 1.0) cos_theta = 1.0;
    if (cos_theta < -1.0) cos_theta = -1.0;
    sin_theta = sqrt(1.0 - cos_theta * cos_theta);
    if (!(ne > 0.0) || !(B > 0.0) || !(sin_theta > 0.0)) return;
    nuc = Q_ELECTRON * B / (2.0 * M_PI * M_ELECTRON * C_LIGHT);
    X = nu / (nuc * sin_theta);
    jn = ne * Q_ELECTRON * Q_ELECTRON * nuc / C_LIGHT;
    an = ne * Q_ELECTRON * Q_ELECTRON / (nu * M_ELECTRON * C_LIGHT);
    if (kind == 1) {
        powerlaw_reduced(pl->pl_p, pl->pl_norm, X, sin_theta, r);
    } else {
        /* kappa: low-frequency asymptotes from F(x) ~ (4 pi/(sqrt3 Gamma(1/3))) (x/2)^1/3,
           G/F -> 1/2, and high-frequency ones from the tail ne A (kappa w)^(kappa+1) gamma^(1-kappa) */
        const double kap = pl->kappa, kw = kap * pl->kappa_w;
        const double g13 = tgamma(1.0 / 3.0);
        double lo[4], hi[4];
        lo[0] = 2.0 * M_PI / g13 * pow(X / 3.0, 1.0 / 3.0) * pl->kap_m23 * sin_theta;
        lo[1] = 0.5 * lo[0];
        lo[2] = 4.0 * M_PI / (3.0 * g13) / X * pow(X / 3.0, 1.0 / 3.0) * pl->kap_m53;
        lo[3] = 0.5 * lo[2];
        powerlaw_reduced(kap - 1.0, pl->kap_norm * pow(kw, kap + 1.0), X, sin_theta, hi);
        for (m = 0; m < 4; ++m) {
            const double b = m == 2 ? 3.0 / 7.0 : 0.5;   /* bridge exponents (alpha_I: 3/7) */
            r[m] = pow(pow(lo[m], -b) + pow(hi[m], -b), -1.0 / b);
        }
    }
    out[0] = jn * r[0];
    out[3] = an * r[2];
    if (!polarized) return;
    out[1] = jn * r[1];
    out[4] = an * r[3];
}

static double dot4(const double g[16], const double a[4], const double b[4])
{
    double s = 0.0;
    int i, j;
    for (i = 0; i < 4; ++i)
        for (j = 0; j < 4; ++j) s += g[4 * i + j] * a[i] * b[j];
    return s;
}

static void lower4(const double g[16], const double a[4], double al[4])
{
    int i, j;
    for (i = 0; i < 4; ++i) {
        al[i] = 0.0;
        for (j = 0; j < 4; ++j) al[i] += g[4 * i + j] * a[j];
    }
}

static int perm_sign(int a, int b, int c, int d)
{
    int p[4] = {a, b, c, d}, s = 1, i, j;
    for (i = 0; i < 4; ++i)
        for (j = i + 1; j < 4; ++j) {
            if (p[i] == p[j]) return 0;
            if (p[i] > p[j]) s = -s;
        }
    return s;
}

/* Orthonormal tetrad for observer u and photon momentum k (covariant), with
   e2 along vector w projected into the screen; e1 completes the right-handed
   screen basis.  e[4][4] contravariant. */
void or_tetrad(const double g[16], const double gi[16], const double u[4],
               const double kcov[4], const double w[4], double e[4][4])
{
    double ku[4], omega = 0.0, ul[4], e2l[4], e3l[4], t[4], nrm, we3, wu;
    const double zhat[4] = {0, 0, 0, 1}, xhat[4] = {0, 1, 0, 0};
    int al, be, ga, de, attempt;
    for (al = 0; al < 4; ++al) {
        ku[al] = 0.0;
        for (be = 0; be < 4; ++be) ku[al] += gi[4 * al + be] * kcov[be];
        omega -= kcov[al] * u[al];
    }
    for (al = 0; al < 4; ++al) {
        e[0][al] = u[al];
        e[3][al] = (ku[al] - omega * u[al]) / omega;
    }
    for (attempt = 0; attempt < 3; ++attempt) {
        const double *v = attempt == 0 ? w : (attempt == 1 ? zhat : xhat);
        double vn = sqrt(fabs(dot4(g, v, v)));
        wu = dot4(g, v, u);
        we3 = dot4(g, v, e[3]);
        for (al = 0; al < 4; ++al) t[al] = v[al] + wu * u[al] - we3 * e[3][al];
        nrm = sqrt(fabs(dot4(g, t, t)));
        if (vn > 0.0 && nrm > 1e-10 * vn) break;
    }
    for (al = 0; al < 4; ++al) e[2][al] = t[al] / nrm;
    lower4(g, u, ul);
    lower4(g, e[2], e2l);
    lower4(g, e[3], e3l);
    for (al = 0; al < 4; ++al) {
        double s = 0.0;
        for (be = 0; be < 4; ++be)
            for (ga = 0; ga < 4; ++ga)
                for (de = 0; de < 4; ++de) {
                    int sg = perm_sign(al, be, ga, de);
                    if (sg) s += sg * ul[be] * e2l[ga] * e3l[de];
                }
        e[1][al] = s;
    }
}

/* a quantity outside its cut limits (section 4.1, Data Cuts) */
static int cut_out(const or_plasma *pl, int k, double q)
{
    return q < pl->cut_lo[k] || q > pl->cut_hi[k];
}

void or_sample_point(const or_spacetime *st, const or_grid *gr, const or_plasma *pl,
                     const double y[8], double n_norm, double out[33])
{
    double g[16], gi[16], prim[8], u[4], ul[4], b[4], bl[4], ku[4];
    double q = 0.0, gam, alpha, beta[3], bt, b2, rho, p, sigma, binv, ne, tr, thetae;
    double Bg, omega, nu_fl, kb, cth, co[8], e[4][4];
    int i, j;
    memset(out, 0, 33 * sizeof(double));
    if (or_grid_sample(gr, pl->interp, y + 1, prim) < 0) return;
    rho = prim[0];
    p = prim[1];
    if (!(rho > 0.0)) return;
    if (pl->use_cuts) {
        double d = 0.0;
        if (cut_out(pl, OR_CUT_RHO, rho) || cut_out(pl, OR_CUT_P, p)) return;
        if (cut_out(pl, OR_CUT_R, or_ks_radius(st->a, y[1], y[2], y[3]))) return;
        for (i = 0; i < 3; ++i) d += (y[1 + i] - pl->plane_x0[i]) * pl->plane_n[i];
        if ((pl->plane > 0 && d < 0.0) || (pl->plane < 0 && d > 0.0)) return;
    }
    or_metric(st->a, st->flat, y, g, gi);
    /* fluid velocity from normal-frame components */
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) q += g[4 * (1 + i) + 1 + j] * prim[2 + i] * prim[2 + j];
    gam = sqrt(1.0 + q);
    alpha = 1.0 / sqrt(-gi[0]);
    for (i = 0; i < 3; ++i) beta[i] = -gi[1 + i] / gi[0];
    u[0] = gam / alpha;
    for (i = 0; i < 3; ++i) u[1 + i] = prim[2 + i] - gam * beta[i] / alpha;
    lower4(g, u, ul);
    /* magnetic 4-vector */
    bt = prim[5] * ul[1] + prim[6] * ul[2] + prim[7] * ul[3];
    b[0] = bt;
    for (i = 0; i < 3; ++i) b[1 + i] = (prim[5 + i] + bt * u[1 + i]) / u[0];
    b2 = dot4(g, b, b);
    sigma = b2 / rho;
    out[29] = sigma;
    if (sigma > pl->sigma_max) return;
    binv = b2 / (2.0 * p);
    ne = rho * gr->rho_unit / (pl->mu * M_PROTON) / (1.0 + 1.0 / pl->ne_ni);
    tr = (pl->r_high + binv * binv * pl->r_low) / (1.0 + binv * binv);
    thetae = pl->mu * M_PROTON / M_ELECTRON * (p / rho) * (pl->ne_ni + 1.0) / (pl->ne_ni + tr);
    Bg = sqrt(b2) * C_LIGHT * sqrt(4.0 * M_PI * gr->rho_unit);
    if (pl->use_cuts && (cut_out(pl, OR_CUT_NE, ne) || cut_out(pl, OR_CUT_THETAE, thetae) ||
                         cut_out(pl, OR_CUT_B, Bg) || cut_out(pl, OR_CUT_SIGMA, sigma) ||
                         cut_out(pl, OR_CUT_BETAINV, binv)))
        return;
    omega = 0.0;
    kb = 0.0;
    for (i = 0; i < 4; ++i) { omega -= y[4 + i] * u[i]; kb += y[4 + i] * b[i]; }
    nu_fl = n_norm * omega;
    cth = (b2 > 0.0) ? kb / (omega * sqrt(b2)) : 0.0;
    /* the populations' coefficients add (paper section 4.5: any admixture) */
    {
        double cn[8];
        int k;
        or_thermal_coeffs(pl->frac[0] * ne, thetae, Bg, nu_fl, cth, pl->polarized, co);
        for (k = 1; k <= 2; ++k) {
            if (!(pl->frac[k] > 0.0)) continue;
            or_nonthermal_coeffs(k, pl, pl->frac[k] * ne, Bg, nu_fl, cth, pl->polarized, cn);
            for (i = 0; i < 8; ++i) co[i] += cn[i];
        }
    }
    for (i = 0; i < 3; ++i) out[i] = co[i] / (nu_fl * nu_fl);
    for (i = 3; i < 8; ++i) out[i] = co[i] * nu_fl;
    out[8] = ne; out[9] = thetae; out[10] = Bg; out[11] = nu_fl;
    out[30] = rho; out[31] = p; out[32] = binv;
    for (i = 0; i < 4; ++i) {
        ku[i] = 0.0;
        for (j = 0; j < 4; ++j) ku[i] += gi[4 * i + j] * y[4 + j];
    }
    lower4(g, b, bl);
    or_tetrad(g, gi, u, y + 4, b, e);
    for (i = 0; i < 4; ++i)
        for (j = 0; j < 4; ++j) out[12 + 4 * i + j] = e[i][j];
    out[28] = 1.0;
}
