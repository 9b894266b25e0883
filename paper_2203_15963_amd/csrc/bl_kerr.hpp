// bl_kerr.hpp -- Kerr geometry in Cartesian Kerr-Schild coordinates on the
// device: metric pieces, the Hamiltonian geodesic right-hand side, the
// connection contracted with the photon momentum, and the plane-parallel
// camera.
//
// Paper section 2, eq. (cks_aux): g = eta + f l l, g^-1 = eta - f l l with
// f = 2 r^3/(r^4 + a^2 z^2), l_mu = (1, (rx+ay)/(r^2+a^2), (ry-ax)/(r^2+a^2),
// z/r) and l^mu = (-1, l_x, l_y, l_z) (M = 1).  Because g differs from eta by
// a rank-one term, every contraction below is written with l.A products
// instead of 4x4 matrices.
#pragma once

#include "bl_common.hpp"

namespace bl {

// Kerr-Schild radius from eq. (cks_aux:r); the second branch is the same root
// written without cancellation when R^2 < a^2.
__device__ __forceinline__ double ks_r(double a, double x, double y, double z) {
    double R2 = x * x + y * y + z * z;
    double d = R2 - a * a;
    double s = sqrt(d * d + 4.0 * a * a * z * z);
    double r2 = (d >= 0.0) ? 0.5 * (d + s) : ((s - d) > 0.0 ? 2.0 * a * a * z * z / (s - d) : 0.0);
    return sqrt(r2);
}

// f and the spatial l (l_x, l_y, l_z); lower l_t = 1, upper l^t = -1.
struct KS {
    double r, f, l[3];
};

__device__ __forceinline__ KS ks_point(double a, int flat, double x, double y, double z) {
    KS k;
    double r = ks_r(a, x, y, z);
    double r2 = r * r;
    double ira = 1.0 / (r2 + a * a);
    k.r = r;
    k.l[0] = (r * x + a * y) * ira;
    k.l[1] = (r * y - a * x) * ira;
    k.l[2] = z / r;
    k.f = flat ? 0.0 : 2.0 * r2 * r / (r2 * r2 + a * a * z * z);
    return k;
}

// l_mu A^mu for a contravariant A (l_t = +1)
__device__ __forceinline__ double l_dot_up(const KS &k, const double A[4]) {
    return A[0] + k.l[0] * A[1] + k.l[1] * A[2] + k.l[2] * A[3];
}
// l^mu A_mu for a covariant A (l^t = -1)
__device__ __forceinline__ double l_dot_dn(const KS &k, const double A[4]) {
    return -A[0] + k.l[0] * A[1] + k.l[1] * A[2] + k.l[2] * A[3];
}
// A_mu = g_mu nu A^nu
__device__ __forceinline__ void lower(const KS &k, const double A[4], double out[4]) {
    double la = k.f * l_dot_up(k, A);
    out[0] = -A[0] + la;
    out[1] = A[1] + la * k.l[0];
    out[2] = A[2] + la * k.l[1];
    out[3] = A[3] + la * k.l[2];
}
// A^mu = g^mu nu A_nu
__device__ __forceinline__ void raise(const KS &k, const double A[4], double out[4]) {
    double la = k.f * l_dot_dn(k, A);
    out[0] = -A[0] + la;
    out[1] = A[1] - la * k.l[0];
    out[2] = A[2] - la * k.l[1];
    out[3] = A[3] - la * k.l[2];
}
// g(A, B) for contravariant A, B
__device__ __forceinline__ double gdot(const KS &k, const double A[4], const double B[4]) {
    return -A[0] * B[0] + A[1] * B[1] + A[2] * B[2] + A[3] * B[3] + k.f * l_dot_up(k, A) * l_dot_up(k, B);
}

// Spatial derivatives of r, f and l at (x, y, z): dr[c], df[c], dl[c][b]
// (c = derivative direction, b = component x, y, z).  From
// r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0 and the definitions of f and l.
struct KSDeriv {
    double dr[3], df[3], dl[3][3];
};

__device__ __forceinline__ void ks_deriv(double a, int flat, double x, double y, double z, const KS &k,
                                         KSDeriv &d) {
    double r = k.r, r2 = r * r;
    double D = r2 * r2 + a * a * z * z;
    double iD = 1.0 / D;
    double ira = 1.0 / (r2 + a * a);
    double ir = 1.0 / r;
    d.dr[0] = x * r2 * r * iD;
    d.dr[1] = y * r2 * r * iD;
    d.dr[2] = z * r * (r2 + a * a) * iD;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double dD = 4.0 * r2 * r * d.dr[c] + (c == 2 ? 2.0 * a * a * z : 0.0);
        d.df[c] = flat ? 0.0 : k.f * (3.0 * d.dr[c] * ir - dD * iD);
        d.dl[c][0] = (d.dr[c] * x + (c == 0 ? r : 0.0) + (c == 1 ? a : 0.0) - 2.0 * r * k.l[0] * d.dr[c]) * ira;
        d.dl[c][1] = (d.dr[c] * y + (c == 1 ? r : 0.0) - (c == 0 ? a : 0.0) - 2.0 * r * k.l[1] * d.dr[c]) * ira;
        d.dl[c][2] = ((c == 2 ? 1.0 : 0.0) - k.l[2] * d.dr[c]) * ir;
    }
}

// Geodesic right-hand side, eq. (geodesic), for the seven evolving components
// y = (t, x, y, z, k_x, k_y, k_z) with the conserved k_t passed separately:
//   dx^mu/dl = eta^mu nu k_nu - f l^mu (l.k),
//   dk_c/dl = -1/2 d_c g^ab k_a k_b = 1/2 d_c f (l.k)^2 + f (l.k) (d_c l . k).
__device__ __forceinline__ void geo_rhs(double a, int flat, const double *y, double kt, double *dy) {
    KS k = ks_point(a, flat, y[1], y[2], y[3]);
    double kc[4] = {kt, y[4], y[5], y[6]};
    double lk = l_dot_dn(k, kc);
    double flk = k.f * lk;
    dy[0] = -kt + flk;
    dy[1] = y[4] - flk * k.l[0];
    dy[2] = y[5] - flk * k.l[1];
    dy[3] = y[6] - flk * k.l[2];
    // (no early return for the flat case: it keeps dy out of private memory)
    KSDeriv d;
    ks_deriv(a, flat, y[1], y[2], y[3], k, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double dlk = d.dl[c][0] * y[4] + d.dl[c][1] * y[5] + d.dl[c][2] * y[6];
        dy[4 + c] = flat ? 0.0 : 0.5 * d.df[c] * lk * lk + flk * dlk;
    }
}

// Proper-length rate of eq. (length): (g_pq k^p k^q)^1/2 with the normal-frame
// components k^p = k^a + beta^a k^t, beta^a = f l^a/(1+f), and g_pq = g_ab =
// delta_ab + f l_a l_b.  (Written out in full rather than as alpha k^t, which
// equals it only on the null cone: the integrated state drifts off the cone
// at the tolerance level.)
__device__ __forceinline__ double ds_dlambda(double a, int flat, const double *y, double kt) {
    KS k = ks_point(a, flat, y[1], y[2], y[3]);
    double kc[4] = {kt, y[4], y[5], y[6]};
    double ku[4];
    raise(k, kc, ku);
    double sb = k.f / (1.0 + k.f) * ku[0];
    double p0 = ku[1] + sb * k.l[0], p1 = ku[2] + sb * k.l[1], p2 = ku[3] + sb * k.l[2];
    double lp = k.l[0] * p0 + k.l[1] * p1 + k.l[2] * p2;
    return sqrt(p0 * p0 + p1 * p1 + p2 * p2 + k.f * lp * lp);
}

// G^a_d = Gamma^a_{c d} k^c at state (x, k_mu), G[a][d] row-major.
// With C_ed = Gamma_{e c d} k^c = 1/2 (T1_ed + T2_ed - T2_de),
//   T1_ed = k^c d_c g_ed = (k.df) l_e l_d + f ((k.dl_e) l_d + l_e (k.dl_d)),
//   T2_ed = d_d g_ec k^c = q (d_d f l_e + f d_d l_e) + f l_e (d_d l . k),
// q = l_mu k^mu, d_t = 0, and G^a_d = g^{a e} C_ed.
__device__ __forceinline__ void conn_k(double a, int flat, const double x[4], const double kc[4],
                                       double G[16]) {
    if (flat) {
#pragma unroll
        for (int m = 0; m < 16; ++m) G[m] = 0.0;
        return;
    }
    KS k = ks_point(a, flat, x[1], x[2], x[3]);
    KSDeriv d;
    ks_deriv(a, flat, x[1], x[2], x[3], k, d);
    double ku[4];
    raise(k, kc, ku);
    double q = l_dot_up(k, ku);
    double l4[4] = {1.0, k.l[0], k.l[1], k.l[2]};
    double Df = d.df[0] * ku[1] + d.df[1] * ku[2] + d.df[2] * ku[3];
    double Dl[4] = {0.0, 0.0, 0.0, 0.0};
    double W[4] = {0.0, 0.0, 0.0, 0.0};
    double df4[4] = {0.0, d.df[0], d.df[1], d.df[2]};
#pragma unroll
    for (int b = 0; b < 3; ++b) Dl[1 + b] = d.dl[0][b] * ku[1] + d.dl[1][b] * ku[2] + d.dl[2][b] * ku[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) W[1 + c] = d.dl[c][0] * ku[1] + d.dl[c][1] * ku[2] + d.dl[c][2] * ku[3];
    // T2[e][d]
    double T2[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        T2[e][0] = 0.0;
#pragma unroll
        for (int dd = 1; dd < 4; ++dd) {
            double dle = (e == 0) ? 0.0 : d.dl[dd - 1][e - 1];
            T2[e][dd] = q * (df4[dd] * l4[e] + k.f * dle) + k.f * l4[e] * W[dd];
        }
    }
    double C[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            double T1 = Df * l4[e] * l4[dd] + k.f * (Dl[e] * l4[dd] + l4[e] * Dl[dd]);
            C[e][dd] = 0.5 * (T1 + T2[e][dd] - T2[dd][e]);
        }
    // raise the first index: G^a_d = eta^{ae} C_ed - f l^a (l^e C_ed)
    double lu[4] = {-1.0, k.l[0], k.l[1], k.l[2]};
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        double lc = lu[0] * C[0][dd] + lu[1] * C[1][dd] + lu[2] * C[2][dd] + lu[3] * C[3][dd];
        G[0 * 4 + dd] = -C[0][dd] - k.f * lu[0] * lc;
        G[1 * 4 + dd] = C[1][dd] - k.f * lu[1] * lc;
        G[2 * 4 + dd] = C[2][dd] - k.f * lu[2] * lc;
        G[3 * 4 + dd] = C[3][dd] - k.f * lu[3] * lc;
    }
}

// The same connection, one column d of G at a time, from scalars prepared
// once per point (keeps the 4x4 temporaries of conn_k out of the registers
// when G is applied immediately).
struct ConnGeom {
    double f, q, Df;
    double l4[4], lu[4], Dl[4], W[4], df4[4];
    double dl[3][3];
};

__device__ __forceinline__ void conn_geom(double a, int flat, const double x[4], const double kc[4], ConnGeom &c) {
    KS k = ks_point(a, flat, x[1], x[2], x[3]);
    KSDeriv d;
    ks_deriv(a, flat, x[1], x[2], x[3], k, d);
    double ku[4];
    raise(k, kc, ku);
    c.f = k.f;
    c.q = l_dot_up(k, ku);
    c.l4[0] = 1.0;
    c.lu[0] = -1.0;
    c.Dl[0] = 0.0;
    c.W[0] = 0.0;
    c.df4[0] = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        c.l4[1 + b] = k.l[b];
        c.lu[1 + b] = k.l[b];
        c.df4[1 + b] = d.df[b];
        c.Dl[1 + b] = d.dl[0][b] * ku[1] + d.dl[1][b] * ku[2] + d.dl[2][b] * ku[3];
        c.W[1 + b] = d.dl[b][0] * ku[1] + d.dl[b][1] * ku[2] + d.dl[b][2] * ku[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) c.dl[b][e] = d.dl[b][e];
    }
    c.Df = d.df[0] * ku[1] + d.df[1] * ku[2] + d.df[2] * ku[3];
}

// column dd of G^a_d (see conn_k)
__device__ __forceinline__ void conn_col(const ConnGeom &c, int dd, double Gc[4]) {
    double C[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double T1 = c.Df * c.l4[e] * c.l4[dd] + c.f * (c.Dl[e] * c.l4[dd] + c.l4[e] * c.Dl[dd]);
        double T2ed = (dd == 0) ? 0.0
                                : c.q * (c.df4[dd] * c.l4[e] + c.f * (e == 0 ? 0.0 : c.dl[dd - 1][e - 1])) +
                                      c.f * c.l4[e] * c.W[dd];
        double T2de = (e == 0) ? 0.0
                               : c.q * (c.df4[e] * c.l4[dd] + c.f * (dd == 0 ? 0.0 : c.dl[e - 1][dd - 1])) +
                                     c.f * c.l4[dd] * c.W[e];
        C[e] = 0.5 * (T1 + T2ed - T2de);
    }
    double lc = c.lu[0] * C[0] + c.lu[1] * C[1] + c.lu[2] * C[2] + c.lu[3] * C[3];
    Gc[0] = -C[0] - c.f * c.lu[0] * lc;
    Gc[1] = C[1] - c.f * c.lu[1] * lc;
    Gc[2] = C[2] - c.f * c.lu[2] * lc;
    Gc[3] = C[3] - c.f * c.lu[3] * lc;
}

// 4-velocity from CKS normal-frame components ut at point k:
// gamma = (1 + g_ab ut^a ut^b)^1/2, u^t = gamma/alpha, u^a = ut^a - gamma beta^a/alpha,
// alpha = (1+f)^-1/2, beta^a = f l^a/(1+f).
__device__ __forceinline__ void velocity_from_normal(const KS &k, const double ut[3], double u[4]) {
    double lu = k.l[0] * ut[0] + k.l[1] * ut[1] + k.l[2] * ut[2];
    double q = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2] + k.f * lu * lu;
    double gam = sqrt(1.0 + q);
    double ialpha = sqrt(1.0 + k.f);
    u[0] = gam * ialpha;
    double sb = gam * ialpha * k.f / (1.0 + k.f);
    u[1] = ut[0] - sb * k.l[0];
    u[2] = ut[1] - sb * k.l[1];
    u[3] = ut[2] - sb * k.l[2];
}

// Initial state of pixel (i, j) of the plane-parallel camera (paper section
// 2.1): x_pix = x_c + a H + b V, k^a = K^a, k^t the root of the null
// condition g k k = 0 that is positive (the lesser positive one inside the
// ergosphere); then k_mu = g_mu nu k^nu and the normalisation n.
__device__ __forceinline__ void camera_pixel(const Frame &fr, const CamParams &cp, double a, int flat,
                                             int i, int j, double y[8], double &n_norm) {
    double N = (double)cp.n;
    double ap = ((double)i - 0.5 * N + 0.5) * cp.width / N;
    double bp = ((double)j - 0.5 * N + 0.5) * cp.width / N;
#pragma unroll
    for (int m = 0; m < 4; ++m) y[m] = fr.xc[m] + (ap * fr.H[m] + bp * fr.V[m]);
    KS k = ks_point(a, flat, y[1], y[2], y[3]);
    double K3[3] = {fr.K[1], fr.K[2], fr.K[3]};
    double lK = k.l[0] * K3[0] + k.l[1] * K3[1] + k.l[2] * K3[2];
    double A = -1.0 + k.f;                       // g_tt
    double B = k.f * lK;                         // g_ta k^a
    double C = K3[0] * K3[0] + K3[1] * K3[1] + K3[2] * K3[2] + k.f * lK * lK;
    double ku[4];
    ku[0] = (-B - sqrt(B * B - A * C)) / A;
    ku[1] = K3[0];
    ku[2] = K3[1];
    ku[3] = K3[2];
    lower(k, ku, y + 4);
    if (cp.freq_mode == 0) {
        n_norm = cp.nu / (-y[4]);
    } else {
        double u[4];
        velocity_from_normal(k, fr.ut, u);
        n_norm = cp.nu / (-(y[4] * u[0] + y[5] * u[1] + y[6] * u[2] + y[7] * u[3]));
    }
}

}  // namespace bl
