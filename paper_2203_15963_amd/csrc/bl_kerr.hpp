// bl_kerr.hpp -- Kerr geometry in Cartesian Kerr-Schild coordinates on the
// device: metric pieces, the Hamiltonian geodesic right-hand side, the
// connection contracted with the photon momentum, and the plane-parallel
// camera.
//
// Paper section 2, eq. (cks_aux): g = eta + f l l, g^-1 = eta - f l l with
// f = 2 r^3/(r^4 + a^2 z^2), l_mu = (1, (rx+ay)/(r^2+a^2), (ry-ax)/(r^2+a^2),
// z/r) and l^mu = (-1, l_x, l_y, l_z) (M = 1).  Because g differs from eta by
// a rank-one term, every contraction below is written with l.A products
// instead of 4x4 matrices.  The metric pieces are templates on the real type:
// the geodesic always runs in double, the transfer of the mixed-precision
// form evaluates its connection and frames in float.
#pragma once

#include "bl_common.hpp"

namespace bl {

// Kerr-Schild radius from eq. (cks_aux:r); the second branch is the same root
// written without cancellation when R^2 < a^2.
template <typename R>
__device__ __forceinline__ R ks_r(R a, R x, R y, R z) {
    R R2 = x * x + y * y + z * z;
    R d = R2 - a * a;
    R s = sqrt(d * d + R(4) * a * a * z * z);
    R r2 = (d >= R(0)) ? R(0.5) * (d + s) : ((s - d) > R(0) ? R(2) * a * a * z * z / (s - d) : R(0));
    return sqrt(r2);
}

// r with the reciprocals the metric functions need: 1/r, 1/(r^2 + a^2) and
// 1/s, s = sqrt((R^2 - a^2)^2 + 4 a^2 z^2).  From the quartic defining r,
// r^4 + a^2 z^2 = r^2 s, so f = 2 r^3/(r^4 + a^2 z^2) = 2 r/s and
// 1/(r^4 + a^2 z^2) = (1/r)^2 (1/s): one square root, one reciprocal square
// root and one reciprocal (in FP64 both from the hardware estimates refined
// by Newton steps).
template <typename R>
struct KSCore {
    R r, ir, ira, is;
};

template <typename R>
__device__ __forceinline__ KSCore<R> ks_core(R a, R x, R y, R z) {
    const R a2 = a * a;
    const R d = x * x + y * y + z * z - a2;
    const R s = sqrt(d * d + R(4) * a2 * z * z);
    // R^2 < a^2 (inside the ring's radius, never on a ray outside the
    // horizon): the same root without cancellation.  In FP64 that branch is
    // taken only when a lane of the wave needs it, so its division is not
    // evaluated speculatively; in FP32 the select is cheaper.
    R r2;
    if constexpr (sizeof(R) == 8) {
        r2 = R(0.5) * (d + s);
        if (__ballot(d < R(0)) != 0ull) {
            if (d < R(0)) r2 = (s - d) > R(0) ? R(2) * a2 * z * z / (s - d) : R(0);
        }
    } else {
        r2 = (d >= R(0)) ? R(0.5) * (d + s) : ((s - d) > R(0) ? R(2) * a2 * z * z / (s - d) : R(0));
    }
    const R q = r2 + a2;
    KSCore<R> c;
    if constexpr (sizeof(R) == 4) {
        c.ir = rsqrtf(r2);
        c.r = r2 > R(0) ? r2 * c.ir : R(0);
        const R inv = R(1) / (q * s);
        c.ira = s * inv;
        c.is = q * inv;
    } else {
        // 1/sqrt(r2): the hardware estimate and two Newton steps (about one
        // ulp), independent of the one reciprocal, so the two chains overlap
        double y = __builtin_amdgcn_rsq(r2);
#pragma unroll
        for (int it = 0; it < 2; ++it) y = y * (1.5 - (0.5 * r2) * (y * y));
        c.ir = y;
        c.r = r2 > R(0) ? r2 * y : R(0);
        const R inv = rcp_nr(q * s);
        c.ira = s * inv;
        c.is = q * inv;
    }
    return c;
}

// f and the spatial l (l_x, l_y, l_z); lower l_t = 1, upper l^t = -1.
template <typename R>
struct KS {
    R r, f, l[3];
};

template <typename R>
__device__ __forceinline__ KS<R> ks_point(R a, int flat, R x, R y, R z) {
    KS<R> k;
    const KSCore<R> c = ks_core(a, x, y, z);
    k.r = c.r;
    k.l[0] = (c.r * x + a * y) * c.ira;
    k.l[1] = (c.r * y - a * x) * c.ira;
    k.l[2] = z * c.ir;
    k.f = flat ? R(0) : R(2) * c.r * c.is;
    return k;
}

// l_mu A^mu for a contravariant A (l_t = +1)
template <typename R>
__device__ __forceinline__ R l_dot_up(const KS<R> &k, const R A[4]) {
    return A[0] + k.l[0] * A[1] + k.l[1] * A[2] + k.l[2] * A[3];
}
// l^mu A_mu for a covariant A (l^t = -1)
template <typename R>
__device__ __forceinline__ R l_dot_dn(const KS<R> &k, const R A[4]) {
    return -A[0] + k.l[0] * A[1] + k.l[1] * A[2] + k.l[2] * A[3];
}
// A_mu = g_mu nu A^nu
template <typename R>
__device__ __forceinline__ void lower(const KS<R> &k, const R A[4], R out[4]) {
    R la = k.f * l_dot_up(k, A);
    out[0] = -A[0] + la;
    out[1] = A[1] + la * k.l[0];
    out[2] = A[2] + la * k.l[1];
    out[3] = A[3] + la * k.l[2];
}
// A^mu = g^mu nu A_nu
template <typename R>
__device__ __forceinline__ void raise(const KS<R> &k, const R A[4], R out[4]) {
    R la = k.f * l_dot_dn(k, A);
    out[0] = -A[0] + la;
    out[1] = A[1] - la * k.l[0];
    out[2] = A[2] - la * k.l[1];
    out[3] = A[3] - la * k.l[2];
}
// g(A, B) for contravariant A, B
template <typename R>
__device__ __forceinline__ R gdot(const KS<R> &k, const R A[4], const R B[4]) {
    return -A[0] * B[0] + A[1] * B[1] + A[2] * B[2] + A[3] * B[3] + k.f * l_dot_up(k, A) * l_dot_up(k, B);
}

// Geodesic right-hand side, eq. (geodesic), for the seven evolving components
// y = (t, x, y, z, k_x, k_y, k_z) with the conserved k_t passed separately:
//   dx^mu/dl = eta^mu nu k_nu - f l^mu (l.k),
//   dk_c/dl = -1/2 d_c g^ab k_a k_b = 1/2 d_c f (l.k)^2 + f (l.k) (d_c l . k).
__device__ __forceinline__ void geo_rhs(double a, int flat, const double *y, double kt, double *dy) {
    // the metric functions and their derivatives from one reciprocal (ks_core)
    const double x = y[1], yy = y[2], z = y[3];
    const KSCore<double> kc = ks_core(a, x, yy, z);
    const double r = kc.r, r2 = r * r, a2 = a * a;
    const double ir = kc.ir, ira = kc.ira;
    const double iD = ir * ir * kc.is;   // 1/(r^4 + a^2 z^2)
    const double l[3] = {(r * x + a * yy) * ira, (r * yy - a * x) * ira, z * ir};
    const double f = flat ? 0.0 : 2.0 * r * kc.is;
    const double lk = -kt + l[0] * y[4] + l[1] * y[5] + l[2] * y[6];   // l^mu k_mu
    const double flk = f * lk;
    dy[0] = -kt + flk;
    dy[1] = y[4] - flk * l[0];
    dy[2] = y[5] - flk * l[1];
    dy[3] = y[6] - flk * l[2];
    // (no early return for the flat case: it keeps dy out of private memory)
    const double r3iD = r * kc.is;   // r^3 / (r^4 + a^2 z^2)
    const double dr[3] = {x * r3iD, yy * r3iD, z * (r2 + a2) * ir * kc.is};
    // d_c l_b = dr_c m_b + K_cb (differentiating the definition of l), so
    // (d_c l).k = dr_c (m.k) + (K k)_c
    const double m[3] = {(x - 2.0 * r * l[0]) * ira, (yy - 2.0 * r * l[1]) * ira, -l[2] * ir};
    const double mk = m[0] * y[4] + m[1] * y[5] + m[2] * y[6];
    const double Kk[3] = {ira * (r * y[4] - a * y[5]), ira * (a * y[4] + r * y[5]), ir * y[6]};
    // d_c f = f (3/r - 4 r^3/D) d_c r - [c = z] 2 f a^2 z / D, D = r^4 + a^2 z^2
    const double g1 = f * (3.0 * ir - 4.0 * r3iD);
    const double hl2 = 0.5 * lk * lk;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double df = g1 * dr[c] - (c == 2 ? 2.0 * f * a2 * z * iD : 0.0);
        const double dlk = dr[c] * mk + Kk[c];
        dy[4 + c] = flat ? 0.0 : df * hl2 + flk * dlk;
    }
}

// Proper-length rate of eq. (length): (g_pq k^p k^q)^1/2 with the normal-frame
// components k^p = k^a + beta^a k^t, beta^a = f l^a/(1+f), and g_pq = g_ab =
// delta_ab + f l_a l_b.  (Written out in full rather than as alpha k^t, which
// equals it only on the null cone: the integrated state drifts off the cone
// at the tolerance level.)
__device__ __forceinline__ double ds_dlambda(double a, int flat, const double *y, double kt) {
    KS<double> k = ks_point(a, flat, y[1], y[2], y[3]);
    double kc[4] = {kt, y[4], y[5], y[6]};
    double ku[4];
    raise(k, kc, ku);
    double sb = k.f / (1.0 + k.f) * ku[0];
    double p0 = ku[1] + sb * k.l[0], p1 = ku[2] + sb * k.l[1], p2 = ku[3] + sb * k.l[2];
    double lp = k.l[0] * p0 + k.l[1] * p1 + k.l[2] * p2;
    return sqrt(p0 * p0 + p1 * p1 + p2 * p2 + k.f * lp * lp);
}

// Connection contracted with the photon momentum, G^a_d = Gamma^a_{c d} k^c,
// in factored form.  With C_ed = Gamma_{e c d} k^c =
// 1/2 (k^c d_c g_ed + k^c d_d g_ec - k^c d_e g_dc), g = eta + f l l and
// d_t = 0, and with the spatial derivatives of l written as
// d_c l_b = dr_c m_b + K_cb (m and the constant-pattern K from differentiating
// the definition of l), the terms collect into
//   C_ed = l_e A_d + Y_e l_d + h Om_ed,   h = q f / 2,   Om_ed = d_d l_e - d_e l_d,
//   A = (Df l + f Dl + q df + f W) / 2,   Y = (f Dl - q df - f W) / 2,
// q = l_mu k^mu, Df = k^c d_c f, Dl_b = k^c d_c l_b, W_d = k^e d_d l_e
// (A_t = Df/2, Y_t = 0, Om spatial and antisymmetric).  Raising the first
// index with g^-1 = eta - f lu lu (lu = l^mu) gives
//   G^a_d = lu^a B_d + Yt^a l_d + h Om_ad,
//   B = (1 - f lu.l) A - h f (l.Om) = A - h f (l.Om),   Yt = Y - f (lu.Y) lu,
// since lu.l = |l|^2 - 1 vanishes for the Kerr-Schild l (its definition of r
// makes |l| = 1; in floating point lu.l is a rounding error, and dropping it
// changes B at that level).  G applied to a tensor then costs three row
// vectors and a 3x3 antisymmetric product instead of 16 entries of G.
template <typename R>
struct ConnF {
    R lu[4], l4[4], B[4], Yt[4];
    R oxy, oxz, oyz;   // h Om for the spatial pairs (x, y), (x, z), (y, z)
};

template <typename R>
__device__ __forceinline__ void conn_geom(R a, int flat, const R x[4], const R kc[4], ConnF<R> &c) {
    const R X = x[1], Yy = x[2], Z = x[3];
    const KSCore<R> kcr = ks_core(a, X, Yy, Z);
    const R r = kcr.r, r2 = r * r, a2 = a * a;
    const R ir = kcr.ir, ira = kcr.ira;
    const R iD = ir * ir * kcr.is;   // 1/(r^4 + a^2 z^2)
    const R l[3] = {(r * X + a * Yy) * ira, (r * Yy - a * X) * ira, Z * ir};
    const R r3iD = r * kcr.is;
    const R f = flat ? R(0) : R(2) * r3iD;
    // k^mu = g^mu nu k_nu
    // q = l_mu k^mu = (lu.k)(1 - f lu.l) = lu.k (lu.l = 0, as for B below)
    const R q = -kc[0] + l[0] * kc[1] + l[1] * kc[2] + l[2] * kc[3];
    const R flk = f * q;
    const R kv[3] = {kc[1] - flk * l[0], kc[2] - flk * l[1], kc[3] - flk * l[2]};
    // d_c r and m
    const R dr[3] = {X * r3iD, Yy * r3iD, Z * (r2 + a2) * ir * kcr.is};
    const R m[3] = {(X - R(2) * r * l[0]) * ira, (Yy - R(2) * r * l[1]) * ira, -l[2] * ir};
    const R mk = m[0] * kv[0] + m[1] * kv[1] + m[2] * kv[2];
    const R drk = dr[0] * kv[0] + dr[1] * kv[1] + dr[2] * kv[2];
    const R W[3] = {dr[0] * mk + ira * (r * kv[0] - a * kv[1]), dr[1] * mk + ira * (a * kv[0] + r * kv[1]),
                    dr[2] * mk + ir * kv[2]};
    const R Dl[3] = {m[0] * drk + ira * (r * kv[0] + a * kv[1]), m[1] * drk + ira * (r * kv[1] - a * kv[0]),
                     m[2] * drk + ir * kv[2]};
    // d_c f = f (3/r - 4 r^3/D) d_c r - [c = z] 2 f a^2 z / D
    const R g1 = f * (R(3) * ir - R(4) * r3iD);
    const R df[3] = {g1 * dr[0], g1 * dr[1], g1 * dr[2] - R(2) * f * a2 * Z * iD};
    const R Df = df[0] * kv[0] + df[1] * kv[1] + df[2] * kv[2];
    const R h = R(0.5) * q * f;
    const R oxy = dr[1] * m[0] - dr[0] * m[1] + R(2) * a * ira;
    const R oxz = dr[2] * m[0] - dr[0] * m[2];
    const R oyz = dr[2] * m[1] - dr[1] * m[2];
    // l.Om (spatial components)
    const R om[3] = {-l[1] * oxy - l[2] * oxz, l[0] * oxy - l[2] * oyz, l[0] * oxz + l[1] * oyz};
    const R hf = h * f;
    c.lu[0] = R(-1);
    c.l4[0] = R(1);
    c.B[0] = R(0.5) * Df;
    R lY = R(0), Yb[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R fD = f * Dl[b], qd = q * df[b], fW = f * W[b];
        Yb[b] = R(0.5) * (fD - qd - fW);
        lY += l[b] * Yb[b];
        c.lu[1 + b] = l[b];
        c.l4[1 + b] = l[b];
        c.B[1 + b] = R(0.5) * (Df * l[b] + fD + qd + fW) - hf * om[b];
    }
    c.Yt[0] = f * lY;
#pragma unroll
    for (int b = 0; b < 3; ++b) c.Yt[1 + b] = Yb[b] - f * lY * l[b];
    c.oxy = h * oxy;
    c.oxz = h * oxz;
    c.oyz = h * oyz;
}

// (h Om)_ad n^d for spatial a (1..3), n = (n1, n2, n3) the spatial part of a column
template <typename R>
__device__ __forceinline__ R conn_om(const ConnF<R> &c, int a, R n1, R n2, R n3) {
    return a == 1 ? c.oxy * n2 + c.oxz * n3 : (a == 2 ? c.oyz * n3 - c.oxy * n1 : -(c.oxz * n1 + c.oyz * n2));
}

// -G v for a contravariant v: the rate of change of a vector parallel
// transported along the ray, dv^a/dlambda = -G^a_d v^d.
template <typename R>
__device__ __forceinline__ void conn_vec(const ConnF<R> &c, const R v[4], R out[4]) {
    const R bv = c.B[0] * v[0] + c.B[1] * v[1] + c.B[2] * v[2] + c.B[3] * v[3];
    const R lv = c.l4[0] * v[0] + c.l4[1] * v[1] + c.l4[2] * v[2] + c.l4[3] * v[3];
    out[0] = -(c.lu[0] * bv + c.Yt[0] * lv);
#pragma unroll
    for (int a = 1; a < 4; ++a) out[a] = -(c.lu[a] * bv + c.Yt[a] * lv + conn_om(c, a, v[1], v[2], v[3]));
}

// The adjoint of conn_vec for a covariant x: out_d = -x_a G^a_d, so that
// x . conn_vec(v) = conn_covec(x) . v.  The spatial h Om is antisymmetric,
// so x_a (h Om)_ad = -((h Om) x)_d.
template <typename R>
__device__ __forceinline__ void conn_covec(const ConnF<R> &c, const R x[4], R out[4]) {
    const R xl = c.lu[0] * x[0] + c.lu[1] * x[1] + c.lu[2] * x[2] + c.lu[3] * x[3];
    const R xy = c.Yt[0] * x[0] + c.Yt[1] * x[1] + c.Yt[2] * x[2] + c.Yt[3] * x[3];
    out[0] = -(xl * c.B[0] + xy * c.l4[0]);
#pragma unroll
    for (int d = 1; d < 4; ++d) out[d] = conn_om(c, d, x[1], x[2], x[3]) - (xl * c.B[d] + xy * c.l4[d]);
}

// Full G (row-major a, d), FP64, for checking.
__device__ __forceinline__ void conn_k(double a, int flat, const double x[4], const double kc[4], double G[16]) {
    ConnF<double> c;
    conn_geom(a, flat, x, kc, c);
#pragma unroll
    for (int aa = 0; aa < 4; ++aa)
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            double v = c.lu[aa] * c.B[dd] + c.Yt[aa] * c.l4[dd];
            if (aa > 0 && dd > 0)
                v += conn_om(c, aa, dd == 1 ? 1.0 : 0.0, dd == 2 ? 1.0 : 0.0, dd == 3 ? 1.0 : 0.0);
            G[4 * aa + dd] = flat ? 0.0 : v;
        }
}

// 4-velocity from CKS normal-frame components ut at point k:
// gamma = (1 + g_ab ut^a ut^b)^1/2, u^t = gamma/alpha, u^a = ut^a - gamma beta^a/alpha,
// alpha = (1+f)^-1/2, beta^a = f l^a/(1+f).
template <typename R>
__device__ __forceinline__ void velocity_from_normal(const KS<R> &k, const R ut[3], R u[4]) {
    R lu = k.l[0] * ut[0] + k.l[1] * ut[1] + k.l[2] * ut[2];
    R q = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2] + k.f * lu * lu;
    R gam = sqrt(R(1) + q);
    R alpha = rsqrt_r(R(1) + k.f);
    u[0] = gam * (R(1) + k.f) * alpha;   // gamma / alpha
    R sb = gam * k.f * alpha;            // gamma beta^a / alpha = sb l^a
    u[1] = ut[0] - sb * k.l[0];
    u[2] = ut[1] - sb * k.l[1];
    u[3] = ut[2] - sb * k.l[2];
}

// Initial state of pixel (i, j) of the plane-parallel camera (paper section
// 2.1): x_pix = x_c + a H + b V, k^a = K^a, k^t the root of the null
// condition g k k = 0 that is positive (the lesser positive one inside the
// ergosphere); then k_mu = g_mu nu k^nu.  The frequency normalisation is
// n = nu / den with den = -k_t (frequency at infinity) or -k.u (at the
// camera); den does not depend on nu, so one traced ray serves every
// frequency.
__device__ __forceinline__ void camera_pixel(const Frame &fr, const CamParams &cp, double a, int flat, int i, int j,
                                             double y[8], double &den) {
    double N = (double)cp.nf;
    double ap = ((double)(i + cp.i0) - 0.5 * N + 0.5) * cp.width / N;
    double bp = ((double)(j + cp.j0) - 0.5 * N + 0.5) * cp.width / N;
#pragma unroll
    for (int m = 0; m < 4; ++m) y[m] = fr.xc[m] + (ap * fr.H[m] + bp * fr.V[m]);
    KS<double> k = ks_point(a, flat, y[1], y[2], y[3]);
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
        den = -y[4];
    } else {
        double u[4];
        velocity_from_normal(k, fr.ut, u);
        den = -(y[4] * u[0] + y[5] * u[1] + y[6] * u[2] + y[7] * u[3]);
    }
}

}  // namespace bl
