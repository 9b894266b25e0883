/*
 * kerr.c -- Kerr metric in Cartesian Kerr-Schild coordinates (oracle).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper section 2, eq. (cks_aux): g = eta + f l l, g^-1 = eta - f l l with
 * f = 2 M r^3 / (r^4 + a^2 z^2), l_alpha = (1, (rx+ay)/(r^2+a^2),
 * (ry-ax)/(r^2+a^2), z/r), l^alpha = (-1, same spatial), and r from R, z.
 * M = 1.  Derivatives are the chain rule applied to these definitions.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

static const double ETA[16] = {-1,0,0,0, 0,1,0,0, 0,0,1,0, 0,0,0,1};

/* eq. (cks_aux:r): 2 r^2 = R^2 - a^2 + sqrt((R^2-a^2)^2 + 4 a^2 z^2).
   When R^2 < a^2 the same root is written in the cancellation-free form
   r^2 = 2 a^2 z^2 / (sqrt(...) - (R^2 - a^2)). */
double or_ks_radius(double a, double x, double y, double z)
{
    double R2 = x * x + y * y + z * z;
    double d = R2 - a * a;
    double s = sqrt(d * d + 4.0 * a * a * z * z);
    double r2;
    if (d >= 0.0)
        r2 = 0.5 * (d + s);
    else
        r2 = (s - d) > 0.0 ? 2.0 * a * a * z * z / (s - d) : 0.0;
    return sqrt(r2);
}

/* f, l_alpha (lower) and their spatial derivatives d_c f, d_c l_alpha. */
static void ks_parts(double a, int flat, const double x[4], double *f, double l[4],
                     double df[3], double dl[3][4])
{
    double X = x[1], Y = x[2], Z = x[3];
    double r = or_ks_radius(a, X, Y, Z);
    double r2 = r * r, s = r2 + a * a;
    double D = r2 * r2 + a * a * Z * Z;
    double dr[3];
    int c;
    l[0] = 1.0;
    l[1] = (r * X + a * Y) / s;
    l[2] = (r * Y - a * X) / s;
    l[3] = Z / r;
    /* from r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0 */
    dr[0] = X * r2 * r / D;
    dr[1] = Y * r2 * r / D;
    dr[2] = Z * r * s / D;
    for (c = 0; c < 3; ++c) {
        double dD = 4.0 * r2 * r * dr[c] + (c == 2 ? 2.0 * a * a * Z : 0.0);
        double dxc_x = (c == 0), dxc_y = (c == 1), dxc_z = (c == 2);
        df[c] = 2.0 * (3.0 * r2 * dr[c] * D - r2 * r * dD) / (D * D);
        dl[c][0] = 0.0;
        dl[c][1] = ((dr[c] * X + r * dxc_x + a * dxc_y) * s - (r * X + a * Y) * 2.0 * r * dr[c]) / (s * s);
        dl[c][2] = ((dr[c] * Y + r * dxc_y - a * dxc_x) * s - (r * Y - a * X) * 2.0 * r * dr[c]) / (s * s);
        dl[c][3] = (r * dxc_z - Z * dr[c]) / r2;
    }
    *f = 2.0 * r2 * r / D;
    if (flat) {
        *f = 0.0;
        for (c = 0; c < 3; ++c) df[c] = 0.0;
    }
}

void or_metric(double a, int flat, const double x[4], double g[16], double gi[16])
{
    double f, l[4], df[3], dl[3][4], lu[4];
    int al, be;
    ks_parts(a, flat, x, &f, l, df, dl);
    lu[0] = -l[0]; lu[1] = l[1]; lu[2] = l[2]; lu[3] = l[3];
    for (al = 0; al < 4; ++al)
        for (be = 0; be < 4; ++be) {
            g[4 * al + be] = ETA[4 * al + be] + f * l[al] * l[be];
            gi[4 * al + be] = ETA[4 * al + be] - f * lu[al] * lu[be];
        }
}

/* dg[c][alpha][beta] = d_c g_{alpha beta}, dgi[c][alpha][beta] = d_c g^{alpha beta}
   for spatial c = x, y, z (index 0..2). */
void or_metric_deriv(double a, int flat, const double x[4], double dg[48], double dgi[48])
{
    double f, l[4], df[3], dl[3][4], lu[4], dlu[4];
    int c, al, be;
    ks_parts(a, flat, x, &f, l, df, dl);
    lu[0] = -l[0]; lu[1] = l[1]; lu[2] = l[2]; lu[3] = l[3];
    for (c = 0; c < 3; ++c) {
        dlu[0] = 0.0; dlu[1] = dl[c][1]; dlu[2] = dl[c][2]; dlu[3] = dl[c][3];
        for (al = 0; al < 4; ++al)
            for (be = 0; be < 4; ++be) {
                double ff = flat ? 0.0 : f;
                dg[16 * c + 4 * al + be] = df[c] * l[al] * l[be]
                                         + ff * (dl[c][al] * l[be] + l[al] * dl[c][be]);
                dgi[16 * c + 4 * al + be] = -(df[c] * lu[al] * lu[be]
                                         + ff * (dlu[al] * lu[be] + lu[al] * dlu[be]));
            }
    }
}

/* Gamma^alpha_{beta gamma} = 1/2 g^{alpha delta} (d_beta g_{delta gamma}
   + d_gamma g_{delta beta} - d_delta g_{beta gamma}); d_t = 0 (stationary).
   Stored gam[16 alpha + 4 beta + gamma]. */
void or_christoffel(double a, int flat, const double x[4], double gam[64])
{
    double g[16], gi[16], dg[48], dgi[48];
    double d[4][16]; /* d[mu][alpha beta] = d_mu g_{alpha beta} */
    int al, be, ga, de;
    or_metric(a, flat, x, g, gi);
    or_metric_deriv(a, flat, x, dg, dgi);
    memset(d[0], 0, sizeof(d[0]));
    for (al = 0; al < 3; ++al) memcpy(d[al + 1], dg + 16 * al, sizeof(d[0]));
    for (al = 0; al < 4; ++al)
        for (be = 0; be < 4; ++be)
            for (ga = 0; ga < 4; ++ga) {
                double sum = 0.0;
                for (de = 0; de < 4; ++de)
                    sum += gi[4 * al + de] * (d[be][4 * de + ga] + d[ga][4 * de + be]
                                              - d[de][4 * be + ga]);
                gam[16 * al + 4 * be + ga] = 0.5 * sum;
            }
}

/* eq. (geodesic): dx^alpha/dlambda = g^{alpha beta} k_beta, dk_t/dlambda = 0,
   dk_a/dlambda = -1/2 d_a g^{alpha beta} k_alpha k_beta.
   y = (t, x, y, z, k_t, k_x, k_y, k_z). */
void or_geodesic_rhs(double a, int flat, const double y[8], double dy[8])
{
    double g[16], gi[16], dg[48], dgi[48];
    const double *k = y + 4;
    int al, be, c;
    or_metric(a, flat, y, g, gi);
    or_metric_deriv(a, flat, y, dg, dgi);
    for (al = 0; al < 4; ++al) {
        double s = 0.0;
        for (be = 0; be < 4; ++be) s += gi[4 * al + be] * k[be];
        dy[al] = s;
    }
    dy[4] = 0.0;
    for (c = 0; c < 3; ++c) {
        double s = 0.0;
        for (al = 0; al < 4; ++al)
            for (be = 0; be < 4; ++be) s += dgi[16 * c + 4 * al + be] * k[al] * k[be];
        dy[5 + c] = -0.5 * s;
    }
}
