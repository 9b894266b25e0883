/*
 * camera.c -- plane-parallel camera (oracle).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper section 2.1 ("Camera Definition"): camera frame based on CKS with
 * basis e_t' = u, e_a' = d_a - (u_a/u_t) d_t and metric g_a'b', g^a'b';
 * line of sight K, vertical v from U = z (y on the polar axis) by
 * Gram-Schmidt, horizontal h = D^-1/2 [abc] v_b' K_c', rotation by psi;
 * pixel offsets (a,b) = ((i,j) - N/2 + 1/2) w/N; plane-parallel pixels
 * x_pix = x + a H + b V, k_pix^a = K^a, k_pix^t from the null condition
 * (the lesser positive root inside the ergosphere); normalisation n from
 * -n k_t = nu (at infinity) or -n k.u = nu (at the camera).
 *
 * Readings:
 *  - the user's k_i are spherical-KS covariant spatial components; k_t is
 *    fixed by the null condition with k^t > 0 (future directed);
 *  - u^p are spherical-KS normal-frame components; they map to CKS
 *    normal-frame components with the spatial Jacobian (the normal observer
 *    is the same in both charts);
 *  - for frequency at the camera, the pixel observer has the camera's CKS
 *    normal-frame velocity components, evaluated with the metric at x_pix.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

/* spatial Jacobian J[a][i] = d x^a / d x^i, i = (r, theta, phi) */
static void sph_jacobian(double a, double r, double th, double ph, double J[3][3])
{
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    J[0][0] = st * cp; J[0][1] = ct * (r * cp - a * sp); J[0][2] = st * (-r * sp - a * cp);
    J[1][0] = st * sp; J[1][1] = ct * (r * sp + a * cp); J[1][2] = st * (r * cp - a * sp);
    J[2][0] = ct;      J[2][1] = -r * st;                J[2][2] = 0.0;
}

/* solve the 3x3 system M x = b by Cramer's rule */
static void solve3(const double M[3][3], const double b[3], double x[3])
{
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
               - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
               + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    int c, r, q;
    for (c = 0; c < 3; ++c) {
        double T[3][3];
        for (r = 0; r < 3; ++r)
            for (q = 0; q < 3; ++q) T[r][q] = (q == c) ? b[r] : M[r][q];
        x[c] = (T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1])
              - T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0])
              + T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0])) / det;
    }
}

/* contravariant 4-velocity from CKS normal-frame components ut[3] at x */
static void velocity_from_normal(double a, int flat, const double x[4], const double ut[3],
                                 double u[4])
{
    double g[16], gi[16], q = 0.0, alpha, beta[3], gam;
    int i, j;
    or_metric(a, flat, x, g, gi);
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) q += g[4 * (1 + i) + 1 + j] * ut[i] * ut[j];
    gam = sqrt(1.0 + q);
    alpha = 1.0 / sqrt(-gi[0]);
    for (i = 0; i < 3; ++i) beta[i] = -gi[1 + i] / gi[0];
    u[0] = gam / alpha;
    for (i = 0; i < 3; ++i) u[1 + i] = ut[i] - gam * beta[i] / alpha;
}

typedef struct {
    double xc[4], u[4], K[4], H[4], V[4];
    double ut_cks[3];
} cam_frame;

static void camera_frame(const or_camera *cam, const or_spacetime *st, cam_frame *fr)
{
    const double a = st->a;
    const int flat = st->flat;
    double J[3][3], JT[3][3], g[16], gi[16], ul[4], kl[4];
    double gp[3][3], gpi[3][3], Kl[3], Ku[3], Kt, U[3], vu[3], vl[3], hu[3];
    double A, B, C, nrm, UK, D;
    int i, j, b;

    fr->xc[0] = 0.0;
    fr->xc[1] = sin(cam->theta) * (cam->r * cos(cam->phi) - a * sin(cam->phi));
    fr->xc[2] = sin(cam->theta) * (cam->r * sin(cam->phi) + a * cos(cam->phi));
    fr->xc[3] = cam->r * cos(cam->theta);
    sph_jacobian(a, cam->r, cam->theta, cam->phi, J);
    for (i = 0; i < 3; ++i) {
        fr->ut_cks[i] = 0.0;
        for (j = 0; j < 3; ++j) fr->ut_cks[i] += J[i][j] * cam->u_normal[j];
    }
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) JT[i][j] = J[j][i];
    if (sin(cam->theta) != 0.0) {
        solve3(JT, cam->k_cov, kl + 1);   /* k_i = J^a_i k_a */
    } else {
        /* on the polar axis d/dphi vanishes: take the minimum-norm solution
           of k_r = J^a_r k_a, k_theta = J^a_theta k_a */
        double w0 = J[0][1], w1 = J[1][1], ww = w0 * w0 + w1 * w1;
        kl[3] = cam->k_cov[0] / J[2][0];
        kl[1] = ww > 0.0 ? cam->k_cov[1] * w0 / ww : 0.0;
        kl[2] = ww > 0.0 ? cam->k_cov[1] * w1 / ww : 0.0;
    }

    or_metric(a, flat, fr->xc, g, gi);
    velocity_from_normal(a, flat, fr->xc, fr->ut_cks, fr->u);
    for (i = 0; i < 4; ++i) {
        ul[i] = 0.0;
        for (j = 0; j < 4; ++j) ul[i] += g[4 * i + j] * fr->u[j];
    }
    /* k_t from the null condition, future directed */
    A = gi[0];
    B = gi[1] * kl[1] + gi[2] * kl[2] + gi[3] * kl[3];
    C = 0.0;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) C += gi[4 * (1 + i) + 1 + j] * kl[1 + i] * kl[1 + j];
    kl[0] = (-B + sqrt(B * B - A * C)) / A;

    /* camera-frame metric */
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            gp[i][j] = g[4 * (1 + i) + 1 + j] - ul[1 + i] / ul[0] * g[1 + j]
                     - ul[1 + j] / ul[0] * g[1 + i]
                     + ul[1 + i] * ul[1 + j] * g[0] / (ul[0] * ul[0]);
            gpi[i][j] = gi[4 * (1 + i) + 1 + j] + fr->u[1 + i] * fr->u[1 + j];
        }
    /* line of sight */
    for (i = 0; i < 3; ++i) Kl[i] = kl[1 + i] - ul[1 + i] / ul[0] * kl[0];
    Kt = 0.0;
    for (i = 0; i < 4; ++i) Kt -= fr->u[i] * kl[i];
    nrm = 0.0;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) nrm += gpi[i][j] * Kl[i] * Kl[j];
    nrm = 1.0 / sqrt(nrm);
    for (i = 0; i < 3; ++i) Kl[i] *= nrm;
    Kt *= nrm;
    for (i = 0; i < 3; ++i) {
        Ku[i] = 0.0;
        for (j = 0; j < 3; ++j) Ku[i] += gpi[i][j] * Kl[j];
    }
    /* vertical */
    U[0] = 0.0; U[1] = 0.0; U[2] = 1.0;
    if (fr->xc[1] == 0.0 && fr->xc[2] == 0.0) { U[1] = 1.0; U[2] = 0.0; }
    UK = U[0] * Kl[0] + U[1] * Kl[1] + U[2] * Kl[2];
    for (i = 0; i < 3; ++i) vu[i] = U[i] - UK * Ku[i];
    for (i = 0; i < 3; ++i) {
        vl[i] = 0.0;
        for (j = 0; j < 3; ++j) vl[i] += gp[i][j] * vu[j];
    }
    nrm = 1.0 / sqrt(vl[0] * vu[0] + vl[1] * vu[1] + vl[2] * vu[2]);
    for (i = 0; i < 3; ++i) { vu[i] *= nrm; vl[i] *= nrm; }
    /* horizontal: h^a = D^-1/2 [a b c] v_b K_c */
    D = gp[0][0] * (gp[1][1] * gp[2][2] - gp[1][2] * gp[2][1])
      - gp[0][1] * (gp[1][0] * gp[2][2] - gp[1][2] * gp[2][0])
      + gp[0][2] * (gp[1][0] * gp[2][1] - gp[1][1] * gp[2][0]);
    hu[0] = (vl[1] * Kl[2] - vl[2] * Kl[1]) / sqrt(D);
    hu[1] = (vl[2] * Kl[0] - vl[0] * Kl[2]) / sqrt(D);
    hu[2] = (vl[0] * Kl[1] - vl[1] * Kl[0]) / sqrt(D);
    /* rotation and return to coordinate components:
       A^t = u^t A^t' - (u_a/u_t) A^a',  A^a = A^a' + u^a A^t' */
    {
        double Hp[3], Vp[3], cps = cos(cam->psi), sps = sin(cam->psi);
        for (i = 0; i < 3; ++i) {
            Hp[i] = hu[i] * cps - vu[i] * sps;
            Vp[i] = vu[i] * cps + hu[i] * sps;
        }
        fr->K[0] = fr->u[0] * Kt;
        fr->H[0] = 0.0;
        fr->V[0] = 0.0;
        for (b = 0; b < 3; ++b) {
            fr->K[0] -= ul[1 + b] / ul[0] * Ku[b];
            fr->H[0] -= ul[1 + b] / ul[0] * Hp[b];
            fr->V[0] -= ul[1 + b] / ul[0] * Vp[b];
        }
        for (i = 0; i < 3; ++i) {
            fr->K[1 + i] = Ku[i] + fr->u[1 + i] * Kt;
            fr->H[1 + i] = Hp[i];
            fr->V[1 + i] = Vp[i];
        }
    }
}

void or_camera_basis(const or_camera *cam, const or_spacetime *st, double out[20])
{
    cam_frame fr;
    camera_frame(cam, st, &fr);
    memcpy(out, fr.xc, 4 * sizeof(double));
    memcpy(out + 4, fr.u, 4 * sizeof(double));
    memcpy(out + 8, fr.K, 4 * sizeof(double));
    memcpy(out + 12, fr.H, 4 * sizeof(double));
    memcpy(out + 16, fr.V, 4 * sizeof(double));
}

/* Pixel state plus the pixel observer u_pix and the horizontal vector H
   (coordinate components) used for the camera Stokes basis. */
void or_camera_pixel(const or_camera *cam, const or_spacetime *st, int i, int j,
                     double y[8], double *n_norm, double upix[4], double Hv[4])
{
    cam_frame fr;
    double N = (double)cam->n, ap, bp, g[16], gi[16], ku[4], A, B, C;
    int al, be;
    camera_frame(cam, st, &fr);
    ap = ((double)i - N / 2.0 + 0.5) * cam->width / N;
    bp = ((double)j - N / 2.0 + 0.5) * cam->width / N;
    for (al = 0; al < 4; ++al) y[al] = fr.xc[al] + (ap * fr.H[al] + bp * fr.V[al]);
    or_metric(st->a, st->flat, y, g, gi);
    ku[1] = fr.K[1]; ku[2] = fr.K[2]; ku[3] = fr.K[3];
    A = g[0];
    B = g[1] * ku[1] + g[2] * ku[2] + g[3] * ku[3];
    C = 0.0;
    for (al = 1; al < 4; ++al)
        for (be = 1; be < 4; ++be) C += g[4 * al + be] * ku[al] * ku[be];
    ku[0] = (-B - sqrt(B * B - A * C)) / A;
    for (al = 0; al < 4; ++al) {
        y[4 + al] = 0.0;
        for (be = 0; be < 4; ++be) y[4 + al] += g[4 * al + be] * ku[be];
    }
    velocity_from_normal(st->a, st->flat, y, fr.ut_cks, upix);
    if (cam->freq_mode == 0) {
        *n_norm = cam->nu_hz / (-y[4]);
    } else {
        double ku_dot = 0.0;
        for (al = 0; al < 4; ++al) ku_dot += y[4 + al] * upix[al];
        *n_norm = cam->nu_hz / (-ku_dot);
    }
    memcpy(Hv, fr.H, 4 * sizeof(double));
}

void or_camera_ray(const or_camera *cam, const or_spacetime *st, int i, int j,
                   double y[8], double *n_norm)
{
    double upix[4], Hv[4];
    or_camera_pixel(cam, st, i, j, y, n_norm, upix, Hv);
}
