/*
 * trace.c -- adaptive Dormand-Prince RK5(4)7M geodesic integration (oracle).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper section 2.2: the tableau of Table "tab:dp", the error norm
 *   eps = max_m |y5_m - y4_m| / (f_abs + f_rel max(|y_init_m|, |y5_m|)),
 * eps > 1 rejects the step; the fourth-order midpoint of Shampine (1986) is
 * the sample state of the step.  Integration runs at negative lambda from the
 * camera and stops when r crosses the camera radius from below, or r < r_in.
 *
 * Readings (the paper cites Numerical Recipes for the controller and prints
 * no constants; it prints the midpoint row without its factor):
 *  - midpoint: y_mid = y0 + (h/2) sum_i bm_i k_i (the printed row sums to 1);
 *  - y5 - y4 is evaluated as h sum_i (b5_i - b4_i) k_i;
 *  - accept iff eps <= 1; new h = h * min(10, max(0.2, 0.9 eps^-1/5)),
 *    factor 10 when eps == 0; after a rejection h = h * max(0.2, 0.9 eps^-1/5)
 *    and the next accepted step may not grow h;
 *  - every step-size factor is rounded to a multiple of 1/4096, and the
 *    first trial step is h0 = -h0_frac * r_pix with r_pix rounded to a
 *    multiple of 2^-10: the error estimate is a sum with heavy cancellation,
 *    so its last bits are noise, and the rounding keeps that noise out of
 *    the step sequence (the sequence is then reproducible across compilers
 *    and hardware except where a factor sits on a rounding boundary);
 *  - stop with STEP_UNDERFLOW when |h| < 1e-14 (1 + |lambda|), MAXSTEPS when
 *    accepted + rejected trials reach max_steps, NONFINITE on a NaN/Inf state;
 *  - termination is tested on accepted steps: r_prev < r_cam <= r_new
 *    (ESCAPED) or r_new < r_in (CAPTURED); the overshooting step is kept.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static void tableau(double c[7], double A[7][7], double b5[7], double b4[7], double bm[7])
{
    memset(A, 0, sizeof(double) * 49);
    c[0] = 0.0; c[1] = 1.0 / 5.0; c[2] = 3.0 / 10.0; c[3] = 4.0 / 5.0;
    c[4] = 8.0 / 9.0; c[5] = 1.0; c[6] = 1.0;
    A[1][0] = 1.0 / 5.0;
    A[2][0] = 3.0 / 40.0;        A[2][1] = 9.0 / 40.0;
    A[3][0] = 44.0 / 45.0;       A[3][1] = -56.0 / 15.0;      A[3][2] = 32.0 / 9.0;
    A[4][0] = 19372.0 / 6561.0;  A[4][1] = -25360.0 / 2187.0; A[4][2] = 64448.0 / 6561.0;
    A[4][3] = -212.0 / 729.0;
    A[5][0] = 9017.0 / 3168.0;   A[5][1] = -355.0 / 33.0;     A[5][2] = 46732.0 / 5247.0;
    A[5][3] = 49.0 / 176.0;      A[5][4] = -5103.0 / 18656.0;
    A[6][0] = 35.0 / 384.0;      A[6][1] = 0.0;               A[6][2] = 500.0 / 1113.0;
    A[6][3] = 125.0 / 192.0;     A[6][4] = -2187.0 / 6784.0;  A[6][5] = 11.0 / 84.0;
    b5[0] = 35.0 / 384.0; b5[1] = 0.0; b5[2] = 500.0 / 1113.0; b5[3] = 125.0 / 192.0;
    b5[4] = -2187.0 / 6784.0; b5[5] = 11.0 / 84.0; b5[6] = 0.0;
    b4[0] = 5179.0 / 57600.0; b4[1] = 0.0; b4[2] = 7571.0 / 16695.0; b4[3] = 393.0 / 640.0;
    b4[4] = -92097.0 / 339200.0; b4[5] = 187.0 / 2100.0; b4[6] = 1.0 / 40.0;
    bm[0] = 6025192743.0 / 30085553152.0; bm[1] = 0.0;
    bm[2] = 51252292925.0 / 65400821598.0; bm[3] = -2691868925.0 / 45128329728.0;
    bm[4] = 187940372067.0 / 1594534317056.0; bm[5] = -1776094331.0 / 19743644256.0;
    bm[6] = 11237099.0 / 235043384.0;
}

void or_dp_tableau(double c[7], double A[49], double b5[7], double b4[7], double bm[7])
{
    double AA[7][7];
    tableau(c, AA, b5, b4, bm);
    memcpy(A, AA, sizeof(AA));
}

static void push_step(or_ray *ray, const double y0[8], const double ym[8],
                      const double y1[8], double h)
{
    double *p;
    if (ray->n_acc >= ray->cap) {
        int64_t nc = ray->cap ? 2 * ray->cap : 256;
        ray->steps = (double *)realloc(ray->steps, sizeof(double) * 25 * (size_t)nc);
        ray->cap = nc;
    }
    p = ray->steps + 25 * ray->n_acc;
    memcpy(p, y0, 8 * sizeof(double));
    memcpy(p + 8, ym, 8 * sizeof(double));
    memcpy(p + 16, y1, 8 * sizeof(double));
    p[24] = h;
}

void or_ray_free(or_ray *ray)
{
    free(ray->steps);
    ray->steps = NULL;
    ray->cap = 0;
}

/* Proper length rate of eq. (length): (g_pq k^p k^q)^(1/2) in the normal
   frame, k^p = k^a + beta^a k^t, beta^a = -g^{ta}/g^{tt}, g_pq = g_ab. */
double or_ds_dlambda(double a, int flat, const double y[8])
{
    double g[16], gi[16], ku[4], kp[3], s = 0.0;
    int al, be;
    or_metric(a, flat, y, g, gi);
    for (al = 0; al < 4; ++al) {
        ku[al] = 0.0;
        for (be = 0; be < 4; ++be) ku[al] += gi[4 * al + be] * y[4 + be];
    }
    for (al = 0; al < 3; ++al) kp[al] = ku[1 + al] + (-gi[1 + al] / gi[0]) * ku[0];
    for (al = 0; al < 3; ++al)
        for (be = 0; be < 3; ++be) s += g[4 * (1 + al) + 1 + be] * kp[al] * kp[be];
    return sqrt(s);
}

static int finite8(const double y[8])
{
    int m;
    for (m = 0; m < 8; ++m)
        if (!isfinite(y[m])) return 0;
    return 1;
}

/* The integration of one ray.  With tlog non-NULL every trial step is also
   logged (up to tcap of them; *tn receives the number of trials) as
   OR_TRIAL_LOG doubles: the state at the start of the trial y[8], the trial
   step h, its error norm eps and 1 if it was accepted, else 0. */
static int trace_impl(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
                      const double ystart[8], or_ray *ray, double *tlog, int64_t tcap, int64_t *tn)
{
    double c[7], A[7][7], b5[7], b4[7], bm[7];
    double y[8], k[7][8], ys[8], y5[8], ym[8], err[8];
    double h, lambda = 0.0, r_prev;
    int no_grow = 0, i, j, m;
    const double a = st->a;
    const int flat = st->flat;

    tableau(c, A, b5, b4, bm);
    memcpy(y, ystart, sizeof(y));
    ray->n_acc = ray->n_rej = 0;
    ray->status = OR_RUNNING;
    ray->s = 0.0;
    r_prev = or_ks_radius(a, y[1], y[2], y[3]);
    h = -in->h0_frac * (rint(r_prev * 1024.0) / 1024.0);
    or_geodesic_rhs(a, flat, y, k[0]);

    while (ray->status == OR_RUNNING) {
        double eps = 0.0;
        if (ray->n_acc + ray->n_rej >= in->max_steps) { ray->status = OR_MAXSTEPS; break; }
        if (fabs(h) < 1e-14 * (1.0 + fabs(lambda))) { ray->status = OR_UNDERFLOW; break; }
        /* stages 2..7 */
        for (i = 1; i < 7; ++i) {
            for (m = 0; m < 8; ++m) {
                double s = 0.0;
                for (j = 0; j < i; ++j) s += A[i][j] * k[j][m];
                ys[m] = y[m] + h * s;
            }
            or_geodesic_rhs(a, flat, ys, k[i]);
        }
        /* fifth-order value (= stage-7 point), error estimate, midpoint */
        for (m = 0; m < 8; ++m) {
            double s5 = 0.0, se = 0.0, sm = 0.0;
            for (j = 0; j < 7; ++j) {
                s5 += b5[j] * k[j][m];
                se += (b5[j] - b4[j]) * k[j][m];
                sm += bm[j] * k[j][m];
            }
            y5[m] = y[m] + h * s5;
            err[m] = h * se;
            ym[m] = y[m] + 0.5 * h * sm;
        }
        {
            int bad = 0;
            for (m = 0; m < 8; ++m) {
                double sc = in->f_abs + in->f_rel * fmax(fabs(y[m]), fabs(y5[m]));
                /* an exactly zero error is no error, also at zero tolerance */
                double e = (err[m] == 0.0) ? 0.0 : fabs(err[m]) / sc;
                if (isnan(e)) bad = 1;
                else if (e > eps) eps = e;
            }
            if (bad || !finite8(y5)) { ray->status = OR_NONFINITE; break; }
        }
        if (tlog) {
            int64_t t = ray->n_acc + ray->n_rej;
            if (t < tcap) {
                double *q = tlog + OR_TRIAL_LOG * t;
                memcpy(q, y, 8 * sizeof(double));
                q[8] = h;
                q[9] = eps;
                q[10] = eps <= 1.0 ? 1.0 : 0.0;
            }
        }
        if (eps <= 1.0) {
            double fac, r_new;
            push_step(ray, y, ym, y5, h);
            ray->n_acc++;
            lambda += h;
            ray->s += fabs(h) * or_ds_dlambda(a, flat, ym);
            fac = (eps == 0.0) ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * pow(eps, -0.2)));
            fac = rint(fac * 4096.0) / 4096.0;
            if (no_grow) fac = fmin(fac, 1.0);
            no_grow = 0;
            memcpy(y, y5, sizeof(y));
            memcpy(k[0], k[6], sizeof(k[0]));   /* first-same-as-last */
            r_new = or_ks_radius(a, y[1], y[2], y[3]);
            if (r_new < st->r_in) ray->status = OR_CAPTURED;
            else if (r_prev < cam->r && r_new >= cam->r) ray->status = OR_ESCAPED;
            r_prev = r_new;
            h *= fac;
        } else {
            ray->n_rej++;
            h *= rint(fmax(0.2, 0.9 * pow(eps, -0.2)) * 4096.0) / 4096.0;
            no_grow = 1;
        }
    }
    memcpy(ray->y_end, y, sizeof(y));
    ray->lambda = fabs(lambda);
    ray->dt = ystart[0] - y[0];
    if (tn) *tn = ray->n_acc + ray->n_rej;
    return ray->status;
}

int or_trace(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
             const double ystart[8], or_ray *ray)
{
    return trace_impl(cam, st, in, ystart, ray, NULL, 0, NULL);
}

int64_t or_trace_trials(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
                        int i, int j, double *trials_out, int64_t cap, double info[8])
{
    or_ray ray;
    double y[8], n;
    int64_t nt = 0;
    memset(&ray, 0, sizeof(ray));
    or_camera_ray(cam, st, i, j, y, &n);
    trace_impl(cam, st, in, y, &ray, trials_out, cap, &nt);
    info[0] = (double)ray.n_acc; info[1] = (double)ray.n_rej; info[2] = ray.status;
    info[3] = ray.lambda; info[4] = ray.s; info[5] = ray.dt;
    info[6] = or_ks_radius(st->a, ray.y_end[1], ray.y_end[2], ray.y_end[3]);
    info[7] = n;
    or_ray_free(&ray);
    return nt;
}

int64_t or_trace_pixel(const or_camera *cam, const or_spacetime *st,
                       const or_integrator *in, int i, int j,
                       double *steps_out, int64_t max_steps,
                       double info[8], double y_end[8])
{
    or_ray ray;
    double y[8], n;
    int64_t ncopy;
    memset(&ray, 0, sizeof(ray));
    or_camera_ray(cam, st, i, j, y, &n);
    or_trace(cam, st, in, y, &ray);
    ncopy = ray.n_acc < max_steps ? ray.n_acc : max_steps;
    if (steps_out && ncopy > 0) memcpy(steps_out, ray.steps, sizeof(double) * 25 * (size_t)ncopy);
    info[0] = (double)ray.n_acc; info[1] = (double)ray.n_rej; info[2] = ray.status;
    info[3] = ray.lambda; info[4] = ray.s; info[5] = ray.dt;
    info[6] = or_ks_radius(st->a, ray.y_end[1], ray.y_end[2], ray.y_end[3]);
    info[7] = n;
    memcpy(y_end, ray.y_end, sizeof(ray.y_end));
    or_ray_free(&ray);
    return ncopy;
}
