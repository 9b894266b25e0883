/*
 * render.c -- whole-pixel pipeline (oracle): camera ray, DP geodesic,
 * sampling of the accepted steps, transfer from source to camera.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sampling (paper section 2.2, last paragraph; section 2.5): each accepted
 * step is represented by its fourth-order midpoint; steps longer than the
 * proper-length limit are subdivided with the quartic through y0, y1, f0, f1
 * and y_mid.  Readings:
 *  - a step is sampled against the grid when the chords y0-y_mid or
 *    y_mid-y1 meet the grid's bounding box (closed, axis aligned); it is
 *    then cut into n = ceil(ds/ds_max) pieces of equal
 *    lambda, ds = |h| (g_pq k^p k^q)^1/2 at y_mid; piece p covers
 *    theta in [p/n, (p+1)/n] (theta = 0 at y0, the camera side); its sample
 *    is the quartic at the piece centre (y_mid itself when n = 1);
 *  - any other step is one vacuum record (sample y_mid, length |h|);
 *  - unpolarised transfer uses the plasma records only;
 *  - polarised transfer starts at the first plasma record from the source
 *    (N = 0 before it) and keeps every later record; consecutive half
 *    transport substeps are merged into one explicit-midpoint step of length
 *    (dl_prev + dl)/2 with the predictor at the previous sample and the
 *    corrector at the boundary between the two records; the last record is
 *    followed by a half-length transport to x_pix (corrector at x_pix);
 *  - the plasma substep projects N on the tetrad (I = N11 + N22,
 *    Q = N11 - N22, U = 2 Re N12, V = -2 Im N12), applies the exact
 *    constant-coefficient solution over the physical length, or S = M^-1 J
 *    when alpha_I dl >= 100, and rebuilds N from S; a record with all
 *    coefficients zero leaves N unchanged;
 *  - lengths: dl_phys = L dl / n with L = G M/c^2 (cm), so that
 *    alpha_I dl_phys = alpha_nu (proper length in the fluid frame);
 *  - camera Stokes: tetrad at x_pix of the pixel observer with e2 = -H,
 *    hence e1 = V: Q > 0 along the vertical, U > 0 towards -H;
 *    I_nu = nu^3 I;
 *  - auxiliary: dt = t_pix - t_end, s = sum ds, lambda = sum |h| over the
 *    whole ray, tau = sum alpha_I dl_phys, I_j = nu^3 sum j_I dl_phys over
 *    plasma records; the number of records (pieces and vacuum steps).
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define C_LIGHT 2.99792458e10
#define G_NEWTON 6.67430e-8
#define M_SUN 1.98841e33

double or_ds_dlambda(double a, int flat, const double y[8]);
void or_camera_pixel(const or_camera *cam, const or_spacetime *st, int i, int j,
                     double y[8], double *n_norm, double upix[4], double Hv[4]);
void or_tetrad(const double g[16], const double gi[16], const double u[4],
               const double kcov[4], const double w[4], double e[4][4]);
void or_solve4(const double M[16], const double J[4], double x[4]);

typedef struct {
    double ys[8];     /* sample state                         */
    double yb[8];     /* boundary on the camera side          */
    double dl;        /* piece length in lambda (> 0)         */
    int in_box;       /* sampled against the grid             */
} record;

/* quartic dense output p(theta) through y0, y1, f0, f1, ymid */
void or_dense_quartic(const double y0[8], const double y1[8], const double f0[8],
                    const double f1[8], const double ym[8], double h, double th,
                    double out[8])
{
    int m;
    for (m = 0; m < 8; ++m) {
        double A = y1[m] - y0[m] - h * f0[m];
        double B = h * (f1[m] - f0[m]);
        double C = 16.0 * (ym[m] - y0[m]) - 8.0 * h * f0[m];
        double c2 = -5.0 * A + B + C, c3 = 14.0 * A - 3.0 * B - 2.0 * C;
        double c4 = -8.0 * A + 2.0 * B + C;
        out[m] = y0[m] + th * h * f0[m] + c2 * th * th + c3 * th * th * th
               + c4 * th * th * th * th;
    }
}

/* does the straight chord from p to q (spatial parts of states) meet the box? */
static int chord_meets_box(const double bb[6], const double p[8], const double q[8])
{
    double t0 = 0.0, t1 = 1.0;
    int d;
    for (d = 0; d < 3; ++d) {
        double a = p[1 + d], dd = q[1 + d] - p[1 + d];
        if (dd == 0.0) {
            if (a < bb[2 * d] || a > bb[2 * d + 1]) return 0;
        } else {
            double ta = (bb[2 * d] - a) / dd, tb = (bb[2 * d + 1] - a) / dd;
            if (ta > tb) { double t = ta; ta = tb; tb = t; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
            if (t0 > t1) return 0;
        }
    }
    return 1;
}

/* Records of the whole ray in source-to-camera order. */
static record *make_records(const or_spacetime *st, const or_integrator *in,
                            const or_grid *gr, const or_ray *ray, int64_t *n_rec)
{
    double bb[6] = {1e300, -1e300, 1e300, -1e300, 1e300, -1e300};
    int64_t cap = 64, n = 0, s;
    record *rec = (record *)malloc(sizeof(record) * (size_t)cap);
    int b, d;
    for (b = 0; b < gr->n_blocks; ++b)
        for (d = 0; d < 3; ++d) {
            bb[2 * d] = fmin(bb[2 * d], gr->bounds[6 * b + 2 * d]);
            bb[2 * d + 1] = fmax(bb[2 * d + 1], gr->bounds[6 * b + 2 * d + 1]);
        }
    for (s = ray->n_acc - 1; s >= 0; --s) {
        const double *y0 = ray->steps + 25 * s, *ym = y0 + 8, *y1 = y0 + 16;
        double h = y0[24];
        int inb = chord_meets_box(bb, y0, ym) || chord_meets_box(bb, ym, y1);
        int64_t nsub = 1, p;
        double f0[8], f1[8];
        if (inb) {
            double ds = fabs(h) * or_ds_dlambda(st->a, st->flat, ym);
            if (in->ds_max > 0.0) {
                /* at most 2^24 pieces per step; a non-finite length gives one */
                double q = ceil(ds / in->ds_max);
                nsub = (q >= 1.0) ? (int64_t)fmin(q, 16777216.0) : 1;
            }
            if (nsub > 1) {
                or_geodesic_rhs(st->a, st->flat, y0, f0);
                or_geodesic_rhs(st->a, st->flat, y1, f1);
            }
        }
        for (p = nsub - 1; p >= 0; --p) {
            record *r;
            if (n >= cap) { cap *= 2; rec = (record *)realloc(rec, sizeof(record) * (size_t)cap); }
            r = rec + n++;
            r->in_box = inb;
            r->dl = fabs(h) / (double)nsub;
            if (nsub == 1) memcpy(r->ys, ym, sizeof(r->ys));
            else or_dense_quartic(y0, y1, f0, f1, ym, h, ((double)p + 0.5) / (double)nsub, r->ys);
            if (p == 0) memcpy(r->yb, y0, sizeof(r->yb));
            else or_dense_quartic(y0, y1, f0, f1, ym, h, (double)p / (double)nsub, r->yb);
        }
    }
    *n_rec = n;
    return rec;
}

static void transport_step(const or_spacetime *st, const double ya[8], const double yb[8],
                           double dl, double Nre[16], double Nim[16])
{
    double dR[16], dI[16], hR[16], hI[16];
    int m;
    or_transport_rhs(st->a, st->flat, ya, Nre, Nim, dR, dI);
    for (m = 0; m < 16; ++m) { hR[m] = Nre[m] + 0.5 * dl * dR[m]; hI[m] = Nim[m] + 0.5 * dl * dI[m]; }
    or_transport_rhs(st->a, st->flat, yb, hR, hI, dR, dI);
    for (m = 0; m < 16; ++m) { Nre[m] += dl * dR[m]; Nim[m] += dl * dI[m]; }
}

/* Stokes parameters of N in tetrad e (e1, e2 spatial screen vectors). */
static void n_to_stokes(const double g[16], double e[4][4], const double Nre[16],
                        const double Nim[16], double S[4])
{
    double e1l[4], e2l[4], n11 = 0, n22 = 0, n12r = 0, n12i = 0;
    int al, be;
    for (al = 0; al < 4; ++al) {
        e1l[al] = 0.0; e2l[al] = 0.0;
        for (be = 0; be < 4; ++be) { e1l[al] += g[4 * al + be] * e[1][be]; e2l[al] += g[4 * al + be] * e[2][be]; }
    }
    for (al = 0; al < 4; ++al)
        for (be = 0; be < 4; ++be) {
            n11 += e1l[al] * e1l[be] * Nre[4 * al + be];
            n22 += e2l[al] * e2l[be] * Nre[4 * al + be];
            n12r += e1l[al] * e2l[be] * Nre[4 * al + be];
            n12i += e1l[al] * e2l[be] * Nim[4 * al + be];
        }
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = 2.0 * n12r;
    S[3] = -2.0 * n12i;
}

static void stokes_to_n(double e[4][4], const double S[4], double Nre[16], double Nim[16])
{
    double n11 = 0.5 * (S[0] + S[1]), n22 = 0.5 * (S[0] - S[1]);
    double n12r = 0.5 * S[2], n12i = -0.5 * S[3];
    int al, be;
    for (al = 0; al < 4; ++al)
        for (be = 0; be < 4; ++be) {
            Nre[4 * al + be] = n11 * e[1][al] * e[1][be] + n22 * e[2][al] * e[2][be]
                             + n12r * (e[1][al] * e[2][be] + e[2][al] * e[1][be]);
            Nim[4 * al + be] = n12i * (e[1][al] * e[2][be] - e[2][al] * e[1][be]);
        }
}

/* Running sums of the averaged quantities (section 4.6, Auxiliary Images) at a
   plasma sample with outputs c of or_sample_point, affine length dl,
   emission increment dj and depth dtau: sl[k] += q dl, sj[k] += q dj and
   qt[k] += (q - qt[k])(1 - e^-dtau). */
static void accumulate_averages(const double *c, double dl, double dj, double dtau,
                                double sl[7], double sj[7], double qt[7])
{
    const double q[7] = {c[30], c[8], c[31], c[9], c[10], c[29], c[32]};
    const double w = -expm1(-dtau);
    int k;
    for (k = 0; k < 7; ++k) {
        sl[k] += q[k] * dl;
        sj[k] += q[k] * dj;
        qt[k] += (q[k] - qt[k]) * w;
    }
}

static void render_one(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
                       const or_grid *gr, const or_plasma *pl, int64_t pix,
                       double img[4], double aux[OR_NAUX], double *avg)
{
    double sl[7] = {0}, sj[7] = {0}, qt[7] = {0};
    int i = (int)(pix % cam->n), j = (int)(pix / cam->n);
    double y[8], n_norm, upix[4], Hv[4];
    double L = G_NEWTON * st->mass_msun * M_SUN / (C_LIGHT * C_LIGHT);
    double nu3 = cam->nu_hz * cam->nu_hz * cam->nu_hz;
    double tau = 0.0, Ij = 0.0;
    int64_t n_rec = 0, r, n_samp = 0;
    or_ray ray;
    record *rec;
    int m;

    memset(&ray, 0, sizeof(ray));
    or_camera_pixel(cam, st, i, j, y, &n_norm, upix, Hv);
    or_trace(cam, st, in, y, &ray);
    rec = make_records(st, in, gr, &ray, &n_rec);
    for (m = 0; m < 4; ++m) img[m] = 0.0;

    if (!pl->polarized) {
        double I = 0.0;
        for (r = 0; r < n_rec; ++r) {
            double c[33], dlp;
            if (!rec[r].in_box) continue;
            or_sample_point(st, gr, pl, rec[r].ys, n_norm, c);
            if (c[28] == 0.0) continue;
            n_samp++;
            dlp = L * rec[r].dl / n_norm;
            I = or_unpol_segment(I, c[0], c[3], dlp);
            tau += c[3] * dlp;
            Ij += c[0] * dlp;
            if (avg) accumulate_averages(c, rec[r].dl, c[0] * dlp, c[3] * dlp, sl, sj, qt);
        }
        img[0] = nu3 * I;
    } else {
        double Nre[16], Nim[16];
        int started = 0;
        int64_t prev = -1;
        memset(Nre, 0, sizeof(Nre));
        memset(Nim, 0, sizeof(Nim));
        for (r = 0; r < n_rec; ++r) {
            double c[33];
            int plasma = 0;
            if (rec[r].in_box) {
                or_sample_point(st, gr, pl, rec[r].ys, n_norm, c);
                plasma = c[28] != 0.0;
            }
            if (!started && !plasma) continue;
            if (started) transport_step(st, rec[prev].ys, rec[prev].yb,
                                        0.5 * (rec[prev].dl + rec[r].dl), Nre, Nim);
            started = 1;
            prev = r;
            if (plasma) {
                double dlp = L * rec[r].dl / n_norm;
                double g[16], gi[16], e[4][4], S[4], S1[4], J[4], M[16];
                int q;
                n_samp++;
                tau += c[3] * dlp;
                Ij += c[0] * dlp;
                if (avg) accumulate_averages(c, rec[r].dl, c[0] * dlp, c[3] * dlp, sl, sj, qt);
                for (q = 0; q < 8; ++q)
                    if (c[q] != 0.0) break;
                if (q == 8) continue;   /* all coefficients zero: identity */
                or_metric(st->a, st->flat, rec[r].ys, g, gi);
                for (q = 0; q < 4; ++q)
                    for (m = 0; m < 4; ++m) e[q][m] = c[12 + 4 * q + m];
                n_to_stokes(g, e, Nre, Nim, S);
                J[0] = c[0]; J[1] = c[1]; J[2] = 0.0; J[3] = c[2];
                /* M rows: (aI aQ aU aV), (aQ aI rV -rU), (aU -rV aI rQ), (aV rU -rQ aI) */
                M[0] = c[3];  M[1] = c[4];  M[2] = 0.0;   M[3] = c[5];
                M[4] = c[4];  M[5] = c[3];  M[6] = c[7];  M[7] = 0.0;
                M[8] = 0.0;   M[9] = -c[7]; M[10] = c[3]; M[11] = c[6];
                M[12] = c[5]; M[13] = 0.0;  M[14] = -c[6]; M[15] = c[3];
                if (c[3] * dlp >= 100.0) or_solve4(M, J, S1);
                else or_stokes_exact(S, J, M, dlp, S1);
                stokes_to_n(e, S1, Nre, Nim);
            }
        }
        if (started) {
            double g[16], gi[16], e[4][4], mH[4], S[4];
            transport_step(st, rec[prev].ys, y, 0.5 * rec[prev].dl, Nre, Nim);
            or_metric(st->a, st->flat, y, g, gi);
            for (m = 0; m < 4; ++m) mH[m] = -Hv[m];
            or_tetrad(g, gi, upix, y + 4, mH, e);
            n_to_stokes(g, e, Nre, Nim, S);
            for (m = 0; m < 4; ++m) img[m] = nu3 * S[m];
        }
    }
    if (avg) {
        for (m = 0; m < 7; ++m) {
            avg[m] = sl[m] / ray.lambda;
            avg[7 + m] = Ij > 0.0 ? sj[m] / Ij : 0.0;
            avg[14 + m] = qt[m];
        }
    }
    aux[OR_AUX_DT] = ray.dt;
    aux[OR_AUX_S] = ray.s;
    aux[OR_AUX_LAMBDA] = ray.lambda;
    aux[OR_AUX_TAU] = tau;
    aux[OR_AUX_IJ] = nu3 * Ij;
    aux[OR_AUX_NACC] = (double)ray.n_acc;
    aux[OR_AUX_NREJ] = (double)ray.n_rej;
    aux[OR_AUX_STATUS] = (double)ray.status;
    aux[OR_AUX_NSAMP] = (double)n_samp;
    aux[OR_AUX_NREC] = (double)n_rec;
    free(rec);
    or_ray_free(&ray);
}

typedef struct {
    const or_camera *cam; const or_spacetime *st; const or_integrator *in;
    const or_grid *gr; const or_plasma *pl;
    int64_t n_pix; const int64_t *pix; double *image, *aux, *avg;
    int64_t next;
    pthread_mutex_t lock;
} job;

static void *worker(void *arg)
{
    job *jb = (job *)arg;
    for (;;) {
        int64_t p;
        pthread_mutex_lock(&jb->lock);
        p = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (p >= jb->n_pix) break;
        render_one(jb->cam, jb->st, jb->in, jb->gr, jb->pl, jb->pix[p],
                   jb->image + 4 * p, jb->aux + OR_NAUX * p, jb->avg ? jb->avg + OR_NAVG * p : NULL);
    }
    return NULL;
}

void or_render_pixels(const or_camera *cam, const or_spacetime *st,
                      const or_integrator *in, const or_grid *gr,
                      const or_plasma *pl, int64_t n_pix, const int64_t *pix,
                      double *image, double *aux, double *avg, int n_threads)
{
    job jb;
    pthread_t th[256];
    int t;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    jb.cam = cam; jb.st = st; jb.in = in; jb.gr = gr; jb.pl = pl;
    jb.n_pix = n_pix; jb.pix = pix; jb.image = image; jb.aux = aux; jb.avg = avg; jb.next = 0;
    pthread_mutex_init(&jb.lock, NULL);
    for (t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, &jb);
    for (t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);
}
