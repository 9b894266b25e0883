/*
 * oracle.h -- plain, slow, FP64 CPU reference of the Blacklight ray-tracing
 * hot path (White 2022, "Blacklight: A General-Relativistic Ray-Tracing and
 * Analysis Tool", arXiv:2203.15963).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this code; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Units: geometric lengths in units of M (G = c = M = 1) for geometry; CGS
 * for plasma and radiation (paper, section 1, last paragraph).
 *
 * Every function is written from the paper's definitions, in the paper's
 * order, with no fusion or reordering beyond what the definition states.
 * Readings of passages the paper leaves open are listed where they are used.
 */
#ifndef BL_ORACLE_H
#define BL_ORACLE_H

#include <stdint.h>

#define OR_NAUX 10
/* auxiliary map order */
enum { OR_AUX_DT = 0, OR_AUX_S, OR_AUX_LAMBDA, OR_AUX_TAU, OR_AUX_IJ,
       OR_AUX_NACC, OR_AUX_NREJ, OR_AUX_STATUS, OR_AUX_NSAMP, OR_AUX_NREC };

/* per-ray termination status */
enum { OR_RUNNING = 0, OR_ESCAPED = 1, OR_CAPTURED = 2, OR_MAXSTEPS = 3,
       OR_UNDERFLOW = 4, OR_NONFINITE = 5 };

typedef struct {
    double r, theta, phi;   /* camera centre, spherical Kerr-Schild        */
    double u_normal[3];     /* u^p, spherical-KS normal frame              */
    double k_cov[3];        /* k_i, spherical KS, unnormalised             */
    double width;           /* w                                           */
    int32_t n;              /* N (pixels per side)                         */
    int32_t freq_mode;      /* 0: nu at infinity, 1: nu at the camera      */
    double psi;             /* rotation about the line of sight            */
    double nu_hz;           /* observing frequency                         */
} or_camera;

typedef struct {
    double a;               /* spin a/M                                    */
    double mass_msun;       /* black-hole mass for the CGS length unit     */
    double r_in;            /* inner termination radius                    */
    int32_t flat;           /* 1: replace g by Minkowski (paper sec. 4.2)  */
    int32_t pad;
} or_spacetime;

typedef struct {
    double f_abs, f_rel;    /* DP tolerances                                */
    double ds_max;          /* proper-length limit per transfer piece       */
    double h0_frac;         /* first trial step = -h0_frac * r_pix          */
    int64_t max_steps;      /* cap on trial steps (accepted + rejected)     */
} or_integrator;

typedef struct {
    int32_t n_blocks, bnx, bny, bnz;
    const double *bounds;   /* [n_blocks][6] = x0,x1,y0,y1,z0,z1            */
    const double *prims;    /* [n_blocks][bnz][bny][bnx][8]:
                               rho, p, u~x, u~y, u~z, Bx, By, Bz (code)     */
    double rho_unit;        /* g cm^-3 per code density unit                */
} or_grid;

/* Data cuts (paper section 4.1, Data Cuts): a sample whose rho, n_e, p,
   Theta_e, B, sigma, beta^-1 or Kerr-Schild r lies below its lower or above
   its upper limit is vacuum, and with a plane cut so is every sample on one
   side of the plane (x - x0).n = 0 (CKS x, y, z).  Limits of -inf / +inf
   leave a quantity uncut.  Units: rho and p as in the grid (code units), n_e
   in cm^-3, B in gauss, r in GM/c^2. */
enum { OR_CUT_RHO, OR_CUT_NE, OR_CUT_P, OR_CUT_THETAE, OR_CUT_B, OR_CUT_SIGMA, OR_CUT_BETAINV, OR_CUT_R,
       OR_NCUT };

typedef struct {
    double mu, ne_ni, r_high, r_low, sigma_max;
    int32_t polarized;      /* 0: I only, 1: I,Q,U,V                        */
    int32_t interp;         /* 0: nearest cell, 1: trilinear within a block */
    int32_t use_cuts;       /* 0: only sigma_max                            */
    int32_t plane;          /* 0: no plane; +1: (x - x0).n < 0 is vacuum;
                               -1: (x - x0).n > 0 is vacuum                 */
    double cut_lo[OR_NCUT], cut_hi[OR_NCUT];
    double plane_x0[3], plane_n[3];
    /* electron populations (paper sections 2.6, 4.5): fractions of n_e in
       the thermal, power-law and kappa distributions (non-negative, summing
       to 1), power-law index and cutoffs, kappa index and width */
    double frac[3];
    double pl_p, pl_gmin, pl_gmax, kappa, kappa_w;
    /* filled by or_nonthermal_prepare from the parameters above:
       power law: (p-1)/(gmin^(1-p) - gmax^(1-p)); kappa: the normalisation A,
       the moments <gamma^-2/3>, <gamma^-5/3> of the normalised distribution */
    double pl_norm, kap_norm, kap_m23, kap_m53;
} or_plasma;

/* ---- geometry (kerr.c) ---- */
double or_ks_radius(double a, double x, double y, double z);
void   or_metric(double a, int flat, const double x[4], double g[16], double gi[16]);
void   or_metric_deriv(double a, int flat, const double x[4],
                       double dg[48], double dgi[48]);
void   or_christoffel(double a, int flat, const double x[4], double gam[64]);
void   or_geodesic_rhs(double a, int flat, const double y[8], double dy[8]);
/* proper-length rate (g_pq k^p k^q)^1/2 of eq. (length) */
double or_ds_dlambda(double a, int flat, const double y[8]);

/* ---- Dormand-Prince tableau (dp.c) ---- */
void   or_dp_tableau(double c[7], double A[49], double b5[7], double b4[7], double bm[7]);

/* ---- camera (camera.c) ---- */
/* Basis in coordinate components: K[4], H[4], V[4], u[4] (contravariant),
   x_c[4]; returned packed as out[0..19] = xc,u,K,H,V.                      */
void   or_camera_basis(const or_camera *cam, const or_spacetime *st, double out[20]);
/* Initial state of pixel (i,j): y[8] = x^alpha, k_alpha; *n_norm = n.      */
void   or_camera_ray(const or_camera *cam, const or_spacetime *st, int i, int j,
                     double y[8], double *n_norm);

/* ---- geodesic integration (trace.c) ---- */
typedef struct {
    int64_t n_acc, n_rej;
    int32_t status;
    double y_end[8];
    double lambda, s, dt;
    /* accepted steps: y0[8], ymid[8], y1[8], h  (25 doubles per step)      */
    double *steps;
    int64_t cap;
} or_ray;
int    or_trace(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
                const double y0[8], or_ray *ray);
void   or_ray_free(or_ray *ray);
/* Trace pixel (i,j) and log every trial step (at most cap of them) into
   trials_out as OR_TRIAL_LOG doubles each: state at the trial's start y[8],
   trial step h, error norm eps, accepted (1) or rejected (0).  Returns the
   number of trials; info[8] as for or_trace_pixel.                         */
#define OR_TRIAL_LOG 11
int64_t or_trace_trials(const or_camera *cam, const or_spacetime *st, const or_integrator *in,
                        int i, int j, double *trials_out, int64_t cap, double info[8]);
/* Trace pixel (i,j) and copy at most max_steps accepted step records
   (25 doubles each) into steps_out.  Returns n_acc; fills info[8] =
   n_acc, n_rej, status, lambda, s, dt, r_end, 0 and y_end[8].             */
int64_t or_trace_pixel(const or_camera *cam, const or_spacetime *st,
                       const or_integrator *in, int i, int j,
                       double *steps_out, int64_t max_steps,
                       double info[8], double y_end[8]);

/* ---- grid lookup and plasma (plasma.c) ---- */
int    or_grid_sample(const or_grid *gr, int interp, const double x[3], double prim[8]);
double or_bessel_k_scaled(int n, double x);   /* e^x K_n(x) */
void   or_thermal_coeffs(double ne, double thetae, double B, double nu,
                         double cos_theta, int polarized, double out[8]);
/* Nonthermal populations (plasma.c): or_nonthermal_prepare fills the
   distribution constants of pl; or_nonthermal_coeffs gives the fluid-frame
   coefficients (as or_thermal_coeffs) of n_e electrons in distribution kind
   (1: power law, 2: kappa).  or_kappa_integral is the integral over gamma of
   gamma^s dn/dgamma / (n_e A) for the kappa distribution (s = 0 gives 1/A). */
void   or_nonthermal_prepare(or_plasma *pl);
double or_kappa_integral(double kappa, double w, double s);
void   or_nonthermal_coeffs(int kind, const or_plasma *pl, double ne, double B, double nu,
                            double cos_theta, int polarized, double out[8]);
/* Everything at one sample point: state y[8], normalisation n.
   out[0..7]   = jI, jQ, jV, aI, aQ, aV, rQ, rV  (invariant: j/nu^2, a*nu)
   out[8..11]  = ne, thetae, B_gauss, nu_fluid
   out[12..27] = tetrad e0..e3 (contravariant, 4 each)
   out[28]     = 1 if the point holds emitting plasma, else 0 (vacuum)
   out[29]     = sigma
   out[30..32] = rho, p (code units) and beta^-1 = b^2/(2p) (plasma only)   */
void   or_sample_point(const or_spacetime *st, const or_grid *gr, const or_plasma *pl,
                       const double y[8], double n_norm, double out[33]);

/* ---- transfer pieces (transfer.c) ---- */
double or_unpol_segment(double I, double j, double alpha, double dl);
void   or_stokes_exact(const double S0[4], const double J[4], const double M[16],
                       double s, double S1[4]);
void   or_transport_rhs(double a, int flat, const double y[8],
                        const double Nre[16], const double Nim[16],
                        double dRe[16], double dIm[16]);

/* ---- whole pixels (render.c) ---- */
/* quartic through y0, y1, f0 = y'(0), f1 = y'(1) (per unit lambda) and the
   midpoint ym over a step h, evaluated at fraction theta of the step */
void   or_dense_quartic(const double y0[8], const double y1[8], const double f0[8],
                        const double f1[8], const double ym[8], double h, double theta,
                        double out[8]);
/* Averaged quantities (paper section 4.6, Auxiliary Images): for q in rho, n_e,
   p, Theta_e, B, sigma, beta^-1 (index k), avg[k] = <q>_lambda =
   (1/lambda) int q dlambda over the plasma samples, avg[7 + k] = <q>_Ij =
   int q j_I dlambda / int j_I dlambda (0 without emission), avg[14 + k] =
   <q>_tau, the solution of d<q>/dtau = q - <q> from 0 at the source end,
   advanced over a sample of depth dtau as <q> += (q - <q>)(1 - e^-dtau). */
#define OR_NAVG 21

/* Render the listed pixels (index = i + N*j).  image[p][4] holds I,Q,U,V
   (I_nu units, erg s^-1 cm^-2 sr^-1 Hz^-1); aux[p][OR_NAUX]; avg (or NULL)
   [p][OR_NAVG] the averaged quantities.                                     */
void   or_render_pixels(const or_camera *cam, const or_spacetime *st,
                        const or_integrator *in, const or_grid *gr,
                        const or_plasma *pl, int64_t n_pix, const int64_t *pix,
                        double *image, double *aux, double *avg, int n_threads);

#endif
