/*
 * blgpu.h -- C ABI of the MI355X (gfx950) implementation of the Blacklight
 * ray-tracing hot path (C. J. White 2022, "Blacklight: A General-Relativistic
 * Ray-Tracing and Analysis Tool", arXiv:2203.15963).
 *
 * For every camera pixel the library integrates a null geodesic of the Kerr
 * metric in Cartesian Kerr-Schild coordinates with adaptive Dormand-Prince
 * RK5(4) steps (paper section 2.2), samples GRMHD-like cell data on the ray
 * (section 2.5), evaluates thermal synchrotron coefficients (section 2.6) and
 * integrates the unpolarized (section 2.3) or polarized (section 2.4,
 * Strang-split coordinate/plasma terms) transfer equation from source to
 * camera.  The camera is the plane-parallel camera of section 2.1.
 *
 * Conventions
 *  - Units: lengths, times and the affine parameter in M (G = c = 1, M = 1);
 *    plasma and radiation in CGS.  Images hold I_nu, Q_nu, U_nu, V_nu in
 *    erg s^-1 cm^-2 sr^-1 Hz^-1.
 *  - Ownership: the caller owns every buffer it passes; the library never
 *    frees caller memory.  Pointers documented "device" must be device
 *    memory of the context's GPU; "host" pointers are read during the call
 *    only.  A bl_grid borrows the caller's device primitive array, which must
 *    stay alive and unchanged while the grid is used.
 *  - Asynchrony: every call that launches work enqueues it on the context's
 *    stream and returns; the caller synchronises the stream before reading
 *    outputs.  Calls on one context must not overlap in time from several
 *    host threads.
 *  - Errors: calls return a bl_status and never abort or throw across the
 *    ABI; bl_last_error() holds a message for the last non-OK status.  Per-ray
 *    numerical outcomes go to the status auxiliary map, not to the return code.
 *  - Layout: images are row-major [stokes][j][i] with i the horizontal pixel
 *    index (offset a along H) and j the vertical one (offset b along V).
 */
#ifndef BLGPU_H
#define BLGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLGPU_ABI_VERSION 2

typedef enum {
    BL_OK = 0,
    BL_E_INVALID_ARG = -1,   /* a pointer, size or parameter is invalid       */
    BL_E_DEVICE = -2,        /* a HIP runtime call failed                      */
    BL_E_OOM = -3,           /* device memory for the workspace is exhausted   */
    BL_E_UNSUPPORTED = -4,   /* a valid request this version does not support  */
    BL_E_STATE = -5          /* the call needs state the context does not hold
                                (no step network installed, a grid of another
                                context)                                      */
} bl_status;

/* Auxiliary maps, each [N][N] doubles, in this order (paper section 4.6,
   Auxiliary Images:
   elapsed time, proper length, affine parameter, optical depth and
   integrated emissivity; plus step counts, status and sample counts). */
#define BL_NAUX 10
enum {
    BL_AUX_DT = 0,       /* t_pixel - t_end (Kerr-Schild t)                     */
    BL_AUX_S = 1,        /* proper length sum of |h| (g_pq k^p k^q)^1/2        */
    BL_AUX_LAMBDA = 2,   /* affine length sum of |h|                           */
    BL_AUX_TAU = 3,      /* sum alpha_I dlambda over plasma samples            */
    BL_AUX_IJ = 4,       /* nu^3 sum j_I dlambda (unabsorbed I_nu)             */
    BL_AUX_NACC = 5,     /* accepted DP steps                                  */
    BL_AUX_NREJ = 6,     /* rejected DP steps                                  */
    BL_AUX_STATUS = 7,   /* bl_ray_status                                      */
    BL_AUX_NSAMP = 8,    /* plasma samples used by the transfer                */
    BL_AUX_NREC = 9      /* transfer records of the ray (pieces + vacuum steps) */
};

typedef enum {
    BL_RAY_ESCAPED = 1,      /* r crossed the camera radius from below         */
    BL_RAY_CAPTURED = 2,     /* r fell below r_in                              */
    BL_RAY_MAXSTEPS = 3,     /* accepted + rejected trials reached max_steps   */
    BL_RAY_UNDERFLOW = 4,    /* |h| < 1e-14 (1 + |lambda|)                     */
    BL_RAY_NONFINITE = 5     /* a NaN or Inf appeared in the state or error    */
} bl_ray_status;

typedef struct bl_context bl_context;   /* one device + one HIP stream */
typedef struct bl_grid bl_grid;         /* device-resident fluid data  */

/* Plane-parallel camera, paper section 2.1. */
typedef struct {
    double r, theta, phi;     /* camera centre in spherical Kerr-Schild       */
    double u_normal[3];       /* u^p: normal-frame velocity (spherical KS)    */
    double k_cov[3];          /* k_i: received momentum, spherical KS, any norm */
    double width;             /* w: full width of the image plane (M)         */
    int32_t n;                /* N: pixels per side (1 .. 16384)              */
    int32_t freq_mode;        /* 0: nu at infinity (-n k_t = nu);
                                 1: nu at the camera (-n k.u = nu)            */
    int32_t kind;             /* 0: plane-parallel camera (the only kind built;
                                 others give BL_E_UNSUPPORTED)                */
    int32_t pad;
    double psi;               /* rotation of the camera about its axis        */
    double nu_hz;             /* observing frequency (Hz)                     */
} bl_camera;

typedef struct {
    double a;                 /* spin a/M, |a| < 1                            */
    double mass_msun;         /* M in solar masses: sets the CGS length GM/c^2 */
    double r_in;              /* inner termination radius (M)                 */
    int32_t flat;             /* 1: Minkowski metric on the same coordinates  */
    int32_t pad;
} bl_spacetime;

/* Dormand-Prince RK5(4)7M, paper section 2.2 and its Table of coefficients. */
typedef struct {
    double f_abs, f_rel;      /* error tolerances of the step norm            */
    double ds_max;            /* proper-length limit of a transfer piece (M);
                                 0 disables subdivision                       */
    double h0_frac;           /* first trial step = -h0_frac * r_pixel (0.1: the
                                 first error estimate then lies well above
                                 rounding noise)                              */
    int64_t max_steps;        /* cap on accepted + rejected trials per ray    */
    int32_t record_cap;       /* step records kept per ray in the fast path
                                 (0 = 512); longer rays take a slower path    */
    int32_t pad;
} bl_integrator;

/* Block-structured fluid data (paper section 2.5): n_blocks logically
   Cartesian blocks of bnx*bny*bnz cells; cell values are cell-centred. */
typedef struct {
    int32_t n_blocks, bnx, bny, bnz;  /* every bn* >= 2                       */
    const double *bounds;     /* host [n_blocks][6] = x0,x1,y0,y1,z0,z1; the
                                 blocks must tile the bounding box without
                                 overlap and be aligned to a common grid of
                                 the smallest block size                      */
    const void *prims;        /* device [n_blocks][bnz][bny][bnx][8]:
                                 rho, p, u~x, u~y, u~z, Bx, By, Bz in code
                                 units (u~ = CKS normal-frame velocity);
                                 16-byte aligned                              */
    int32_t dtype;            /* 0: float64, 1: float32 (mixed precision)     */
    int32_t pad;
    double rho_unit;          /* g cm^-3 per code density unit; p is in units
                                 of rho_unit c^2 and B of c sqrt(4 pi rho_unit) */
} bl_grid_desc;

/* Plasma model, paper section 2.6 (thermal electrons, R_high/R_low) and
   section 4.5 (nonthermal electrons): n_e is shared by thermal, power-law
   and kappa populations in the given fractions, whose coefficients add.  The
   nonthermal populations' coefficients are ultrarelativistic synchrotron
   ones: for the power law the closed forms of gamma_min^2 << X << gamma_max^2
   (X = nu/(nu_c sin theta), nu_c = e B/(2 pi m_e c)); for the kappa
   distribution its exact low- and high-frequency asymptotes joined by a
   bridge; their circular and rotative coefficients are zero.  Renders with a
   nonthermal population take the general constant-coefficient Stokes step
   (no Kirchhoff relation) and are single-image renders without data cuts or
   averages (else BL_E_UNSUPPORTED). */
typedef struct {
    double mu, ne_ni;         /* molecular weight, n_e/n_i                    */
    double r_high, r_low;     /* T_i/T_e prescription                         */
    double sigma_max;         /* sigma above this is vacuum                   */
    int32_t polarized;        /* 0: I only (eq. unpolarized); 1: I,Q,U,V      */
    int32_t interp;           /* 0: nearest cell; 1: trilinear within a block */
    double fractions[3];      /* of n_e: thermal, power law, kappa; >= 0,
                                 summing to 1 (all 0: thermal only)           */
    double pl_p;              /* power-law index p > 1                        */
    double pl_gamma_min, pl_gamma_max;  /* cutoffs, 1 <= min < max < inf      */
    double kappa, kappa_w;    /* kappa index (>= 2.5) and width w > 0         */
} bl_plasma;

typedef struct {
    int32_t precision;        /* 0: FP64 throughout; 1: FP64 geodesics with
                                 FP32 coefficients and transfer               */
    int32_t step_model;       /* 0: the plain step-size controller; k in
                                 1..64: learned step proposals from the
                                 network installed with bl_set_step_model,
                                 for the first step and after an accepted
                                 step whose trial count (accepted plus
                                 rejected) is a multiple of k (the plain
                                 controller proposes after the others)       */
} bl_mode;

/* ABI version of the loaded library (BLGPU_ABI_VERSION). */
int bl_abi_version(void);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
   (a hipStream_t; NULL = the null stream).  *out receives the handle. */
bl_status bl_create(int device, void *hip_stream, bl_context **out);
void bl_destroy(bl_context *ctx);
/* Message of the last non-OK status on this context ("" if none). */
const char *bl_last_error(const bl_context *ctx);

/* Describe device-resident cell data for sampling; copies the block table
   (host) and builds the block lookup table on the device: 64 bytes per cell
   of the lattice of the smallest block size (at most 2^24 cells, so at most
   1 GiB), each holding what locating a point in its block needs.  The
   primitive array is borrowed, not copied.  BL_E_UNSUPPORTED for blocks not
   on that lattice or a larger lattice, BL_E_INVALID_ARG for overlapping
   blocks, BL_E_OOM if the table does not fit. */
bl_status bl_grid_create(bl_context *ctx, const bl_grid_desc *desc, bl_grid **out);
void bl_grid_destroy(bl_grid *grid);

/* Initial pixel states (paper section 2.1): state_out device [N*N][8] =
   x^alpha (t,x,y,z), k_alpha (t,x,y,z) with pixel index i + N j;
   norm_out device [N*N] = n, the frequency normalisation. */
bl_status bl_camera_rays(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                         double *state_out, double *norm_out);

/* Geodesics only (paper section 2.2): state_out device [N*N][8] final
   states; aux_out device [BL_NAUX][N*N] with the geodesic maps (dt, s,
   lambda, n_acc, n_rej, status) filled and the transfer maps zero. */
bl_status bl_trace_geodesics(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, double *state_out, double *aux_out);

/* Full image (paper sections 2.1-2.6): image_out device [4][N][N] doubles
   (I, Q, U, V; Q, U, V zero when unpolarized); aux_out device
   [BL_NAUX][N][N].  Q > 0 means polarization along the vertical V, U > 0
   along the direction 45 degrees from V towards -H. */
bl_status bl_render(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                    const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                    const bl_mode *mode, double *image_out, double *aux_out);

/* bl_render for callers that cannot allocate device memory (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): the same
   render with every workspace buffer carved from a static device array of
   256 MiB that each GPU the library runs on holds until the process ends.
   The call allocates nothing (no hipMalloc or hipFree, no host heap for the
   image descriptor) and records no timing events; the caller passes the
   inputs and the outputs as for bl_render.  Results equal bl_render's bit for
   bit with the same arguments.  The image is processed in chunks of rays
   that fit the array (about 1,900 rays with the default 512-record slots,
   more with a smaller integ->record_cap), so it is slower than bl_render.
   BL_E_INVALID_ARG for integ->max_steps above 4095 (the bound of the
   overflow path's buffer), BL_E_UNSUPPORTED if not even 64 rays fit, and
   BL_E_DEVICE if the array has no address on this device.  The array
   keeps the last call's contents; every call clears what it needs.  All
   calls on one GPU share the array: calls that overlap in time on one GPU
   (from several contexts or streams) race and must be serialised by the
   caller. */
bl_status bl_render_noalloc(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                            const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                            const bl_mode *mode, double *image_out, double *aux_out);

/* Schedule of a render (how the work is laid out on the GPU; results do not
   depend on it).  bl_render and bl_render_batch use the context's tuning
   (bl_set_tuning; defaults below) unless bl_render_batch is given one. */
typedef struct {
    int32_t tile_w, tile_h;   /* pixels that share a wave: a tile_w x tile_h
                                 tile with tile_w * tile_h = 64 (default
                                 8 x 8); 0, 0 = plain row-major order         */
    int32_t transfer_waves_per_cu; /* resident waves of the persistent transfer
                                 kernel per compute unit; 0 = as many as fit
                                 (default)                                    */
    int32_t refill_min;       /* a transfer wave takes new rays once this many
                                 of its lanes are idle (1..64; default 4)     */
    int64_t chunk_rays;       /* rays traced per geodesic/transfer launch pair
                                 (multiple of 64; 0 = as many as the step-
                                 record workspace holds, the default: 128 GiB
                                 or half the free device memory at
                                 bl_create, whichever is less)                */
    int32_t order;            /* 0: images in the given order; 1: largest
                                 first                                        */
    int32_t reserved;         /* must be 0                                    */
} bl_tuning;

bl_status bl_set_tuning(bl_context *ctx, const bl_tuning *tuning);
bl_status bl_get_tuning(const bl_context *ctx, bl_tuning *tuning_out);

/* One image of a batch: camera, spacetime (spin, mass and r_in may differ per
   image; `flat` too) and device outputs as for bl_render. */
typedef struct {
    bl_camera cam;
    bl_spacetime st;
    double *image_out;        /* device [4][N][N]                             */
    double *aux_out;          /* device [BL_NAUX][N][N]                       */
} bl_image_desc;

/* Many images of uneven size, frequency, inclination and spin over one grid
   (the batched form of the paper's section 2 pipeline): all rays of all
   images are dealt to the same geodesic and persistent transfer launches
   (in chunks of tuning.chunk_rays), so small images do not leave the GPU
   idle.  Each image's results equal those of bl_render for that image.
   images: host [n_images]; tuning: host or NULL (the context's).  Total ray
   count below 2^31. */
bl_status bl_render_batch(bl_context *ctx, int32_t n_images, const bl_image_desc *images,
                          const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                          const bl_mode *mode, const bl_tuning *tuning);

/* Averaged quantities (paper section 4.6, Auxiliary Images): a render of one
   image (as bl_render: image_out and aux_out) followed by a pass over the
   same step records that writes avg_out, device [BL_NAVG][N][N] doubles:
   for q = rho, n_e, p, Theta_e, B, sigma, beta^-1 (k = 0..6; units as for
   bl_cuts), map k = <q>_lambda = (1/lambda) int q dlambda over the plasma
   samples (lambda the aux map of that name), map 7 + k = <q>_Ij =
   int q j_I dlambda / int j_I dlambda (0 without emission), map 14 + k =
   <q>_tau, the solution of d<q>/dtau = q - <q> from 0 at the source end,
   advanced over a sample of depth dtau as <q> += (q - <q>)(1 - e^-dtau).
   Data cuts apply.  The image and aux equal those of bl_render. */
#define BL_NAVG 21
bl_status bl_render_averages(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                             const bl_mode *mode, double *image_out, double *aux_out, double *avg_out);

/* Adaptive ray tracing (paper section 4.4, Adaptive Ray Tracing).  A pixel is
   a square of the image plane sampled at its centre.  Level 0 is the camera's
   N x N image cut into blocks of B x B pixels; a block that refines is
   replaced at the next level by four blocks of B x B pixels of half the size,
   so a level-l block (bx, by) holds pixels bx B .. bx B + B - 1 (columns) and
   by B .. by B + B - 1 (rows) of an N 2^l image of the same camera width, and
   each of its pixels equals that pixel of bl_render at N 2^l.  A block of a
   level below max_level refines if its centre lies in a region (closed
   rectangle x0 <= x <= x1, y0 <= y <= y1 in image-plane coordinates, units of
   M, the axes of the pixel columns and rows, origin at the image centre)
   whose minimum level exceeds the block's level, or if, for an enabled
   criterion c, at least frac B^2 of its pixels have a value above thr[c].
   The criteria act on Stokes I (image units) of the block's own pixels:
   c = 0: I; 1: (Di^2 + Dj^2)^1/2 with Di = (I[i+1] - I[i-1]) / 2;
   2: the same with Di = 2 (I[i+1] - I[i-1]) / (I[i-1] + 2 I[i] + I[i+1]);
   3: |Di + Dj| with Di = I[i-1] - 2 I[i] + I[i+1]; 4: the same divided by
   (I[i-1] + 2 I[i] + I[i+1]) / 4 (Dj alike along the column).  At block
   edges the gradient takes the one-sided two-point difference (relative:
   over the pair's mean) and the Laplacian the second difference of the
   nearest interior pixel; along a direction of one pixel (two for the
   Laplacian) the difference is 0; a relative difference whose weighted sum
   is 0 is 0. */
#define BL_ADAPT_MAX_REGIONS 8
typedef struct {
    int32_t block_n;          /* B: pixels per block side; divides cam->n     */
    int32_t max_level;        /* highest level (0: root only); n 2^max_level
                                 <= 2^20                                      */
    int32_t use[5];           /* criteria on (1) or off (0), order as above   */
    int32_t n_regions;        /* 0 .. BL_ADAPT_MAX_REGIONS                    */
    double thr[5];            /* thresholds of the criteria (not NaN if used) */
    double frac;              /* critical fraction of a block's pixels, (0, 1] */
    double region[BL_ADAPT_MAX_REGIONS][5]; /* x0, x1, y0, y1, minimum level   */
} bl_adaptive;

/* The adaptive render.  Outputs for up to max_blocks blocks over all levels,
   in level order; the blocks of level 0 row by row, those of level l + 1 in
   the order of their parents, each parent's four children as (2bx, 2by),
   (2bx+1, 2by), (2bx, 2by+1), (2bx+1, 2by+1).  blocks_out: device
   [max_blocks][3] int32 (level, bx, by); image_out: device
   [max_blocks][4][B][B] doubles (as bl_render's image, per block);
   aux_out: device [max_blocks][BL_NAUX][B][B] doubles; level_counts_out:
   host [max_level + 1], blocks per level (0 past the last level reached).
   Returns when the outputs are complete.  BL_E_UNSUPPORTED if a level's
   blocks would pass max_blocks (the levels before it are complete),
   BL_E_INVALID_ARG for a bad parameter. */
bl_status bl_render_adaptive(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                             const bl_mode *mode, const bl_adaptive *adaptive, int32_t max_blocks,
                             int32_t *blocks_out, double *image_out, double *aux_out, int32_t *level_counts_out);

/* Data cuts (paper section 4.1, Data Cuts): a sample whose rho, n_e, p,
   Theta_e, B, sigma, beta^-1 or Kerr-Schild r lies below its lower limit
   ([0]) or above its upper limit ([1]) is vacuum, and with plane = +1 (-1)
   so is every sample with (x - x0).n < 0 (> 0), x the CKS position (x, y, z).
   -inf / +inf leave a quantity uncut.  Units: rho and p as in the grid
   (code units), n_e in cm^-3, B in gauss, r in GM/c^2; sigma = b^2/rho and
   beta^-1 = b^2/(2 p).  These act besides bl_plasma.sigma_max.  The limits
   are compared in the arithmetic's own precision (FP32 in the mixed form), the
   plane test in FP64. */
typedef struct {
    double rho[2], ne[2], p[2], theta_e[2], b[2], sigma[2], beta_inv[2], r[2];
    int32_t plane;            /* 0: no plane cut; +1 or -1 as above           */
    int32_t pad;
    double plane_origin[3], plane_normal[3];
} bl_cuts;

/* Install data cuts for the context's following renders (all render entry
   points and bl_eval_samples); NULL removes them.  The struct is copied.
   BL_E_INVALID_ARG for NaN limits, a plane flag other than -1, 0, 1, or a
   non-finite plane origin or normal. */
bl_status bl_set_cuts(bl_context *ctx, const bl_cuts *cuts);

/* One camera at several frequencies (paper section 4.8, True-Color Images:
   images at many frequencies for a fixed camera and fixed data; section 5:
   tracing several images at once amortises the geodesic integration).  The
   geodesics do not depend on the frequency (n = nu / den with den = -k_t or
   -k.u), so each chunk of rays is traced once and the transfer runs once per
   frequency on the same step records.  cam->nu_hz is ignored; nu_hz: host
   [n_freq] frequencies (Hz, positive, finite), 1 <= n_freq <= 4096;
   images_out, aux_out: host arrays of n_freq device pointers, each an
   output as for bl_render.  Image f equals bl_render with
   cam->nu_hz = nu_hz[f], aux maps included.  Uses the context's tuning. */
bl_status bl_render_multifreq(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                              const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                              const bl_mode *mode, int32_t n_freq, const double *nu_hz,
                              double *const *images_out, double *const *aux_out);

/* One camera and one set of geodesics, several plasma models (paper
   section 5: an imaging study varies the frequency and the electron model of
   a snapshot for a fixed camera; section 4.8: images at several frequencies
   for fixed camera and data).  Neither the frequency nor the plasma enters
   the geodesic equation, so each chunk of rays is traced once and the
   transfer runs once per output on the same step records, each with its own
   frequency and its own bl_plasma: electron temperature prescription
   (R_high, R_low), sigma_max, mu, ne/ni, polarized or not, interpolation and
   electron populations may all differ between outputs.  nu_hz: host
   [n_out] frequencies (Hz, positive, finite) or NULL for cam->nu_hz in every
   output; plasmas: host [n_out] structs, read during the call;
   1 <= n_out <= 4096; images_out, aux_out: host arrays of n_out device
   pointers, each an output as for bl_render.  Output f equals bl_render
   with cam->nu_hz = nu_hz[f] and plasmas[f], aux maps included.  The
   restrictions of bl_render apply per output (nonthermal populations
   without data cuts: BL_E_UNSUPPORTED).  Uses the context's tuning. */
bl_status bl_render_models(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                           const bl_integrator *integ, const bl_grid *grid, int32_t n_out,
                           const double *nu_hz, const bl_plasma *plasmas, const bl_mode *mode,
                           double *const *images_out, double *const *aux_out);

/* Autotuner: times bl_render_batch of the given images (which it renders,
   into their outputs, several times) under a coordinate search over tile
   shape, transfer waves per CU, refill threshold, chunk size and image
   order, starting from the context's tuning, with at most max_trials timed
   renders.  Writes the fastest tuning and its time (ms per batch, from HIP
   events on the context's stream) to host best_out / best_ms_out (either
   may be NULL) and installs it as the context's tuning.  Synchronises the
   stream. */
bl_status bl_autotune(bl_context *ctx, int32_t n_images, const bl_image_desc *images,
                      const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                      const bl_mode *mode, int32_t max_trials, bl_tuning *best_out, double *best_ms_out);

/* Learned step proposals.  A multilayer perceptron 11 -> 64 -> 64 -> 64 -> 1
   (SiLU) maps the state at the start of a step -- x^mu, k_mu, spin, log|h|
   and log eps (eps floored at 1e-10) of the last accepted step -- to log|h| of
   the step to try; the embedded RK5(4) error estimate of section 2.2 still
   accepts or rejects every trial, and after a rejection the plain
   controller shrinks the step.  BF16 weights and activations on the matrix
   cores with FP32 accumulation; FP32 master weights trained with Adam.
   Model vector (FP32, BL_MLP_NMODEL floats): W1[64][11], b1[64], W2[64][64],
   b2[64], W3[64][64], b3[64], w4[64], b4, feature mean[11], feature
   standard deviation[11] (features are normalised as (x - mean) / std). */
#define BL_MLP_NIN 11
#define BL_MLP_NHID 64
#define BL_MLP_NPARAM 9153
#define BL_MLP_NMODEL 9175
#define BL_STEPLOG_REC 12     /* floats per step-log record: 11 features, target */

/* Step log of the plain integrator (section 2.2 controller): traces the rays
   of the given images (geodesics only; their aux_out maps receive the
   geodesic auxiliary maps, image_out is not used) and appends one record per
   accepted step to records_out (device [capacity][12]): the features of the
   step's start state (previous accepted step's log|h| and log eps; h0 and
   eps = 1 before the first) and the accepted log|h|.  *n_out (host) receives
   the number of accepted steps (records beyond capacity are dropped; their
   order is not deterministic).  Synchronises the stream. */
bl_status bl_steplog(bl_context *ctx, int32_t n_images, const bl_image_desc *images, const bl_integrator *integ,
                     float *records_out, int64_t capacity, int64_t *n_out);

/* Initial model (device [BL_MLP_NMODEL]) for records device [n][12]: feature
   mean and standard deviation of the records, LeCun-uniform weights from a
   counter-based generator seeded by `seed`, zero biases, output bias at the
   mean target. */
bl_status bl_mlp_init(bl_context *ctx, const float *records, int64_t n, int64_t seed, float *model_out);

typedef struct {
    int32_t epochs;           /* passes over the training rows               */
    int32_t batch;            /* rows per Adam step (multiple of 64)         */
    float lr, beta1, beta2, eps;   /* Adam                                   */
    int64_t seed;             /* order of the rows (a fresh affine
                                 permutation per epoch)                      */
    int64_t n_val;            /* records held out: the last n_val of a fixed
                                 pseudo-random order of the rows (seeded)     */
} bl_mlp_hparams;

/* Train model_inout (device [BL_MLP_NMODEL], FP32 master weights; the feature
   statistics are kept) on records device [n][12] by Adam on the mean squared
   error of log|h|.  loss_out device [epochs][2]: mean training loss of the
   epoch and the held-out loss after it. */
bl_status bl_mlp_train(bl_context *ctx, const float *records, int64_t n, const bl_mlp_hparams *hp,
                       float *model_inout, float *loss_out);

/* One forward and backward pass (exposed for gradient checks): for model
   device [BL_MLP_NMODEL] and records device [n][12] writes the outputs
   y_out device [n] (may be NULL), the mean squared error loss_out device [1]
   and its gradient grad_out device [BL_MLP_NPARAM] with respect to the
   first BL_MLP_NPARAM model entries. */
bl_status bl_mlp_forward_backward(bl_context *ctx, const float *model, const float *records, int64_t n, float *y_out,
                                  float *loss_out, float *grad_out);

/* Install the network used by step_model = 1 (copied and packed; the caller
   may free the model afterwards). */
bl_status bl_set_step_model(bl_context *ctx, const float *model);

/* Per-sample evaluation for checking (paper sections 2.2, 2.5, 2.6): for
   states device [n][8] and norms device [n], writes out device [n][64]:
   [0..7]   geodesic right-hand side dy/dlambda,
   [8..23]  G^a_d = Gamma^a_cd k^c (row-major a, d),
   [24..31] jI, jQ, jV, aI, aQ, aV, rQ, rV (invariants j/nu^2, alpha*nu),
   [32..35] n_e, Theta_e, B (gauss), nu in the fluid frame,
   [36..51] tetrad e0..e3 (contravariant),
   [52]     1 for emitting plasma, 0 for vacuum, [53] sigma, [54..63] 0. */
#define BL_NSAMPLE_OUT 64
bl_status bl_eval_samples(bl_context *ctx, const bl_spacetime *st, const bl_grid *grid,
                          const bl_plasma *plasma, int64_t n, const double *states,
                          const double *norms, double *out);

/* The fluid-frame synchrotron coefficients alone, for checking (paper
   section 2.6): for rows in device [n][5] = n_e (cm^-3), Theta_e, B (gauss),
   nu (Hz), cos theta_B, writes out device [n][8] = jI, jQ, jV, aI, aQ, aV, rQ,
   rV (CGS) of the electrons of plasma (its populations and polarized flag;
   the other fields unused), in FP64 (precision 0) or FP32 (precision 1:
   inputs rounded to FP32, results widened).  Asynchronous on the context's
   stream.  BL_E_INVALID_ARG for NULL pointers, n < 0, another precision or
   invalid populations. */
bl_status bl_eval_coeffs(bl_context *ctx, int32_t precision, const bl_plasma *plasma, int64_t n,
                         const double *in, double *out);

/* The polarized plasma substep alone, for checking (paper section 2.4, the
   constant-coefficient solution of the polarized transfer equation over one
   segment): for coefficient sets coeffs device [n][8] = jI, jQ, jV, aI, aQ,
   aV, rQ, rV (jU = aU = rU = 0: the frame's U axis is perpendicular to the
   field; the segment length folded in, so the segment has unit length) and
   Stokes vectors s0 device [n][4], writes S1 to s_out device [n][4].
   precision 0: FP64, 1: FP32 (inputs rounded to FP32, results widened).
   general 0: the thermal closed form of the image kernels, which assumes
   Kirchhoff's law J = (jI/aI) M e_I and reads only jI of the emissivities;
   general 1: the substep of the nonthermal kernels (any source vector).
   aI >= 100 gives M^-1 J.  Asynchronous on the context's stream.
   BL_E_INVALID_ARG for NULL pointers, n < 0 or flags other than 0 and 1. */
bl_status bl_eval_stokes(bl_context *ctx, int32_t precision, int32_t general, int64_t n,
                         const double *coeffs, const double *s0, double *s_out);

/* Kernel timing with HIP events recorded around every launch on the context's
   stream (tracing aid; off by default).  Kernel classes: */
#define BL_NKERNEL 4
enum { BL_K_SETUP = 0, BL_K_GEODESIC = 1, BL_K_TRANSFER = 2, BL_K_OVERFLOW = 3 };
bl_status bl_profile_enable(bl_context *ctx, int enable);
/* Synchronises the stream, then writes the summed durations (ms) and launch
   counts per kernel class since the last read into host arrays
   ms_out[BL_NKERNEL] and launches_out[BL_NKERNEL], and clears them. */
bl_status bl_profile_read(bl_context *ctx, double *ms_out, int64_t *launches_out);

#ifdef __cplusplus
}
#endif

#endif /* BLGPU_H */
