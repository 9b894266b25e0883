// bl_common.hpp -- constants and device-side parameter blocks shared by the
// gfx950 kernels of libblgpu.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bl {

// CGS constants (CODATA 2018; IAU nominal solar mass).
constexpr double kC = 2.99792458e10;
constexpr double kG = 6.67430e-8;
constexpr double kMsun = 1.98841e33;
constexpr double kMe = 9.1093837015e-28;
constexpr double kMp = 1.67262192369e-24;
constexpr double kQe = 4.80320471e-10;
constexpr double kH = 6.62607015e-27;
constexpr double kKb = 1.380649e-16;
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

// Exponential, logarithm and cube root for smooth fitting-formula terms: the
// hardware transcendental unit in FP32 (relative error a few 1e-7 times the
// argument's magnitude for exp, far inside the mixed form's tolerance); in
// FP64 the branch-free exponential and logarithm below (a few ulp), whose
// straight-line code lets independent evaluations interleave.
__device__ __forceinline__ float fexp(float x) { return __expf(x); }
// e^x in FP64: x = k ln2 + r with the reduction in two parts (Cody and Waite;
// ln2_hi has eleven trailing zero bits, so k ln2_hi is exact), e^r from its
// Taylor polynomial through r^13/13! on |r| <= ln2/2 (truncation below 1e-17;
// even and odd parts in r^2 evaluated side by side to halve the chain of
// dependent operations), then scaled by 2^k: within about one ulp.
__device__ __forceinline__ double fexp(double x) {
    x = x < -750.0 ? -750.0 : (x > 710.0 ? 710.0 : x);
    const double k = rint(x * 1.4426950408889634);
    double r = fma(-k, 0x1.62e42fefa3800p-1, x);
    r = fma(-k, 5.497923018708371e-14, r);
    const double u = r * r;
    double ev = 1.0 / 479001600.0, od = 1.0 / 6227020800.0;   // 1/12!, 1/13!
    ev = fma(ev, u, 1.0 / 3628800.0);
    od = fma(od, u, 1.0 / 39916800.0);
    ev = fma(ev, u, 1.0 / 40320.0);
    od = fma(od, u, 1.0 / 362880.0);
    ev = fma(ev, u, 1.0 / 720.0);
    od = fma(od, u, 1.0 / 5040.0);
    ev = fma(ev, u, 1.0 / 24.0);
    od = fma(od, u, 1.0 / 120.0);
    ev = fma(ev, u, 0.5);
    od = fma(od, u, 1.0 / 6.0);
    ev = fma(ev, u, 1.0);
    od = fma(od, u, 1.0);
    return ldexp(fma(r, od, ev), (int)k);
}
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ float fcbrt(float x) { return __expf(__logf(x) * (1.0f / 3.0f)); }   // x > 0
// e^x - 1 with relative accuracy near zero: in FP32 the Taylor polynomial
// through x^8/8! for |x| < 0.35 (truncation below 1e-9 relative), the hardware
// exponential minus one elsewhere.
__device__ __forceinline__ float fexpm1(float x) {
    float p = 1.0f / 40320.0f;
    p = p * x + 1.0f / 5040.0f;
    p = p * x + 1.0f / 720.0f;
    p = p * x + 1.0f / 120.0f;
    p = p * x + 1.0f / 24.0f;
    p = p * x + 1.0f / 6.0f;
    p = p * x + 0.5f;
    p = p * x + 1.0f;
    return fabsf(x) < 0.35f ? p * x : __expf(x) - 1.0f;
}
// In FP64: for |x| < 0.7 the Taylor polynomial x (1 + x/2! + ... + x^15/16!)
// (truncation below 1e-17 relative; even and odd parts side by side), else
// fexp(x) - 1 (within a few ulp there, |e^x - 1| >= 0.5 |e^x|).
constexpr double rfact(int n) {   // 1/n!
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return 1.0 / f;
}
__device__ __forceinline__ double fexpm1(double x) {
    const double u = x * x;
    double ev = rfact(15), od = rfact(16);   // c_j = 1/(j+1)!, j = 14, 15
#pragma unroll
    for (int j = 12; j >= 0; j -= 2) {
        ev = fma(ev, u, rfact(j + 1));
        od = fma(od, u, rfact(j + 2));
    }
    const double small = x * fma(x, od, ev);
    return fabs(x) < 0.7 ? small : fexp(x) - 1.0;
}
// 1/x in FP64: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y), which square the estimate's relative error each time:
// within about an ulp, though not always the correctly rounded quotient.  For
// normal finite x (x = 0 gives a NaN rather than an infinity).
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}
// 1/sqrt(x): the hardware unit in FP32; in FP64 its estimate refined by two
// Newton steps y <- y (3/2 - x y^2 / 2) (about an ulp), for normal x > 0
__device__ __forceinline__ float rsqrt_r(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_r(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = y * (1.5 - (0.5 * x) * (y * y));
    return y;
}
// a / b: the hardware reciprocal in FP32 (about 1 ulp), in FP64 a times the
// refined reciprocal (within about two ulp)
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a * rcp_nr(b); }
// 1/x and 1/sqrt(x) for quantities whose rounding error compounds along a ray:
// in FP32 the hardware estimates (whose errors of about an ulp lean to one
// side) refined by one Newton step, y <- y + y (1 - x y) and
// y <- y + y (1/2 - (x y / 2) y), each formed with fused multiply-adds; in
// FP64 the refined reciprocal and reciprocal square root above.
__device__ __forceinline__ float rcp_acc(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, y, 1.0f), y, y);
}
__device__ __forceinline__ double rcp_acc(double x) { return rcp_nr(x); }
__device__ __forceinline__ float rsqrt_acc(float x) {
    const float y = rsqrtf(x);
    return fmaf(fmaf(-(0.5f * x * y), y, 0.5f), y, y);
}
__device__ __forceinline__ double rsqrt_acc(double x) { return rsqrt_r(x); }
// ln x in FP64, branch free: x = m 2^e with m in [sqrt(1/2), sqrt(2)) from
// the hardware mantissa/exponent split, ln m = 2 atanh(s) with
// s = (m - 1)/(m + 1), |s| <= 0.1716, from its series 2 s (1 + s^2/3 + ... +
// s^20/21) (truncation below 1e-17 relative; even and odd parts in s^4 side by
// side), and e ln 2 added with ln 2 in two parts (the high part has eleven
// trailing zero bits): within a few ulp, also near x = 1.  x <= 0 gives -inf
// (x = 0) or NaN.
__device__ __forceinline__ double flog(double x) {
    int e = __builtin_amdgcn_frexp_exp(x);         // x = mant 2^e, mant in [1/2, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    const bool lo = m < 0x1.6a09e667f3bcdp-1;     // sqrt(1/2)
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double s = (m - 1.0) * rcp_nr(m + 1.0);
    const double z = s * s, z2 = z * z;
    double ev = 1.0 / 21.0, od = 1.0 / 19.0;       // coefficients 1/(2j+1) of z^j
    ev = fma(ev, z2, 1.0 / 17.0);
    od = fma(od, z2, 1.0 / 15.0);
    ev = fma(ev, z2, 1.0 / 13.0);
    od = fma(od, z2, 1.0 / 11.0);
    ev = fma(ev, z2, 1.0 / 9.0);
    od = fma(od, z2, 1.0 / 7.0);
    ev = fma(ev, z2, 1.0 / 5.0);
    od = fma(od, z2, 1.0 / 3.0);
    ev = fma(ev, z2, 1.0);
    const double lnm = 2.0 * s * fma(od, z, ev);
    const double de = (double)e;
    const double r = fma(de, 0x1.62e42fefa3800p-1, fma(de, 5.497923018708371e-14, lnm));
    return x > 0.0 ? (__builtin_isinf(x) ? x : r) : (x == 0.0 ? -__builtin_inf() : __builtin_nan(""));
}
// cos for arguments of moderate size: the hardware unit in FP32; in FP64
// from fsincos below
__device__ __forceinline__ float fcos(float x) { return __cosf(x); }
// sin and cos: in FP32 the argument is reduced by 2 pi in two parts (Cody and
// Waite; 6.28125 has eight significant bits, so n * 6.28125 is exact for the
// argument sizes met here) and the hardware unit evaluates on [-pi, pi]
__device__ __forceinline__ void fsincos(float x, float &s, float &c) {
    const float n = rintf(x * 0.15915494309189535f);
    float r = fmaf(-n, 6.28125f, x);
    r = fmaf(-n, 1.9353071795864769e-3f, r);
    s = __sinf(r);
    c = __cosf(r);
}
// In FP64, branch free: x = k pi/2 + r with the reduction in three parts
// (Cody and Waite; the first two parts of pi/2 carry 33 significant bits, so
// k times them is exact for |k| < 2^20, i.e. |x| below about 1.6e6, the
// range met here), sin r and cos r on |r| <= pi/4 from their Taylor
// polynomials through r^15/15! and r^16/16! (truncation below 1e-16
// relative), and the quadrant of k choosing signs and order: within a few ulp.
__device__ __forceinline__ void fsincos(double x, double &s, double &c) {
    const double k = rint(x * 0x1.45f306dc9c883p-1);   // 2/pi
    double r = fma(-k, 0x1.921fb54400000p+0, x);
    r = fma(-k, 0x1.0b4611a600000p-34, r);
    r = fma(-k, 0x1.3198a2e037073p-69, r);
    const double u = r * r;
    double ps = rfact(15), pc = fma(rfact(16), -u, rfact(14));
#pragma unroll
    for (int j = 13; j >= 1; j -= 2) {
        ps = fma(ps, -u, rfact(j));
        pc = fma(pc, -u, rfact(j - 1));
    }
    const double sr = r * ps;   // sin r = r (1 - r^2/3! + ...), cos r = 1 - r^2/2! + ...
    const double cr = pc;
    const int q = (int)(((long long)k) & 3);
    const double sq = (q & 1) ? cr : sr, cq = (q & 1) ? sr : cr;
    s = (q & 2) ? -sq : sq;
    c = ((q + 1) & 2) ? -cq : cq;
}
__device__ __forceinline__ double fcos(double x) {
    double s, c;
    fsincos(x, s, c);
    return c;
}
// ln(1 + x) for x >= 0 where only absolute accuracy is needed
__device__ __forceinline__ float flog1p_abs(float x) { return __logf(1.0f + x); }
__device__ __forceinline__ double flog1p_abs(double x) { return flog(1.0 + x); }

// per-ray status codes (blgpu.h bl_ray_status); kRayOverflow is internal:
// the ray needs more step records than the fast path keeps.
enum : int { kRunning = 0, kEscaped = 1, kCaptured = 2, kMaxSteps = 3, kUnderflow = 4,
             kNonfinite = 5, kRayOverflow = 99 };

constexpr int kNaux = 9;
constexpr int kRecDoubles = 24;   // one step record = 192 bytes

// Camera frame in CKS coordinate components (computed once per image on the
// device): centre, observer 4-velocity, line of sight K, horizontal H,
// vertical V, and the observer's CKS normal-frame 3-velocity.
struct Frame {
    double xc[4], u[4], K[4], H[4], V[4], ut[3];
    double pad;
};

struct CamParams {
    double r, theta, phi, u_normal[3], k_cov[3], width, psi, nu;
    int n, freq_mode;
    // the pixels rendered are pixels (i0 .. i0 + n - 1, j0 .. j0 + n - 1) of
    // an nf x nf image of the same width (nf = n, i0 = j0 = 0 for a whole
    // image; a block of an adaptive level otherwise)
    int nf, i0, j0, pad_c;
};

struct GeoParams {
    double a;          // spin
    double r_in;       // inner termination radius
    double r_cam;      // camera radius (outward crossing terminates)
    double f_abs, f_rel, h0_frac;
    long long max_steps;
    int flat;
    int cap;           // step records per ray slot
    int n;             // pixels per side
    int rec_quart32;   // records carry the FP32 quartic of sampled steps (the mixed form)
    int net_every;     // learned proposals: the network proposes after every net_every-th accepted step
    double bb[6];      // grid bounding box (x0, x1, y0, y1, z0, z1) for the sampling decision
    double ds_max;     // proper-length limit of a piece (0: no cut)
};

// Device view of the block-structured grid.
struct DevGrid {
    const void *prims;        // [nb][bnz][bny][bnx][8], float64 or float32
    // [tnz][tny][tnx][8] per cell of the block lattice, as doubles: the
    // covering leaf block's origin x0, y0, z0, inverse cell sizes 1/dx, 1/dy,
    // 1/dz and the index of its first cell (-1: no block), then a pad; 64
    // bytes, so that one lookup brings what locating a cell needs
    const double *table;
    double bb[6];             // bounding box x0,x1,y0,y1,z0,z1
    double t0[3], tb[3];      // table origin and cell size
    double itb[3];            // 1 / table cell size
    int tn[3];
    int nb, bnx, bny, bnz, dtype;
    double rho_unit;
};

struct PlasmaParams {
    double mu, ne_ni, r_high, r_low, sigma_max;
    double mass_msun;
    int polarized, interp;
    // per-render constants of the plasma state, formed on the host:
    double ne_per_rho;   // rho_unit / (mu m_p) / (1 + 1/(n_e/n_i))
    double th_per_pr;    // mu m_p / m_e
    double gauss_per_b;  // c sqrt(4 pi rho_unit)
    // data cuts (bl_cuts), read from device memory only when set, so that
    // they take no scalar registers in the kernels' loops
    int cuts;                      // 0: none set
    const struct CutParams *cut;   // device copy of the limits
    // nonthermal electron populations (read by the kernels compiled for them)
    int nonthermal;                // 0: thermal electrons only
    const struct NthParams *nth;   // device copy of their constants
};

// Electron populations (paper sections 2.6 and 4.5): fractions of n_e in the
// thermal, power-law and kappa distributions, and per nonthermal population
// (index 0: power law, 1: kappa) the constants of its synchrotron
// coefficients, formed on the host.  With X = nu/(nu_c sin theta) and
// nu_c = e B/(2 pi m c), in units of n_e e^2 nu_c/c (emissivities) and
// n_e e^2/(nu m c) (absorptivities):
//   power-law terms  jI = hj sin X^ej, jQ = hjq jI, aI = ha X^ea, aQ = haq aI
//   (the whole coefficient of the power law; the high-frequency asymptote of
//   the kappa distribution, whose tail is a power law);
//   kappa low-frequency asymptotes  jI = lj sin X^(1/3), aI = la X^(-2/3),
//   jQ, aQ half of them, joined to the high-frequency ones as
//   (low^-b + high^-b)^(-1/b) with b = 1/2 (jI, jQ, aQ) and 3/7 (aI).
// The constant factors are stored as natural logarithms (l* fields).
struct NthParams {
    double frac[3];
    double lhj[2], ej[2], lhjq[2], lha[2], ea[2], lhaq[2];
    double llj, lla;
};

// Data-cut limits in the order rho, n_e, p, Theta_e, B, sigma, beta^-1, r
// (FP64 and rounded to FP32 on the host), and the half-space plane.
struct CutParams {
    double lo[8], hi[8];
    float lo_f[8], hi_f[8];
    double x0[3], n[3];
    int plane;   // 0: none; +1: (x - x0).n < 0 is vacuum; -1: (x - x0).n > 0 is vacuum
    int pad;
};
constexpr int kCutRho = 0, kCutNe = 1, kCutP = 2, kCutThetaE = 3, kCutB = 4, kCutSigma = 5, kCutBetaInv = 6,
              kCutR = 7;

// One image of a render (a batch of one for bl_render): the camera frame
// (filled on the device), camera and spacetime parameters, where its results
// go, and the first global ray id it owns.
struct ImgDev {
    Frame fr;
    CamParams cp;
    double a, r_in;
    double L;            // GM/c^2 in cm
    double *image;       // [4][n][n]
    double *aux;         // [naux][n][n]
    double *avg;         // [21][n][n] averaged quantities (their own render pass), or null
    long long ray0;      // first global ray id
    long long nray;      // ray ids owned: n^2, or whole pixel tiles
    int flat, pad;
};

// The images of one render and how ray ids map to pixels.  Ray ids of an image
// are dealt out tile by tile: a tile of tw x th pixels (tw th = 64, so one
// wave traces one tile of neighbouring pixels), tiles in row-major order over
// the image, pixels row-major within the tile; ids of pixels past the image
// edge are skipped.  tw = 0 means plain row-major pixel order.
struct Batch {
    ImgDev *imgs;
    const long long *ray0;   // [n_img] copy of imgs[k].ray0 for the search
    int n_img, tw, th, pad;
};

// Rays that outgrow their record slot move to an extension slot of cap_rec
// records (up to cap_rays per chunk, taken in order by count): of[slot] is
// the extension of a slot (-1: none).
struct ExtQueue {
    int *count;
    int *of;
    double *rec;
    int cap_rays, cap_rec;
};

__device__ __forceinline__ int find_image(const Batch &B, long long gid) {
    int lo = 0, hi = B.n_img - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B.ray0[mid] <= gid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Pixel (i, j) of ray id rl (counted from the image's first id); false for
// the ids of tile pixels that lie outside the image.
__device__ __forceinline__ bool ray_pixel(const Batch &B, int n, long long rl, int &i, int &j) {
    if (B.tw <= 0) {
        i = (int)(rl % n);
        j = (int)(rl / n);
        return rl < (long long)n * n;
    }
    const int tsz = B.tw * B.th;
    const int ntx = (n + B.tw - 1) / B.tw;
    const long long tile = rl / tsz;
    const int o = (int)(rl - tile * tsz);
    i = (int)(tile % ntx) * B.tw + o % B.tw;
    j = (int)(tile / ntx) * B.th + o / B.tw;
    return i < n && j < n;
}

}  // namespace bl
