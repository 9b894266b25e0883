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

// per-ray status codes (blgpu.h bl_ray_status); kRayOverflow is internal:
// the ray needs more step records than the fast path keeps.
enum : int { kRunning = 0, kEscaped = 1, kCaptured = 2, kMaxSteps = 3, kUnderflow = 4,
             kNonfinite = 5, kRayOverflow = 99 };

constexpr int kNaux = 9;
constexpr int kRecDoubles = 16;   // one step record = 128 bytes

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
    int pad;
};

// Device view of the block-structured grid.
struct DevGrid {
    const void *prims;        // [nb][bnz][bny][bnx][8], float64 or float32
    const double *bmeta;      // [nb][6] = x0, y0, z0, dx, dy, dz (cell sizes)
    const int *table;         // [tnz][tny][tnx] leaf block per table cell, -1 = none
    double bb[6];             // bounding box x0,x1,y0,y1,z0,z1
    double t0[3], tb[3];      // table origin and cell size
    int tn[3];
    int nb, bnx, bny, bnz, dtype;
    double rho_unit;
};

struct PlasmaParams {
    double mu, ne_ni, r_high, r_low, sigma_max;
    double mass_msun;
    int polarized, interp;
};

}  // namespace bl
