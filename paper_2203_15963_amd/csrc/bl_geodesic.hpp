// bl_geodesic.hpp -- adaptive Dormand-Prince RK5(4)7M integration of one
// ray per lane (paper section 2.2 and its coefficient table).
//
// The error of a trial step is eps = max_m |y5_m - y4_m| / (f_abs + f_rel
// max(|y_init_m|, |y5_m|)) over the eight variables (x^mu, k_mu); eps > 1
// rejects.  y5 - y4 is formed as h sum_i (b5_i - b4_i) k_i (no cancellation
// of two nearly equal states).  The Shampine midpoint of the step,
// y_mid = y0 + (h/2) sum_i bm_i k_i (the printed midpoint row sums to one), is
// stored with the step for the transfer.  Controller: after an accepted step
// h *= min(10, max(0.2, 0.9 eps^-1/5)) (10 for eps = 0), not growing right
// after a rejection; after a rejection h *= max(0.2, 0.9 eps^-1/5).  Every
// factor is rounded to a multiple of 1/4096 and the first step h0 =
// -h0_frac r_pix uses r_pix rounded to a multiple of 2^-10: the last bits of
// the error estimate (a sum with heavy cancellation) are rounding noise, and
// the rounding keeps them out of the step sequence.
// Integration runs at negative lambda from the camera and stops on an
// accepted step with r_prev < r_cam <= r_new or r_new < r_in.
#pragma once

#include "bl_kerr.hpp"
#include "bl_mlp.hpp"

namespace bl {

// Tableau (paper, Table "tab:dp").
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                 A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0, A64 = 49.0 / 176.0,
                 A65 = -5103.0 / 18656.0;
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0, B5 = -2187.0 / 6784.0,
                 B6 = 11.0 / 84.0;
constexpr double E1 = B1 - 5179.0 / 57600.0, E3 = B3 - 7571.0 / 16695.0, E4 = B4 - 393.0 / 640.0,
                 E5 = B5 - (-92097.0 / 339200.0), E6 = B6 - 187.0 / 2100.0, E7 = 0.0 - 1.0 / 40.0;
constexpr double M1 = 6025192743.0 / 30085553152.0, M3 = 51252292925.0 / 65400821598.0,
                 M4 = -2691868925.0 / 45128329728.0, M5 = 187940372067.0 / 1594534317056.0,
                 M6 = -1776094331.0 / 19743644256.0, M7 = 11237099.0 / 235043384.0;

struct TraceOut {
    int status;
    int n_acc, n_rej;
    int work;   // transfer iterations: pieces of the steps from the last sampled one to the camera
    double lambda, s, dt;
};

// One Dormand-Prince trial step of size h from y (with k1 = f(y)): the
// fifth-order state y5, k7 = f(y5) (the next k1 when accepted), the Shampine
// midpoint ym, the error norm eps and whether anything was not finite.
__device__ __forceinline__ void dp_trial(const GeoParams &P, const double y[7], double kt, const double k1[7],
                                         double h, double y5[7], double k7[7], double ym[7], double &eps,
                                         bool &bad) {
    const double a = P.a;
    const int flat = P.flat;
    double k2[7], k3[7], k4[7], k5[7], k6[7], ys[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) ys[m] = y[m] + h * (A21 * k1[m]);
    geo_rhs(a, flat, ys, kt, k2);
#pragma unroll
    for (int m = 0; m < 7; ++m) ys[m] = y[m] + h * (A31 * k1[m] + A32 * k2[m]);
    geo_rhs(a, flat, ys, kt, k3);
#pragma unroll
    for (int m = 0; m < 7; ++m) ys[m] = y[m] + h * (A41 * k1[m] + A42 * k2[m] + A43 * k3[m]);
    geo_rhs(a, flat, ys, kt, k4);
#pragma unroll
    for (int m = 0; m < 7; ++m) ys[m] = y[m] + h * (A51 * k1[m] + A52 * k2[m] + A53 * k3[m] + A54 * k4[m]);
    geo_rhs(a, flat, ys, kt, k5);
#pragma unroll
    for (int m = 0; m < 7; ++m)
        ys[m] = y[m] + h * (A61 * k1[m] + A62 * k2[m] + A63 * k3[m] + A64 * k4[m] + A65 * k5[m]);
    geo_rhs(a, flat, ys, kt, k6);
#pragma unroll
    for (int m = 0; m < 7; ++m) y5[m] = y[m] + h * (B1 * k1[m] + B3 * k3[m] + B4 * k4[m] + B5 * k5[m] + B6 * k6[m]);
    geo_rhs(a, flat, y5, kt, k7);
    // error norm over (t, x, y, z, k_t, k_x, k_y, k_z); the k_t error is 0
    eps = 0.0;
    bad = false;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double err, y0m, y5m;
        if (m < 4) {
            err = h * (E1 * k1[m] + E3 * k3[m] + E4 * k4[m] + E5 * k5[m] + E6 * k6[m] + E7 * k7[m]);
            y0m = y[m];
            y5m = y5[m];
        } else if (m == 4) {
            err = 0.0;
            y0m = kt;
            y5m = kt;
        } else {
            int q = m - 1;
            err = h * (E1 * k1[q] + E3 * k3[q] + E4 * k4[q] + E5 * k5[q] + E6 * k6[q] + E7 * k7[q]);
            y0m = y[q];
            y5m = y5[q];
        }
        double sc = P.f_abs + P.f_rel * fmax(fabs(y0m), fabs(y5m));
        // (a zero scale, with both tolerances zero, divides: |err|/0 = inf)
        double e = (err == 0.0) ? 0.0 : (sc > 0.0 ? fabs(err) * rcp_nr(sc) : fabs(err) / sc);
        if (isnan(e)) bad = true;
        else if (e > eps) eps = e;
    }
    bool fin = true;
#pragma unroll
    for (int m = 0; m < 7; ++m) fin = fin && isfinite(y5[m]);
    bad = bad || !fin;
#pragma unroll
    for (int m = 0; m < 7; ++m)
        ym[m] = y[m] + 0.5 * h * (M1 * k1[m] + M3 * k3[m] + M4 * k4[m] + M5 * k5[m] + M6 * k6[m] + M7 * k7[m]);
}

// eps^(-1/5) for eps > 0: an FP32 estimate from the hardware exp and log
// refined by two Newton steps on y^-5 - eps = 0, y <- y (6 - eps y^5)/5
// (relative error 1e-6, then about 3e-12, then below the FP64 rounding).
// Outside [1e-30, 1e30] the controller's clamps decide the factor, so a
// bound stands in for the root there.
__device__ __forceinline__ double inv_fifth_root(double eps) {
    if (!(eps > 1e-30)) return 1e6;
    if (!(eps < 1e30)) return 0.0;
    double y = (double)__expf(-0.2f * __logf((float)eps));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y2 = y * y;
        y = y * (6.0 - eps * (y2 * y2 * y)) * 0.2;
    }
    return y;
}

// Controller factor after an accepted step (rounded to a multiple of 1/4096).
__device__ __forceinline__ double grow_factor(double eps) {
    double fac = (eps == 0.0) ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * inv_fifth_root(eps)));
    return rint(fac * 4096.0) / 4096.0;
}
__device__ __forceinline__ double shrink_factor(double eps) {
    return rint(fmax(0.2, 0.9 * inv_fifth_root(eps)) * 4096.0) / 4096.0;
}

// Does the chord from p to q (spatial components 1..3 of states (t, x, y, z,
// ...)) meet the closed box?  A chord starting inside the box meets it; the
// slab test agrees exactly there (each slab's parameter interval then holds
// t = 0: its bounds are quotients of numbers of opposite or zero sign), so
// the shortcut changes no decision and saves the divisions for the steps
// inside the grid.
__device__ __forceinline__ bool chord_meets_box(const double bb[6], const double *p, const double *q) {
    if (p[1] >= bb[0] && p[1] <= bb[1] && p[2] >= bb[2] && p[2] <= bb[3] && p[3] >= bb[4] && p[3] <= bb[5])
        return true;
    double t0 = 0.0, t1 = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double a0 = p[1 + d], dd = q[1 + d] - p[1 + d];
        if (dd == 0.0) {
            if (a0 < bb[2 * d] || a0 > bb[2 * d + 1]) return false;
        } else {
            double ta = (bb[2 * d] - a0) / dd, tb = (bb[2 * d + 1] - a0) / dd;
            double lo = fmin(ta, tb), hi = fmax(ta, tb);
            t0 = fmax(t0, lo);
            t1 = fmin(t1, hi);
            if (t0 > t1) return false;
        }
    }
    return true;
}

// Store an accepted step's record, with the transfer's per-step decisions
// taken here, where the step's end state y1 and the right-hand sides f0 (at
// y0) and f1 (at y1) are at hand (paper section 2.2, last paragraph): the
// step is sampled against the grid when its chords y0-ym or ym-y1 meet the
// grid's bounding box, and is then cut into n = ceil(ds/ds_max) pieces (at
// most 2^24; one for a non-finite length or without a cut).  Slot 23 holds n
// for a sampled step and -1 for a vacuum step.  In the FP32-quartic layout
// (the mixed form) a step of n > 1 pieces stores, in place of ym, ds and f0,
// the coefficients c1..c4 of its dense output
//   y(theta) = y0 + theta (c1 + theta (c2 + theta (c3 + theta c4))),
// the quartic through y0, y1, f0, f1 and ym, formed in FP64 and rounded to
// FP32 (28 floats, c_j of component m at float 7 (j - 1) + m of slots 8..21).
__device__ __forceinline__ int write_record(const GeoParams &P, double *rec, int nacc, const double y0[7], double h,
                                             const double ym[7], const double y1[7], const double f0[7],
                                             const double f1[7], double ds) {
    double *r = rec + (long long)nacc * kRecDoubles;
#pragma unroll
    for (int m = 0; m < 7; ++m) r[m] = y0[m];
    r[7] = h;
    const bool inb = chord_meets_box(P.bb, y0, ym) || chord_meets_box(P.bb, ym, y1);
    int nsub = 1;
    if (inb && P.ds_max > 0.0) {
        const double q = ceil(ds / P.ds_max);
        nsub = (q >= 1.0) ? (int)fmin(q, 16777216.0) : 1;
    }
    r[23] = inb ? (double)nsub : -1.0;
    if (P.rec_quart32 && nsub > 1) {
        float *c = reinterpret_cast<float *>(r + 8);
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const double A = y1[m] - y0[m] - h * f0[m];
            const double B = h * (f1[m] - f0[m]);
            const double C = 16.0 * (ym[m] - y0[m]) - 8.0 * h * f0[m];
            c[m] = (float)(h * f0[m]);
            c[7 + m] = (float)(-5.0 * A + B + C);
            c[14 + m] = (float)(14.0 * A - 3.0 * B - 2.0 * C);
            c[21 + m] = (float)(-8.0 * A + 2.0 * B + C);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 7; ++m) r[8 + m] = ym[m];
        r[15] = ds;
#pragma unroll
        for (int m = 0; m < 7; ++m) r[16 + m] = f0[m];
    }
    return inb ? nsub : 0;
}

// The final state and its right-hand side after the last step, and in slot
// 23 the index of the last step sampled against the grid (-1 if none): the
// transfer starts there, the vacuum steps beyond it (towards the source)
// leaving nothing to do before the first emitting sample.
__device__ __forceinline__ void write_final(double *rec, int nacc, const double y[7], const double f[7],
                                            int last_sampled) {
    double *r = rec + (long long)nacc * kRecDoubles;
#pragma unroll
    for (int m = 0; m < 7; ++m) r[m] = y[m];
#pragma unroll
    for (int m = 0; m < 7; ++m) r[16 + m] = f[m];
    r[23] = (double)last_sampled;
}

// A ray that has filled its record slot moves to an extension slot (when one
// is free): its records so far are copied there and the integration goes on
// with the extension's capacity.  Returns false when none is free.
__device__ __forceinline__ bool move_to_extension(const ExtQueue *X, int slot, int nacc, double *&rec, int &cap) {
    if (!X || X->cap_rec <= cap) return false;
    const int k = atomicAdd(X->count, 1);
    if (k >= X->cap_rays) return false;
    double *nr = X->rec + (long long)k * X->cap_rec * kRecDoubles;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 *src = reinterpret_cast<const d2 *>(rec);
    d2 *dst = reinterpret_cast<d2 *>(nr);
    const long long n2 = (long long)nacc * (kRecDoubles / 2);
    long long i = 0;
    for (; i + 8 <= n2; i += 8) {   // eight loads in flight
        d2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[i + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[i + u] = v[u];
    }
    for (; i < n2; ++i) dst[i] = src[i];
    X->of[slot] = k;
    rec = nr;
    cap = X->cap_rec;
    return true;
}

// Step log: one record per accepted step of the plain controller, the
// features of the step's start state (x^mu, k_mu, spin, log|h| and log eps of
// the previous accepted step; h0 and eps = 1 before the first) and the
// accepted log|h|.
struct StepLog {
    float *buf;
    long long cap;
    unsigned long long *count;
};

// Trace one ray from its pixel state y (x^mu, k_x, k_y, k_z; k_t = kt held
// fixed).  Step records (16 doubles each, see below) go to rec[0..cap); the
// final state goes to record n_acc.  A ray needing more than cap records
// stops with status kRayOverflow.  Without WREC nothing is stored; with LOG
// every accepted step is appended to the step log.
//   record: [0..3] x^mu of y0, [4..6] k_a of y0, [7] h,
//           [8..11] x^mu of y_mid, [12..14] k_a of y_mid, [15] ds of the step,
//           [16..22] dy/dlambda at y0 (the first stage of the step),
//           [23] pieces of a sampled step, -1 for a vacuum step
//           (slots 8..22 hold the FP32 quartic instead for a step of more
//           than one piece in the FP32-quartic layout; see write_record)
//   final record n_acc: [0..6] the final state, [16..22] dy/dlambda there,
//           [23] the last step sampled against the grid (-1: none)
template <bool WREC, bool LOG = false>
__device__ __forceinline__ void trace_ray(const GeoParams &P, double y[7], double kt, double *rec, int cap,
                                          TraceOut &o, StepLog lg = StepLog{nullptr, 0, nullptr},
                                          const ExtQueue *X = nullptr, int slot = -1) {
    const double a = P.a;
    const int flat = P.flat;
    double k1[7], y5[7], k7[7], ym[7];
    double t_pix = y[0];
    geo_rhs(a, flat, y, kt, k1);
    double r_prev = ks_r(a, y[1], y[2], y[3]);
    double h = -P.h0_frac * (rint(r_prev * 1024.0) / 1024.0);
    double h_last = h, eps_last = 1.0;
    double lambda = 0.0, s = 0.0;
    int nacc = 0, nrej = 0, status = kRunning, last_sampled = -1, pieces = 0, work = 0;
    bool no_grow = false;
    while (status == kRunning) {
        if ((long long)nacc + nrej >= P.max_steps) { status = kMaxSteps; break; }
        if (fabs(h) < 1e-14 * (1.0 + fabs(lambda))) { status = kUnderflow; break; }
        double eps;
        bool bad;
        dp_trial(P, y, kt, k1, h, y5, k7, ym, eps, bad);
        if (bad) { status = kNonfinite; break; }
        if (eps <= 1.0) {
            if (WREC && nacc + 2 > cap && !move_to_extension(X, slot, nacc, rec, cap)) {
                status = kRayOverflow;
                break;
            }
            double ds = fabs(h) * ds_dlambda(a, flat, ym, kt);
            if (WREC) {
                const int np = write_record(P, rec, nacc, y, h, ym, y5, k1, k7, ds);
                pieces += np > 0 ? np : 1;
                if (np > 0) {
                    last_sampled = nacc;
                    work = pieces;
                }
            }
            if (LOG) {
                unsigned long long idx = atomicAdd(lg.count, 1ull);
                if ((long long)idx < lg.cap) {
                    float f[kMlpIn];
                    step_features(y, kt, a, h_last, eps_last, f);
                    float *q = lg.buf + idx * kLogRec;
#pragma unroll
                    for (int m = 0; m < kMlpIn; ++m) q[m] = f[m];
                    q[kMlpIn] = __logf(fabsf((float)h));   // the same map as the log|h| feature
                }
                h_last = h;
                eps_last = eps;
            }
            ++nacc;
            lambda += h;
            s += ds;
            double fac = grow_factor(eps);
            if (no_grow) fac = fmin(fac, 1.0);
            no_grow = false;
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                y[m] = y5[m];
                k1[m] = k7[m];
            }
            double r_new = ks_r(a, y[1], y[2], y[3]);
            if (r_new < P.r_in) status = kCaptured;
            else if (r_prev < P.r_cam && r_new >= P.r_cam) status = kEscaped;
            r_prev = r_new;
            h *= fac;
        } else {
            ++nrej;
            h *= shrink_factor(eps);
            no_grow = true;
        }
    }
    if (WREC && status != kRayOverflow) write_final(rec, nacc, y, k1, last_sampled);
    o.status = status;
    o.n_acc = nacc;
    o.n_rej = nrej;
    o.work = work + (nacc - 1 - last_sampled);
    o.lambda = fabs(lambda);
    o.s = s;
    o.dt = t_pix - y[0];
}

// The same integration with learned step proposals: for the first step and
// after an accepted step whose trial count is a multiple of P.net_every the
// wave evaluates the step-proposal network for its lanes and a lane tries
// h = -exp(net) (clamped to 0.2..10 times the last accepted |h|; the plain
// controller's proposal if the output is not finite); after the other
// accepted steps the plain controller proposes.  The embedded error estimate still accepts or rejects each trial;
// after a rejection the plain controller shrinks h for the retry.  The loop
// runs wave-converged (every lane reaches the network call each iteration);
// lanes with active = false only take part in it.
template <bool WREC>
__device__ __forceinline__ void trace_ray_learned(const GeoParams &P, bool active, double y[7], double kt, double *rec,
                                                  int cap, TraceOut &o, const u32x4 *pk, const float *tail,
                                                  u32x4 *stage, const ExtQueue *X = nullptr, int slot = -1) {
    const double a = P.a;
    const int flat = P.flat;
    double k1[7], y5[7], k7[7], ym[7];
    double t_pix = y[0];
    double r_prev = 0.0, h = -1.0;
    if (active) {
        geo_rhs(a, flat, y, kt, k1);
        r_prev = ks_r(a, y[1], y[2], y[3]);
        h = -P.h0_frac * (rint(r_prev * 1024.0) / 1024.0);
    }
    double h_last = h, eps_last = 1.0;
    double lambda = 0.0, s = 0.0;
    int nacc = 0, nrej = 0, status = active ? kRunning : kEscaped, last_sampled = -1, pieces = 0, work = 0;
    bool need = true, no_grow = false;
    for (;;) {
        const bool run = status == kRunning;
        if (__ballot(run && need)) {
            float f[kMlpIn];
            step_features(y, kt, a, h_last, eps_last, f);
            const float lh = mlp_forward(pk, tail, f, stage);
            if (run && need) {
                const double hp = exp((double)lh), hl = fabs(h_last);
                if (isfinite(hp) && hp > 0.0) h = -fmin(10.0 * hl, fmax(0.2 * hl, hp));
                else if (nacc > 0) h = h_last * grow_factor(eps_last);
                need = false;
            }
        }
        if (__ballot(run) == 0) break;
        if (!run) continue;
        if ((long long)nacc + nrej >= P.max_steps) { status = kMaxSteps; continue; }
        if (fabs(h) < 1e-14 * (1.0 + fabs(lambda))) { status = kUnderflow; continue; }
        double eps;
        bool bad;
        dp_trial(P, y, kt, k1, h, y5, k7, ym, eps, bad);
        if (bad) { status = kNonfinite; continue; }
        if (eps <= 1.0) {
            if (WREC && nacc + 2 > cap && !move_to_extension(X, slot, nacc, rec, cap)) {
                status = kRayOverflow;
                continue;
            }
            double ds = fabs(h) * ds_dlambda(a, flat, ym, kt);
            if (WREC) {
                const int np = write_record(P, rec, nacc, y, h, ym, y5, k1, k7, ds);
                pieces += np > 0 ? np : 1;
                if (np > 0) {
                    last_sampled = nacc;
                    work = pieces;
                }
            }
            ++nacc;
            lambda += h;
            s += ds;
            h_last = h;
            eps_last = eps;
            // every running lane of the wave has made the same number of
            // trials (one per loop pass), so this is a wave-wide choice and
            // the network runs in one pass of net_every
            need = (nacc + nrej) % P.net_every == 0;
            if (!need) {
                double fac = grow_factor(eps);
                if (no_grow) fac = fmin(fac, 1.0);
                h *= fac;
            }
            no_grow = false;
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                y[m] = y5[m];
                k1[m] = k7[m];
            }
            double r_new = ks_r(a, y[1], y[2], y[3]);
            if (r_new < P.r_in) status = kCaptured;
            else if (r_prev < P.r_cam && r_new >= P.r_cam) status = kEscaped;
            r_prev = r_new;
        } else {
            ++nrej;
            h *= shrink_factor(eps);
            no_grow = true;
        }
    }
    if (WREC && active && status != kRayOverflow) write_final(rec, nacc, y, k1, last_sampled);
    o.status = status;
    o.n_acc = nacc;
    o.n_rej = nrej;
    o.work = work + (nacc - 1 - last_sampled);
    o.lambda = fabs(lambda);
    o.s = s;
    o.dt = t_pix - y[0];
}

}  // namespace bl
