// bl_transfer.hpp -- source-to-camera radiative transfer along one traced ray
// (one ray per lane).
//
// Paper section 2.2 (last paragraph): each accepted geodesic step is
// represented by its fourth-order midpoint; a step longer than the proper
// length limit is cut into pieces using the quartic through y0, y1, f0, f1 and
// y_mid.  Section 2.3: unpolarized segments use the exact solution with
// Delta tau_max = 100.  Section 2.4: polarized transfer Strang-splits every
// segment into coordinate transport of the coherency tensor N (half, whole
// plasma step in the fluid tetrad, half), merging adjacent transport halves
// into one explicit-midpoint step (the paper's predictor-corrector table),
// with the exact constant-coefficient Stokes solution for the plasma part.
//
// Sampling rule: a step is sampled against the grid when its chords y0-y_mid
// or y_mid-y1 meet the grid's bounding box; it is then cut into
// n = ceil(ds/ds_max) pieces of equal lambda whose samples are the quartic at
// the piece centres (y_mid when n = 1).  Other steps are single vacuum
// records.  Polarized transfer starts at the first plasma record from the
// source; the merged transport between two records uses the previous sample
// as predictor point and the boundary between the records as corrector point;
// the last record is followed by a half-length transport to the pixel.
#pragma once

#include "bl_plasma.hpp"

namespace bl {

// ------------------------------------------------------ coherency tensor
// Hermitian N = R + i I with R symmetric (10 entries) and I antisymmetric (6).
__host__ __device__ constexpr int sidx_ord(int a, int b) {   // a <= b
    return a == 0 ? b : (a == 1 ? 3 + b : (a == 2 ? 5 + b : 9));
}
__host__ __device__ constexpr int sidx(int a, int b) { return a <= b ? sidx_ord(a, b) : sidx_ord(b, a); }
__host__ __device__ constexpr int aidx(int a, int b) {   // a < b
    return a == 0 ? b - 1 : (a == 1 ? 1 + b : 5);
}

struct Coh {
    double r[10], i[6];
};

__device__ __forceinline__ double Rget(const Coh &N, int a, int b) { return N.r[sidx(a, b)]; }
__device__ __forceinline__ double Iget(const Coh &N, int a, int b) {
    return a == b ? 0.0 : (a < b ? N.i[aidx(a, b)] : -N.i[aidx(b, a)]);
}

// dN^ab/dlambda = -(G^a_d N^db + G^b_d N^ad), the parallel transport of N.
__device__ __forceinline__ void transport_rhs(const double G[16], const Coh &N, Coh &dN) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < 4; ++d) s += G[4 * a + d] * Rget(N, d, b) + G[4 * b + d] * Rget(N, a, d);
            dN.r[sidx(a, b)] = -s;
        }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < 4; ++d) s += G[4 * a + d] * Iget(N, d, b) + G[4 * b + d] * Iget(N, a, d);
            dN.i[aidx(a, b)] = -s;
        }
}

// dN = F(N) with the connection applied one column of G at a time.
__device__ __forceinline__ void transport_apply(const ConnGeom &c, const Coh &N, Coh &dN) {
#pragma unroll
    for (int m = 0; m < 10; ++m) dN.r[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) dN.i[m] = 0.0;
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        double Gc[4];
        conn_col(c, dd, Gc);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b) dN.r[sidx(a, b)] -= Gc[a] * Rget(N, dd, b) + Gc[b] * Rget(N, a, dd);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a + 1; b < 4; ++b) dN.i[aidx(a, b)] -= Gc[a] * Iget(N, dd, b) + Gc[b] * Iget(N, a, dd);
    }
}

// One explicit-midpoint transport step of length dl: predictor with the
// connection at ya, corrector at yb (states x^mu, k_mu).
__device__ __forceinline__ void transport_step(double a, int flat, const double ya[8], const double yb[8],
                                               double dl, Coh &N) {
    if (flat) return;   // the connection vanishes
    ConnGeom c;
    Coh d, h;
    conn_geom(a, flat, ya, ya + 4, c);
    transport_apply(c, N, d);
#pragma unroll
    for (int m = 0; m < 10; ++m) h.r[m] = N.r[m] + 0.5 * dl * d.r[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) h.i[m] = N.i[m] + 0.5 * dl * d.i[m];
    conn_geom(a, flat, yb, yb + 4, c);
    transport_apply(c, h, d);
#pragma unroll
    for (int m = 0; m < 10; ++m) N.r[m] += dl * d.r[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) N.i[m] += dl * d.i[m];
}

// Stokes parameters of N in the screen vectors e1, e2 (contravariant) of a
// tetrad: I = N11 + N22, Q = N11 - N22, U = 2 Re N12, V = -2 Im N12.
__device__ __forceinline__ void coh_to_stokes(const KS &k, const double e1[4], const double e2[4], const Coh &N,
                                              double S[4]) {
    double p[4], q[4];
    lower(k, e1, p);
    lower(k, e2, q);
    double n11 = 0.0, n22 = 0.0, n12r = 0.0, n12i = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double R = Rget(N, a, b);
            n11 += p[a] * p[b] * R;
            n22 += q[a] * q[b] * R;
            n12r += p[a] * q[b] * R;
            n12i += p[a] * q[b] * Iget(N, a, b);
        }
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = 2.0 * n12r;
    S[3] = -2.0 * n12i;
}

// N = 1/2 [(I+Q) e1 e1 + (I-Q) e2 e2 + (U - iV) e1 e2 + (U + iV) e2 e1]
__device__ __forceinline__ void stokes_to_coh(const double e1[4], const double e2[4], const double S[4], Coh &N) {
    double n11 = 0.5 * (S[0] + S[1]), n22 = 0.5 * (S[0] - S[1]), n12r = 0.5 * S[2], n12i = -0.5 * S[3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b)
            N.r[sidx(a, b)] = n11 * e1[a] * e1[b] + n22 * e2[a] * e2[b] + n12r * (e1[a] * e2[b] + e2[a] * e1[b]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) N.i[aidx(a, b)] = n12i * (e1[a] * e2[b] - e2[a] * e1[b]);
}

// Exact solution of dS/ds = J - M S over length s for thermal coefficients
// (J = B_nu M e_I, so the fixed point is S_eq = (j_I/alpha_I) e_I):
//   S(s) = S_eq + e^{-alpha_I s} e^{-s K'} (S0 - S_eq),
// where K' is the traceless part of M with eigenvalues +-L1, +-i L2,
// L1^2, L2^2 = sqrt(((a^2 - r^2)/2)^2 + (a.r)^2) +- (a^2 - r^2)/2, and
// e^{-sK'} = [cosh(sL1) P1 + cos(sL2) P2] - K' [sinh(sL1)/L1 P1 + sin(sL2)/L2 P2]
// with projectors P1 = (K'^2 + L2^2)/(L1^2 + L2^2), P2 = (L1^2 - K'^2)/(L1^2 + L2^2).
// If alpha_I s >= 100 the result is S_eq.  c = jI, jQ, jV, aI, aQ, aV, rQ, rV.
__device__ __forceinline__ void kprime(const double c[8], const double v[4], double w[4]) {
    w[0] = c[4] * v[1] + c[5] * v[3];
    w[1] = c[4] * v[0] + c[7] * v[2];
    w[2] = -c[7] * v[1] + c[6] * v[3];
    w[3] = c[5] * v[0] - c[6] * v[2];
}

__device__ __forceinline__ void stokes_step(const double c[8], double s, double S[4]) {
    double aI = c[3];
    double Seq = aI > 0.0 ? c[0] / aI : 0.0;
    if (aI * s >= 100.0) {
        S[0] = Seq;
        S[1] = S[2] = S[3] = 0.0;
        return;
    }
    double v[4] = {S[0] - Seq, S[1], S[2], S[3]};
    double w1[4], w2[4], w3[4];
    kprime(c, v, w1);
    kprime(c, w1, w2);
    kprime(c, w2, w3);
    double al2 = c[4] * c[4] + c[5] * c[5];
    double rh2 = c[6] * c[6] + c[7] * c[7];
    double ar = c[4] * c[6] + c[5] * c[7];
    double dif = 0.5 * (al2 - rh2);
    double rt = sqrt(dif * dif + ar * ar);
    double L1s, L2s;
    if (dif >= 0.0) {
        L1s = rt + dif;
        L2s = L1s > 0.0 ? ar * ar / L1s : 0.0;
    } else {
        L2s = rt - dif;
        L1s = L2s > 0.0 ? ar * ar / L2s : 0.0;
    }
    double Th = L1s + L2s;
    double E = exp(-aI * s);
    double out[4];
    if (!(Th > 1e-12 * (al2 + rh2))) {
        // K' (nearly) nilpotent: K'^4 ~ 0, the cubic Taylor polynomial is exact
#pragma unroll
        for (int m = 0; m < 4; ++m)
            out[m] = E * (v[m] - s * w1[m] + 0.5 * s * s * w2[m] - (s * s * s / 6.0) * w3[m]);
    } else {
        double L1 = sqrt(L1s), L2 = sqrt(L2s);
        double ch = E * cosh(s * L1);
        double sh = E * (L1 > 0.0 ? sinh(s * L1) / L1 : s);
        double co = E * cos(s * L2);
        double sn = E * (L2 > 0.0 ? sin(s * L2) / L2 : s);
        double iT = 1.0 / Th;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            out[m] = (ch * (w2[m] + L2s * v[m]) + co * (L1s * v[m] - w2[m])
                      - sh * (w3[m] + L2s * w1[m]) - sn * (L1s * w1[m] - w3[m])) * iT;
    }
    S[0] = Seq + out[0];
    S[1] = out[1];
    S[2] = out[2];
    S[3] = out[3];
}

// unpolarized segment, eq. (unpolarized)
__device__ __forceinline__ double unpol_segment(double I, double j, double al, double dl) {
    if (al > 0.0) {
        double dtau = al * dl;
        if (dtau < 100.0) return exp(-dtau) * (I + expm1(dtau) * j / al);
        return j / al;
    }
    return I + j * dl;
}

struct TransferOut {
    double S[4];
    double tau, Ij;
    int nsamp, nrec;
};

struct TransferParams {
    double ds_max;
    double L;          // GM/c^2 in cm
};

// Per-lane state of the source-to-camera walk over one ray's records.  The
// walk is a state machine so that a persistent wave can interleave rays:
// begin_ray -> (next_step -> piece*)* -> finish_ray.  The quartic of the step
// being cut into pieces lives in LDS (35 doubles per lane, lane-interleaved)
// and is read back for every piece through an offset the compiler cannot
// hoist, so it does not occupy registers across pieces.  blockDim.x == 64.
struct RayWalk {
    const double *rec;   // the ray's records
    double kt, n_norm, lscale;
    int st;              // next step to open (counting down), -1: all opened
    int p;               // next piece of the open step (counting down), -1: none
    int nsub;
    bool inb, started;
    double dl, pdl;
    double I, tau, Ij;
    int nsamp, nrec;
    double pys[7], pyb[7];   // previous record: sample and boundary (x^mu, k_a)
    Coh N;
};

__device__ __forceinline__ void begin_ray(RayWalk &w, const double *rec, int n_acc, double kt, double n_norm,
                                          double L) {
    w.rec = rec;
    w.kt = kt;
    w.n_norm = n_norm;
    w.lscale = L / n_norm;
    w.st = n_acc - 1;
    w.p = -1;
    w.nsub = 0;
    w.inb = false;
    w.started = false;
    w.dl = w.pdl = 0.0;
    w.I = w.tau = w.Ij = 0.0;
    w.nsamp = w.nrec = 0;
#pragma unroll
    for (int m = 0; m < 10; ++m) w.N.r[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) w.N.i[m] = 0.0;
}

__device__ __forceinline__ void load_state7(const double *r, double y[7]) {
#pragma unroll
    for (int m = 0; m < 7; ++m) y[m] = r[m];
}

// Open step w.st: sampling decision, number of pieces, quartic into LDS.
__device__ __forceinline__ void next_step(RayWalk &w, const GeoParams &P, const DevGrid &g,
                                          const TransferParams &tp, double *s_q, int lane) {
    const double *r = w.rec + (long long)w.st * kRecDoubles;
    double y0[7], ym[7], y1[7];
    load_state7(r, y0);
    load_state7(r + 8, ym);
    load_state7(r + kRecDoubles, y1);
    double h = r[7], ds = r[15];
    // chords use the spatial components 1..3 of (t, x, y, z, ...)
    w.inb = chord_meets_box(g.bb, y0, ym) || chord_meets_box(g.bb, ym, y1);
    int nsub = 1;
    if (w.inb && tp.ds_max > 0.0) {
        // at most 2^24 pieces per step; a non-finite length gives one piece
        double q = ceil(ds / tp.ds_max);
        nsub = (q >= 1.0) ? (int)fmin(q, 16777216.0) : 1;
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) s_q[m * 64 + lane] = y0[m];
    if (nsub > 1) {
        double f0[7], f1[7];
        geo_rhs(P.a, P.flat, y0, w.kt, f0);
        geo_rhs(P.a, P.flat, y1, w.kt, f1);
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            double A = y1[m] - y0[m] - h * f0[m];
            double B = h * (f1[m] - f0[m]);
            double C = 16.0 * (ym[m] - y0[m]) - 8.0 * h * f0[m];
            s_q[(7 + m) * 64 + lane] = h * f0[m];
            s_q[(14 + m) * 64 + lane] = -5.0 * A + B + C;
            s_q[(21 + m) * 64 + lane] = 14.0 * A - 3.0 * B - 2.0 * C;
            s_q[(28 + m) * 64 + lane] = -8.0 * A + 2.0 * B + C;
        }
    }
    w.nsub = nsub;
    w.dl = fabs(h) / (double)nsub;
    w.nrec += nsub;
    w.p = nsub - 1;
    --w.st;
}

__device__ __forceinline__ void quartic_at(const double *s_q, int off, double th, double y[8], double kt) {
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        int q = m < 4 ? m : m + 1;
        y[q] = s_q[m * 64 + off] +
               th * (s_q[(7 + m) * 64 + off] +
                     th * (s_q[(14 + m) * 64 + off] + th * (s_q[(21 + m) * 64 + off] + th * s_q[(28 + m) * 64 + off])));
    }
    y[4] = kt;
}

// Process piece w.p of the open step.
template <bool POL>
__device__ __forceinline__ void piece(RayWalk &w, const GeoParams &P, const DevGrid &g, const PlasmaParams &pp,
                                      const double *s_q, int lane) {
    const double a = P.a;
    const int flat = P.flat;
    int off = lane;
    asm volatile("" : "+v"(off));   // keep the LDS reads here
    const int p = w.p;
    double ys[8], yb[8];
    if (w.nsub == 1) {
        const double *rr = w.rec + (long long)(w.st + 1) * kRecDoubles + 8;
        ys[0] = rr[0]; ys[1] = rr[1]; ys[2] = rr[2]; ys[3] = rr[3];
        ys[5] = rr[4]; ys[6] = rr[5]; ys[7] = rr[6];
        ys[4] = w.kt;
    } else {
        quartic_at(s_q, off, ((double)p + 0.5) / (double)w.nsub, ys, w.kt);
    }
    if (p == 0) {
#pragma unroll
        for (int m = 0; m < 7; ++m) yb[m < 4 ? m : m + 1] = s_q[m * 64 + off];
        yb[4] = w.kt;
    } else {
        quartic_at(s_q, off, (double)p / (double)w.nsub, yb, w.kt);
    }
    w.p = p - 1;
    Sample smp;
    smp.plasma = false;
    if (w.inb) sample_point(a, flat, g, pp, ys, w.n_norm, smp);
    double dlp = w.lscale * w.dl;
    if (!POL) {
        if (smp.plasma) {
            ++w.nsamp;
            w.I = unpol_segment(w.I, smp.c[0], smp.c[3], dlp);
            w.tau += smp.c[3] * dlp;
            w.Ij += smp.c[0] * dlp;
        }
        return;
    }
    if (!w.started && !smp.plasma) return;
    if (w.started) {
        double ya[8] = {w.pys[0], w.pys[1], w.pys[2], w.pys[3], w.kt, w.pys[4], w.pys[5], w.pys[6]};
        double yc[8] = {w.pyb[0], w.pyb[1], w.pyb[2], w.pyb[3], w.kt, w.pyb[4], w.pyb[5], w.pyb[6]};
        transport_step(a, flat, ya, yc, 0.5 * (w.pdl + w.dl), w.N);
    }
    w.started = true;
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        w.pys[m] = ys[m < 4 ? m : m + 1];
        w.pyb[m] = yb[m < 4 ? m : m + 1];
    }
    w.pdl = w.dl;
    if (smp.plasma) {
        ++w.nsamp;
        w.tau += smp.c[3] * dlp;
        w.Ij += smp.c[0] * dlp;
        bool any = false;
#pragma unroll
        for (int m = 0; m < 8; ++m) any = any || (smp.c[m] != 0.0);
        if (any) {
            KS k = ks_point(a, flat, ys[1], ys[2], ys[3]);
            double e[4][4];
            tetrad(k, smp.u, ys + 4, smp.b, e);
            double S[4];
            coh_to_stokes(k, e[1], e[2], w.N, S);
            stokes_step(smp.c, dlp, S);
            stokes_to_coh(e[1], e[2], S, w.N);
        }
    }
}

// Close the ray at the pixel: final half transport, camera Stokes basis.
template <bool POL>
__device__ __forceinline__ void finish_ray(RayWalk &w, const GeoParams &P, const double upix[4], const double Hv[4],
                                           TransferOut &o) {
    o.tau = w.tau;
    o.Ij = w.Ij;
    o.nsamp = w.nsamp;
    o.nrec = w.nrec;
    o.S[0] = o.S[1] = o.S[2] = o.S[3] = 0.0;
    if (!POL) {
        o.S[0] = w.I;
        return;
    }
    if (!w.started) return;
    const double *rec = w.rec;
    double y0[8];
    y0[0] = rec[0]; y0[1] = rec[1]; y0[2] = rec[2]; y0[3] = rec[3];
    y0[4] = w.kt; y0[5] = rec[4]; y0[6] = rec[5]; y0[7] = rec[6];
    double ya[8] = {w.pys[0], w.pys[1], w.pys[2], w.pys[3], w.kt, w.pys[4], w.pys[5], w.pys[6]};
    transport_step(P.a, P.flat, ya, y0, 0.5 * w.pdl, w.N);
    KS k = ks_point(P.a, P.flat, y0[1], y0[2], y0[3]);
    double mH[4] = {-Hv[0], -Hv[1], -Hv[2], -Hv[3]};
    double e[4][4];
    tetrad(k, upix, y0 + 4, mH, e);
    coh_to_stokes(k, e[1], e[2], w.N, o.S);
}

// Whole ray by one lane (used where rays are not interleaved).
template <bool POL>
__device__ __forceinline__ void transfer_ray(const GeoParams &P, const DevGrid &g, const PlasmaParams &pp,
                                             const TransferParams &tp, const double *rec, int n_acc, double kt,
                                             double n_norm, const double upix[4], const double Hv[4],
                                             TransferOut &o) {
    __shared__ double s_q[35 * 64];
    const int lane = threadIdx.x;
    RayWalk w;
    begin_ray(w, rec, n_acc, kt, n_norm, tp.L);
    while (w.st >= 0 || w.p >= 0) {
        if (w.p < 0) next_step(w, P, g, tp, s_q, lane);
        piece<POL>(w, P, g, pp, s_q, lane);
    }
    finish_ray<POL>(w, P, upix, Hv, o);
}

}  // namespace bl
