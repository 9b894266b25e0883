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

template <typename R>
struct Coh {
    R r[10], i[6];
};

template <typename R>
__device__ __forceinline__ R Rget(const Coh<R> &N, int a, int b) {
    return N.r[sidx(a, b)];
}
template <typename R>
__device__ __forceinline__ R Iget(const Coh<R> &N, int a, int b) {
    return a == b ? R(0) : (a < b ? N.i[aidx(a, b)] : -N.i[aidx(b, a)]);
}

// dN^ab/dlambda = -(G^a_d N^db + G^b_d N^ad), the parallel transport of N,
// with G in the factored form of conn_geom:
//   (G N)^ab = lu^a (B.N)^b + Yt^a (l.N)^b + (h Om N)^ab,
// and dRe N = -(G R + (G R)^T), dIm N = -(G I - (G I)^T) for the symmetric
// real part R and the antisymmetric imaginary part I.
template <typename R>
__device__ __forceinline__ void transport_apply(const ConnF<R> &c, const Coh<R> &N, Coh<R> &dN) {
    R bR[4], bI[4], lR[4], lI[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        bR[b] = R(0);
        bI[b] = R(0);
        lR[b] = R(0);
        lI[b] = R(0);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            bR[b] += c.B[d] * Rget(N, d, b);
            lR[b] += c.l4[d] * Rget(N, d, b);
            if (d != b) {
                bI[b] += c.B[d] * Iget(N, d, b);
                lI[b] += c.l4[d] * Iget(N, d, b);
            }
        }
    }
    // (G R)^ab and (G I)^ab
    auto GR = [&](int a, int b) -> R {
        R v = c.lu[a] * bR[b] + c.Yt[a] * lR[b];
        if (a > 0) v += conn_om(c, a, Rget(N, 1, b), Rget(N, 2, b), Rget(N, 3, b));
        return v;
    };
    auto GI = [&](int a, int b) -> R {
        R v = c.lu[a] * bI[b] + c.Yt[a] * lI[b];
        if (a > 0) v += conn_om(c, a, Iget(N, 1, b), Iget(N, 2, b), Iget(N, 3, b));
        return v;
    };
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) dN.r[sidx(a, b)] = -(GR(a, b) + GR(b, a));
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) dN.i[aidx(a, b)] = GI(b, a) - GI(a, b);
}

// One explicit-midpoint transport step of length dl: predictor with the
// connection at ya, corrector at yb (states x^mu, k_mu).
template <typename R>
__device__ __forceinline__ void transport_step(R a, int flat, const R ya[8], const R yb[8], R dl, Coh<R> &N) {
    if (flat) return;   // the connection vanishes
    ConnF<R> c;
    Coh<R> d, h;
    conn_geom(a, flat, ya, ya + 4, c);
    transport_apply(c, N, d);
#pragma unroll
    for (int m = 0; m < 10; ++m) h.r[m] = N.r[m] + R(0.5) * dl * d.r[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) h.i[m] = N.i[m] + R(0.5) * dl * d.i[m];
    conn_geom(a, flat, yb, yb + 4, c);
    transport_apply(c, h, d);
#pragma unroll
    for (int m = 0; m < 10; ++m) N.r[m] += dl * d.r[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) N.i[m] += dl * d.i[m];
}

// Stokes parameters of N in the screen vectors of a tetrad, given covariant
// (p = e1_a, q = e2_a): I = N11 + N22, Q = N11 - N22, U = 2 Re N12,
// V = -2 Im N12 with N11 = N^ab p_a p_b etc.
template <typename R>
__device__ __forceinline__ void coh_to_stokes(const R p[4], const R q[4], const Coh<R> &N, R S[4]) {
    // through the vectors Re(N) p, Re(N) q and Im(N) q
    R rp[4], rq[4], iq[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        rp[a] = R(0);
        rq[a] = R(0);
        iq[a] = R(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            rp[a] += Rget(N, a, b) * p[b];
            rq[a] += Rget(N, a, b) * q[b];
            if (a != b) iq[a] += Iget(N, a, b) * q[b];
        }
    }
    R n11 = R(0), n22 = R(0), n12r = R(0), n12i = R(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        n11 += p[a] * rp[a];
        n22 += q[a] * rq[a];
        n12r += p[a] * rq[a];
        n12i += p[a] * iq[a];
    }
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = R(2) * n12r;
    S[3] = R(-2) * n12i;
}

// N = 1/2 [(I+Q) e1 e1 + (I-Q) e2 e2 + (U - iV) e1 e2 + (U + iV) e2 e1]
template <typename R>
__device__ __forceinline__ void stokes_to_coh(const R e1[4], const R e2[4], const R S[4], Coh<R> &N) {
    R n11 = R(0.5) * (S[0] + S[1]), n22 = R(0.5) * (S[0] - S[1]), n12r = R(0.5) * S[2], n12i = R(-0.5) * S[3];
    // Re N^ab = al^a e1^b + be^a e2^b with al = n11 e1 + n12r e2, be = n22 e2 + n12r e1
    R al[4], be[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        al[a] = n11 * e1[a] + n12r * e2[a];
        be[a] = n22 * e2[a] + n12r * e1[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) N.r[sidx(a, b)] = al[a] * e1[b] + be[a] * e2[b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) N.i[aidx(a, b)] = n12i * (e1[a] * e2[b] - e2[a] * e1[b]);
}

// Right after a Stokes step N = E S E^T exactly (stokes_to_coh), E = (e1, e2)
// of that sample, so the state is kept as those two vectors and the Stokes
// parameters, in the storage of N: r[0..3] = e1, r[4..7] = e2 and
// (r[8], r[9], i[0], i[1]) = (I, Q, U, V).
template <typename R>
__device__ __forceinline__ void pack_screen(const R e1[4], const R e2[4], const R S[4], Coh<R> &N) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        N.r[m] = e1[m];
        N.r[4 + m] = e2[m];
    }
    N.r[8] = S[0];
    N.r[9] = S[1];
    N.i[0] = S[2];
    N.i[1] = S[3];
}

// The full N of a packed state.
template <typename R>
__device__ __forceinline__ void unpack_screen(Coh<R> &N) {
    R e1[4], e2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        e1[m] = N.r[m];
        e2[m] = N.r[4 + m];
    }
    const R S[4] = {N.r[8], N.r[9], N.i[0], N.i[1]};
    stokes_to_coh(e1, e2, S, N);
}

// a . b over four components
template <typename R>
__device__ __forceinline__ R dot4(const R *a, const R *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

// Stokes parameters on the screen (p, q: covariant e1, e2 of the new sample)
// of a packed state after one merged transport step, without forming N.  The
// step (transport_step) is N' = N + dl A_b(h), h = N + dl/2 A_a(N) with
// A(N) = L N + N L^T, L = -G at the predictor (a) and corrector (b) points.
// With N = E S E^T and F = L_a E (conn_vec at a):
//   h  = P S P^T - dl^2/4 F S F^T,   P = E + dl/2 F,
//   N' = E S E^T + dl (L_b P S P^T + P S (L_b P)^T)
//        - dl^3/4 (L_b F S F^T + F S (L_b F)^T),
// so x^T N' y needs only the contractions of E and F with x and with
// xt = L_b^T x (conn_covec at b; (L_b P)^T x = P^T xt): the same numbers as
// the merged transport followed by coh_to_stokes, up to rounding, in about
// 40 % of the operations.  pt, qt = L_b^T p, L_b^T q.
template <typename R>
__device__ __forceinline__ void screen_transport_stokes(const Coh<R> &N, const R F[2][4], const R pt[4], const R qt[4],
                                                        const R p[4], const R q[4], R dl, R S[4]) {
    const R hd = R(0.5) * dl, c3 = R(0.25) * dl * dl * dl;
    // per covector x and column I: E_x = E_I.x, F_x = F_I.x, R_x = F_I.xt,
    // P_x = E_x + dl/2 F_x, Q_x = E_I.xt + dl/2 R_x
    R Ep[2], Fp[2], Rp[2], Pp[2], Qp[2], Eq[2], Fq[2], Rq[2], Pq[2], Qq[2];
#pragma unroll
    for (int I = 0; I < 2; ++I) {
        const R *EI = N.r + 4 * I;
        Ep[I] = dot4(EI, p);
        Fp[I] = dot4(F[I], p);
        Rp[I] = dot4(F[I], pt);
        Pp[I] = Ep[I] + hd * Fp[I];
        Qp[I] = dot4(EI, pt) + hd * Rp[I];
        Eq[I] = dot4(EI, q);
        Fq[I] = dot4(F[I], q);
        Rq[I] = dot4(F[I], qt);
        Pq[I] = Eq[I] + hd * Fq[I];
        Qq[I] = dot4(EI, qt) + hd * Rq[I];
    }
    // M_IJ(x, y) = E_x,I E_y,J + dl (Q_x,I P_y,J + P_x,I Q_y,J) - dl^3/4 (R_x,I F_y,J + F_x,I R_y,J)
    auto M = [&](const R *Ex, const R *Fx, const R *Rx, const R *Px, const R *Qx, const R *Ey, const R *Fy,
                 const R *Ry, const R *Py, const R *Qy, int I, int J) -> R {
        return Ex[I] * Ey[J] + dl * (Qx[I] * Py[J] + Px[I] * Qy[J]) - c3 * (Rx[I] * Fy[J] + Fx[I] * Ry[J]);
    };
    // S_11 = (I + Q)/2, S_22 = (I - Q)/2, S_12 = conj S_21 = (U - i V)/2
    const R s11 = R(0.5) * (N.r[8] + N.r[9]), s22 = R(0.5) * (N.r[8] - N.r[9]);
    const R rho = R(0.5) * N.i[0], sig = R(-0.5) * N.i[1];
    const R n11 = s11 * M(Ep, Fp, Rp, Pp, Qp, Ep, Fp, Rp, Pp, Qp, 0, 0) +
                  s22 * M(Ep, Fp, Rp, Pp, Qp, Ep, Fp, Rp, Pp, Qp, 1, 1) +
                  R(2) * rho * M(Ep, Fp, Rp, Pp, Qp, Ep, Fp, Rp, Pp, Qp, 0, 1);
    const R n22 = s11 * M(Eq, Fq, Rq, Pq, Qq, Eq, Fq, Rq, Pq, Qq, 0, 0) +
                  s22 * M(Eq, Fq, Rq, Pq, Qq, Eq, Fq, Rq, Pq, Qq, 1, 1) +
                  R(2) * rho * M(Eq, Fq, Rq, Pq, Qq, Eq, Fq, Rq, Pq, Qq, 0, 1);
    const R m01 = M(Ep, Fp, Rp, Pp, Qp, Eq, Fq, Rq, Pq, Qq, 0, 1);
    const R m10 = M(Ep, Fp, Rp, Pp, Qp, Eq, Fq, Rq, Pq, Qq, 1, 0);
    const R n12r = s11 * M(Ep, Fp, Rp, Pp, Qp, Eq, Fq, Rq, Pq, Qq, 0, 0) +
                   s22 * M(Ep, Fp, Rp, Pp, Qp, Eq, Fq, Rq, Pq, Qq, 1, 1) + rho * (m01 + m10);
    const R n12i = sig * (m01 - m10);
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = R(2) * n12r;
    S[3] = R(-2) * n12i;
}

// Exact solution of dS/ds = J - M S over unit length (the coefficients carry
// the segment length) for thermal coefficients, where Kirchhoff's law gives
// J = B_nu M e_I (B_nu = j_I/alpha_I):
//   S = e^{-M} S0 + B_nu (1 - e^{-M}) e_I,   M = alpha_I + K',
// K' the traceless part of M, whose square has eigenvalues p = L1^2 >= 0 and
// q = -L2^2 <= 0 with L1^2, L2^2 = sqrt(((a^2 - r^2)/2)^2 + (a.r)^2) +- (a^2 - r^2)/2.
// Any f(K') = F_e(K'^2) + K' F_o(K'^2) with F_e, F_o the even and odd parts
// of f as functions of the squared eigenvalue, and on the two-point spectrum
// F(K'^2) = F(x0) + F[p,q] (K'^2 - x0) for either x0 in {p, q}, F[p,q] the
// divided difference.  For f = e^{-mu} the parts are C(x) = cosh sqrt(x) and
// -Sh(x) = -sinh sqrt(x)/sqrt(x), both entire in x.  The propagator acts on
// S0 in the form based at q; the source acts on e_I in the form based at p,
// since K'^2 e_I - p e_I = (X^2/((a^2+r^2)/2 + sqrt(...)), 0, -X, 0) with
// X = aQ rV - aV rQ is small exactly where e_I lies near the p eigenspace:
//   src = (1 - e^{-a} cosh L1) e_I - e^{-a} C[p,q] u + e^{-a} Sh(p) K' e_I
//         + e^{-a} Sh[p,q] K' u,   u = K'^2 e_I - p e_I.
// Nothing cancels when the step is optically thin and B_nu dwarfs S0:
// 1 - e^{-a} cosh L1 = -(expm1(L1 - a) + expm1(-L1 - a))/2 with a >= L1, and
// when p - q <= 1 (so |p|, |q| <= 1) the divided differences are summed from
// the Taylor series of C and Sh instead of differenced; in that common case
// cos L2 = C(q) and 1 - e^{-a} cosh L1 = -expm1(-a) - e^{-a} (C(p) - 1) come
// from the series too, so one expm1 and one square root remain.  If alpha_I >= 100 the
// result is B_nu e_I.  c = jI, jQ, jV, aI, aQ, aV, rQ, rV.
template <typename R>
__device__ __forceinline__ void kprime(const R c[8], const R v[4], R w[4]) {
    w[0] = c[4] * v[1] + c[5] * v[3];
    w[1] = c[4] * v[0] + c[7] * v[2];
    w[2] = -c[7] * v[1] + c[6] * v[3];
    w[3] = c[5] * v[0] - c[6] * v[2];
}



// Sh(x) = sum_k x^k / (2k+1)! for |x| <= 1 (the first omitted term is below
// 1/(2K+3)!: 2e-20 in FP64, 3e-8 in FP32)
template <typename R>
__device__ __forceinline__ R sh_series(R x) {
    constexpr int K = sizeof(R) == 8 ? 9 : 4;
    R s = R(0);
#pragma unroll
    for (int k = K; k >= 1; --k) s = (s + R(rfact(2 * k + 1))) * x;
    return s + R(1);
}

// C(x) - 1 = sum_{k>=1} x^k / (2k)! for |x| <= 1 (omitted terms below
// 1/(2K+2)!: 9e-22 in FP64, 2e-9 in FP32)
template <typename R>
__device__ __forceinline__ R cm1_series(R x) {
    constexpr int K = sizeof(R) == 8 ? 10 : 5;
    R s = R(0);
#pragma unroll
    for (int k = K; k >= 1; --k) s = (s + R(rfact(2 * k))) * x;
    return s;
}

// C[p,q] and Sh[p,q] from the series: sum_{k>=1} h_{k-1}(p,q) / (2k)! and
// / (2k+1)!, h_m the complete homogeneous polynomial of degree m.
// (h_K <= K + 1 for |p|, |q| <= 1, so the omitted terms are below
// (K + 1)/(2K+2)!: 1e-20 in FP64, 1e-8 in FP32)
template <typename R>
__device__ __forceinline__ void dd_series(R p, R q, R &dc, R &ds) {
    constexpr int K = sizeof(R) == 8 ? 10 : 5;
    R h = R(1), qk = R(1);
    dc = R(0);
    ds = R(0);
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        dc += h * R(rfact(2 * k));
        ds += h * R(rfact(2 * k + 1));
        qk *= q;
        h = p * h + qk;                               // h_k = p h_{k-1} + q^k
    }
}

template <typename R>
__device__ __forceinline__ void stokes_step(const R c[8], R S[4]) {
    const R aI = c[3];
    const R Bnu = aI > R(0) ? fdiv(c[0], aI) : R(0);
    if (aI >= R(100)) {
        S[0] = Bnu;
        S[1] = S[2] = S[3] = R(0);
        return;
    }
    R w1[4], w2[4], w3[4];
    kprime(c, S, w1);
    kprime(c, w1, w2);
    kprime(c, w2, w3);
    const R al2 = c[4] * c[4] + c[5] * c[5];
    const R rh2 = c[6] * c[6] + c[7] * c[7];
    const R ar = c[4] * c[6] + c[5] * c[7];
    const R dif = R(0.5) * (al2 - rh2);
    const R rt = sqrt(dif * dif + ar * ar);
    R L1s, L2s;
    if (dif >= R(0)) {
        L1s = rt + dif;
        L2s = L1s > R(0) ? fdiv(ar * ar, L1s) : R(0);
    } else {
        L2s = rt - dif;
        L1s = L2s > R(0) ? fdiv(ar * ar, L2s) : R(0);
    }
    const R Th = L1s + L2s;
    const R em1 = fexpm1(-aI);
    // e^{-aI}: 1 + expm1 for a thin step, the exponential itself for a thick
    // one (1 + expm1 keeps only the absolute accuracy of numbers near 1)
    const R E = aI <= R(1) ? R(1) + em1 : fexp(-aI);
    R cq, shq, shp, dc, ds, fp;   // cos L2 - 1, Sh(q), e^{-a} Sh(p), e^{-a} C[p,q], e^{-a} Sh[p,q], 1 - e^{-a} cosh L1
    if (Th <= R(1)) {
        // |p|, |q| <= 1: everything from the series; cos L2 = C(q)
        cq = cm1_series(-L2s);
        shq = sh_series(-L2s);
        shp = E * sh_series(L1s);
        dd_series(L1s, -L2s, dc, ds);
        dc *= E;
        ds *= E;
        fp = -em1 - E * cm1_series(L1s);
    } else {
        const R L1 = sqrt(L1s), L2 = sqrt(L2s);
        R sn, cs;
        fsincos(L2, sn, cs);
        cq = L2s <= R(1) ? cm1_series(-L2s) : cs - R(1);
        const R ep = fexp(L1 - aI), em = fexp(-L1 - aI);   // e^{-aI} e^{+-L1}
        shq = L2s <= R(1) ? sh_series(-L2s) : fdiv(sn, L2);
        shp = L1s <= R(1) ? E * sh_series(L1s) : fdiv(R(0.5) * (ep - em), L1);
        const R iT = fdiv(R(1), Th);
        dc = (R(0.5) * (ep + em) - E * (R(1) + cq)) * iT;
        ds = (shp - E * shq) * iT;
        fp = R(-0.5) * (fexpm1(L1 - aI) + fexpm1(-L1 - aI));
    }
    // a thin step as an increment, with e^{-a} cos L2 - 1 formed without
    // e^{-a} cos L2 (its attenuation would otherwise be quantised to the
    // spacing of numbers near 1); a thick one directly (an increment would
    // lose a strongly attenuated S0 to cancellation)
    const R es = E * shq;
    if (aI <= R(1)) {
        const R ecm1 = em1 + E * cq;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            S[m] += ecm1 * S[m] + dc * (w2[m] + L2s * S[m]) - es * w1[m] - ds * (w3[m] + L2s * w1[m]);
    } else {
        const R ec = E + E * cq;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            S[m] = ec * S[m] + dc * (w2[m] + L2s * S[m]) - es * w1[m] - ds * (w3[m] + L2s * w1[m]);
    }
    if (Bnu > R(0)) {
        const R X = c[4] * c[7] - c[5] * c[6];
        const R den = R(0.5) * (al2 + rh2) + rt;
        const R u0 = den > R(0) ? fdiv(X * X, den) : R(0);
        // K' e_I = (0, aQ, 0, aV);  K' u for u = (u0, 0, -X, 0)
        const R ku1 = c[4] * u0 - c[7] * X, ku3 = c[5] * u0 + c[6] * X;
        S[0] += Bnu * (fp - dc * u0);
        S[1] += Bnu * (shp * c[4] + ds * ku1);
        S[2] += Bnu * (dc * X);
        S[3] += Bnu * (shp * c[5] + ds * ku3);
    }
}

// The plasma substep for any source vector (nonthermal electrons: no
// Kirchhoff relation between J and M): with the segment length folded into
// the coefficients, dS/ds = J - M S over s in [0, 1] gives
// S1 = e^-M S0 + int_0^1 e^-M(1-s) J ds, the upper block of the exponential of
// the augmented matrix A = [[-M, J], [0, 0]].  Evaluated in FP64 in both
// forms: A is scaled by 2^-k to a row-sum norm of at most 1/4, its Taylor
// series summed through A^14/14! in Horner form on pairs (E, v) standing for
// [[E, v], [0, 1]] (truncation below 1e-20), then squared k times.  With
// aI >= 100 (the optical-depth cap of the unpolarized equation) S = M^-1 J.
__device__ __forceinline__ void mat4_mul(const double A[16], const double B[16], double C[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            C[4 * i + j] = A[4 * i] * B[j] + A[4 * i + 1] * B[4 + j] + A[4 * i + 2] * B[8 + j] + A[4 * i + 3] * B[12 + j];
}

template <typename R>
__device__ __forceinline__ void stokes_step_general(const R cr[8], R Sr[4]) {
    const double aI = cr[3], aQ = cr[4], aV = cr[5], rQ = cr[6], rV = cr[7];
    // M rows: (aI aQ 0 aV), (aQ aI rV 0), (0 -rV aI rQ), (aV 0 -rQ aI); aU, rU = 0
    const double M[16] = {aI, aQ, 0.0, aV, aQ, aI, rV, 0.0, 0.0, -rV, aI, rQ, aV, 0.0, -rQ, aI};
    const double J[4] = {(double)cr[0], (double)cr[1], 0.0, (double)cr[2]};
    double S0[4] = {(double)Sr[0], (double)Sr[1], (double)Sr[2], (double)Sr[3]};
    if (aI >= 100.0) {
        // x = M^-1 J by the adjugate, from the 2x2 minors of the first two and
        // of the last two rows (no indexed arrays, so nothing goes to scratch)
        const double *m = M;
        const double s0 = m[0] * m[5] - m[4] * m[1], s1 = m[0] * m[6] - m[4] * m[2];
        const double s2 = m[0] * m[7] - m[4] * m[3], s3 = m[1] * m[6] - m[5] * m[2];
        const double s4 = m[1] * m[7] - m[5] * m[3], s5 = m[2] * m[7] - m[6] * m[3];
        const double c5 = m[10] * m[15] - m[14] * m[11], c4 = m[9] * m[15] - m[13] * m[11];
        const double c3 = m[9] * m[14] - m[13] * m[10], c2 = m[8] * m[15] - m[12] * m[11];
        const double c1 = m[8] * m[14] - m[12] * m[10], c0 = m[8] * m[13] - m[12] * m[9];
        const double id = 1.0 / (s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0);
        // rows of adj(M)
        const double a00 = m[5] * c5 - m[6] * c4 + m[7] * c3, a01 = -m[1] * c5 + m[2] * c4 - m[3] * c3;
        const double a02 = m[13] * s5 - m[14] * s4 + m[15] * s3, a03 = -m[9] * s5 + m[10] * s4 - m[11] * s3;
        const double a10 = -m[4] * c5 + m[6] * c2 - m[7] * c1, a11 = m[0] * c5 - m[2] * c2 + m[3] * c1;
        const double a12 = -m[12] * s5 + m[14] * s2 - m[15] * s1, a13 = m[8] * s5 - m[10] * s2 + m[11] * s1;
        const double a20 = m[4] * c4 - m[5] * c2 + m[7] * c0, a21 = -m[0] * c4 + m[1] * c2 - m[3] * c0;
        const double a22 = m[12] * s4 - m[13] * s2 + m[15] * s0, a23 = -m[8] * s4 + m[9] * s2 - m[11] * s0;
        const double a30 = -m[4] * c3 + m[5] * c1 - m[6] * c0, a31 = m[0] * c3 - m[1] * c1 + m[2] * c0;
        const double a32 = -m[12] * s3 + m[13] * s1 - m[14] * s0, a33 = m[8] * s3 - m[9] * s1 + m[10] * s0;
        Sr[0] = (R)((a00 * J[0] + a01 * J[1] + a02 * J[2] + a03 * J[3]) * id);
        Sr[1] = (R)((a10 * J[0] + a11 * J[1] + a12 * J[2] + a13 * J[3]) * id);
        Sr[2] = (R)((a20 * J[0] + a21 * J[1] + a22 * J[2] + a23 * J[3]) * id);
        Sr[3] = (R)((a30 * J[0] + a31 * J[1] + a32 * J[2] + a33 * J[3]) * id);
        return;
    }
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        nrm = fmax(nrm, fabs(M[4 * i]) + fabs(M[4 * i + 1]) + fabs(M[4 * i + 2]) + fabs(M[4 * i + 3]) + fabs(J[i]));
    int k = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++k;
    }
    const double sc = ldexp(1.0, -k);
    double B[16], b[4];
#pragma unroll
    for (int m = 0; m < 16; ++m) B[m] = -M[m] * sc;
#pragma unroll
    for (int m = 0; m < 4; ++m) b[m] = J[m] * sc;
    // P = I + B/14; P = I + (B P)/i for i = 13 .. 1 (pairs (E, v))
    double E[16], v[4];
#pragma unroll
    for (int m = 0; m < 16; ++m) E[m] = ((m % 5) == 0 ? 1.0 : 0.0) + B[m] * (1.0 / 14.0);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = b[m] * (1.0 / 14.0);
    for (int i = 13; i >= 1; --i) {
        double T[16], w[4];
        mat4_mul(B, E, T);
        const double ri = 1.0 / (double)i;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            w[r] = (B[4 * r] * v[0] + B[4 * r + 1] * v[1] + B[4 * r + 2] * v[2] + B[4 * r + 3] * v[3] + b[r]) * ri;
#pragma unroll
        for (int m = 0; m < 16; ++m) E[m] = ((m % 5) == 0 ? 1.0 : 0.0) + T[m] * ri;
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = w[m];
    }
    for (int q = 0; q < k; ++q) {   // [[E, v], [0, 1]]^2 = [[E E, E v + v], [0, 1]]
        double T[16], w[4];
        mat4_mul(E, E, T);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            w[r] = E[4 * r] * v[0] + E[4 * r + 1] * v[1] + E[4 * r + 2] * v[2] + E[4 * r + 3] * v[3] + v[r];
#pragma unroll
        for (int m = 0; m < 16; ++m) E[m] = T[m];
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = w[m];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        Sr[r] = (R)(E[4 * r] * S0[0] + E[4 * r + 1] * S0[1] + E[4 * r + 2] * S0[2] + E[4 * r + 3] * S0[3] + v[r]);
}

// The same general plasma substep in closed form, for the FP32 transfer:
// S1 = e^-M S0 + Phi J with Phi = int_0^1 e^-Ms ds = phi(M), phi(x) = (1 - e^-x)/x.
// With M = a + K' and e^{-K's} = C(K'^2 s^2) - K' s Sh(K'^2 s^2),
// Phi = E(K'^2) - K' O(K'^2), E(x) = int_0^1 e^{-as} C(x s^2) ds and
// O(x) = int_0^1 e^{-as} s Sh(x s^2) ds, both taken on the two-point spectrum
// {p = L1^2, q = -L2^2} of K'^2 in the form based at q (as the propagator of
// the thermal step).  At x = p, E = (phi(a - L1) + phi(a + L1))/2 and
// O = (phi(a - L1) - phi(a + L1))/(2 L1), the latter from
// O = sum_k L1^2k m_{2k+1}/(2k+1)! when L1^2 <= 1/16 (m_j = int_0^1 s^j e^{-as} ds:
// the difference would cancel); at x = q with b = L2,
// E = (a X + b e^-a sin b)/(a^2 + b^2) and O = (X - a e^-a sin b / b)/(a^2 + b^2),
// X = 1 - e^-a cos b = -expm1(-a) + 2 e^-a sin^2(b/2) (no cancellation).
// Where a <= 1 and p - q <= 1 the series Phi J = sum_n (-M)^n J/(n+1)! (through
// n = 14) is summed instead.  The propagator is the thermal step's; for a > 1
// it is applied directly (e^-a cos b S0 + ...) with e^-a from the
// exponential, not as an increment of S0.  With a >= 100, S = M^-1 J (the
// optical-depth cap), from (a - K') (a^2 - K'^2)^-1 on the same spectrum.
template <typename R>
__device__ __forceinline__ R phi_r(R y) {   // (1 - e^-y)/y
    if (fabs(y) < R(1e-6)) return R(1) - R(0.5) * y;
    return -fexpm1(-y) * fdiv(R(1), y);
}

template <typename R>
__device__ __forceinline__ void stokes_step_nth(const R c[8], R S[4]) {
    const R a = c[3];
    const R J[4] = {c[0], c[1], R(0), c[2]};
    const R al2 = c[4] * c[4] + c[5] * c[5];
    const R rh2 = c[6] * c[6] + c[7] * c[7];
    const R ar = c[4] * c[6] + c[5] * c[7];
    const R dif = R(0.5) * (al2 - rh2);
    const R rt = sqrt(dif * dif + ar * ar);
    R L1s, L2s;
    if (dif >= R(0)) {
        L1s = rt + dif;
        L2s = L1s > R(0) ? fdiv(ar * ar, L1s) : R(0);
    } else {
        L2s = rt - dif;
        L1s = L2s > R(0) ? fdiv(ar * ar, L2s) : R(0);
    }
    const R Th = L1s + L2s;
    R out[4] = {R(0), R(0), R(0), R(0)};
    if (a < R(100)) {
        R w1[4], w2[4], w3[4];
        kprime(c, S, w1);
        kprime(c, w1, w2);
        kprime(c, w2, w3);
        const R em1 = fexpm1(-a);
        const R E = a <= R(1) ? R(1) + em1 : fexp(-a);
        R cq, shq, dc, ds;
        if (Th <= R(1)) {
            cq = cm1_series(-L2s);
            shq = sh_series(-L2s);
            dd_series(L1s, -L2s, dc, ds);
            dc *= E;
            ds *= E;
        } else {
            const R L1 = sqrt(L1s), L2 = sqrt(L2s);
            R sn, cs;
            fsincos(L2, sn, cs);
            cq = L2s <= R(1) ? cm1_series(-L2s) : cs - R(1);
            const R ep = fexp(L1 - a), em = fexp(-L1 - a);
            shq = L2s <= R(1) ? sh_series(-L2s) : fdiv(sn, L2);
            const R shp = L1s <= R(1) ? E * sh_series(L1s) : fdiv(R(0.5) * (ep - em), L1);
            const R iT = fdiv(R(1), Th);
            dc = (R(0.5) * (ep + em) - E * (R(1) + cq)) * iT;
            ds = (shp - E * shq) * iT;
        }
        const R es = E * shq;
        if (a <= R(1)) {
            const R ecm1 = em1 + E * cq;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                out[m] = S[m] + ecm1 * S[m] + dc * (w2[m] + L2s * S[m]) - es * w1[m] - ds * (w3[m] + L2s * w1[m]);
        } else {
            const R ec = E + E * cq;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                out[m] = ec * S[m] + dc * (w2[m] + L2s * S[m]) - es * w1[m] - ds * (w3[m] + L2s * w1[m]);
        }
    }
    if (a <= R(1) && Th <= R(1)) {
        // Phi J = sum_n (-M)^n J / (n+1)!, Horner: t <- J/(n+1)! - M t
        R t[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) t[m] = J[m] * R(rfact(15));
#pragma unroll
        for (int n = 13; n >= 0; --n) {
            R kt[4];
            kprime(c, t, kt);
#pragma unroll
            for (int m = 0; m < 4; ++m) t[m] = J[m] * R(rfact(n + 1)) - (a * t[m] + kt[m]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) S[m] = out[m] + t[m];
        return;
    }
    R j1[4], j2[4], j3[4];
    kprime(c, J, j1);
    kprime(c, j1, j2);
    kprime(c, j2, j3);
    if (a >= R(100)) {
        // M^-1 J = (a - K') g(K'^2) J with g(x) = 1/(a^2 - x) on {p, q}: g(q) =
        // 1/(a^2 + L2^2), g[p,q] = g(p) g(q), a^2 - p = (a - L1)(a + L1) > 0
        const R L1 = sqrt(L1s);
        const R gq = fdiv(R(1), a * a + L2s);
        const R gpq = gq * fdiv(R(1), (a - L1) * (a + L1));
#pragma unroll
        for (int m = 0; m < 4; ++m)
            S[m] = a * (gq * J[m] + gpq * (j2[m] + L2s * J[m])) - gq * j1[m] - gpq * (j3[m] + L2s * j1[m]);
        return;
    }
    const R L1 = sqrt(L1s), b = sqrt(L2s);
    const R pm = phi_r(a - L1), pp = phi_r(a + L1);
    const R Ep = R(0.5) * (pm + pp);
    R Op;
    if (L1s <= R(0.0625)) {
        // m_1, m_3, m_5, m_7: for a <= 1 their series sum_i (-a)^i/(i! (i+j+1)),
        // else the recurrence m_j = (j m_{j-1} - e^-a)/a from m_0 = phi(a)
        R m1, m3, m5, m7;
        if (a <= R(1)) {
            R t1 = R(0), t3 = R(0), t5 = R(0), t7 = R(0);
#pragma unroll
            for (int i = 12; i >= 0; --i) {
                t1 = t1 * (-a) + R(rfact(i) / (i + 2));
                t3 = t3 * (-a) + R(rfact(i) / (i + 4));
                t5 = t5 * (-a) + R(rfact(i) / (i + 6));
                t7 = t7 * (-a) + R(rfact(i) / (i + 8));
            }
            m1 = t1;
            m3 = t3;
            m5 = t5;
            m7 = t7;
        } else {
            const R ea = fexp(-a), ia = fdiv(R(1), a);
            const R m0 = -fexpm1(-a) * ia;
            m1 = (m0 - ea) * ia;
            const R m2 = (R(2) * m1 - ea) * ia;
            m3 = (R(3) * m2 - ea) * ia;
            const R m4 = (R(4) * m3 - ea) * ia;
            m5 = (R(5) * m4 - ea) * ia;
            const R m6 = (R(6) * m5 - ea) * ia;
            m7 = (R(7) * m6 - ea) * ia;
        }
        Op = m1 + L1s * (m3 * R(rfact(3)) + L1s * (m5 * R(rfact(5)) + L1s * m7 * R(rfact(7))));
    } else {
        Op = (pm - pp) * fdiv(R(1), R(2) * L1);
    }
    const R Ea = fexp(-a);
    R sn, cs;
    fsincos(b, sn, cs);
    const R sinc = L2s <= R(1) ? sh_series(-L2s) : fdiv(sn, b);
    R hs, hc;
    fsincos(R(0.5) * b, hs, hc);
    const R X = -fexpm1(-a) + R(2) * Ea * hs * hs;   // 1 - e^-a cos b
    const R iden = fdiv(R(1), a * a + L2s);
    const R Eq = (a * X + b * Ea * sn) * iden;
    const R Oq = (X - a * Ea * sinc) * iden;
    R Edd = R(0), Odd = R(0);
    if (Th > R(1e-30)) {
        const R iT = fdiv(R(1), Th);
        Edd = (Ep - Eq) * iT;
        Odd = (Op - Oq) * iT;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
        S[m] = out[m] + Eq * J[m] + Edd * (j2[m] + L2s * J[m]) - Oq * j1[m] - Odd * (j3[m] + L2s * j1[m]);
}

// unpolarized segment, eq. (unpolarized), with j and alpha carrying the length:
// e^{-dtau} (I + (e^{dtau} - 1) j/dtau) written as I + (e^{-dtau} - 1) (I - j/dtau),
// which cannot overflow in FP32 below the cut at 100 and keeps a thin
// segment's attenuation exact to the accuracy of e^{-dtau} - 1
template <typename R>
__device__ __forceinline__ R unpol_segment(R I, R j, R dtau) {
    if (dtau > R(0)) {
        if (dtau < R(100)) return I + fexpm1(-dtau) * (I - fdiv(j, dtau));
        return fdiv(j, dtau);
    }
    return I + j;
}

struct TransferOut {
    double S[4];
    double tau, Ij;
    int nsamp, nrec;
};

struct TransferParams {
    double ds_max;
    double L;          // GM/c^2 in cm
    double nu_cam;     // observing frequency
};

// Per-lane state of the source-to-camera walk over one ray's records.  The
// walk is a state machine so that a persistent wave can interleave rays:
// begin_ray -> (next_step -> piece*)* -> finish_ray.  Positions and the
// quartic are FP64; R is the type of the coefficients, frames, transport and
// Stokes state.  Intensities are carried in camera units (nu^3 times the
// invariant), with the segment length folded into the coefficients:
//   emission  j' = j_nu L dl (nu_cam/n)^3 / omega^2,
//   depths    a' = alpha_nu L dl omega,  r' = rho_nu L dl omega,
// which equal nu_cam^3 j/nu^2 dlambda_phys and alpha nu dlambda_phys with
// dlambda_phys = L dl/n, nu = n omega.  The quartic of the step being cut into
// pieces lives in LDS (the node in FP64, coefficients in R; lane-interleaved) and is read back
// for every piece through an offset the compiler cannot hoist, so it does not
// occupy registers across pieces.  blockDim.x == 64.
// The open step's dense output in LDS, lane-interleaved: the node y0 in FP64
// and the quartic's coefficients c1..c4 in R, so that
// y(theta) = y0 + theta (c1 + theta (c2 + theta (c3 + theta c4))), for the six
// components x, y, z, k_x, k_y, k_z (the metric and the fluid data are
// stationary, so nothing in the transfer reads the coordinate time).
constexpr int kQC = 6;   // quartic components kept: state components 1..6
template <typename R>
struct QuartLds {
    double y0[kQC * 64];
    R c[4 * kQC * 64];
};

template <typename R>
struct RayWalk {
    const double *rec;   // the ray's records
    R kt, n_norm;        // k_t (held fixed) and the frequency normalisation
    R L;                 // GM/c^2 in cm
    R lj;                // L (nu_cam/n)^3
    int st;              // next step to open (counting down), -1: all opened
    int p;               // next piece of the open step (counting down), -1: none
    int nsub;
    double inv_nsub;     // 1 / nsub
    bool inb, started;
    bool fresh;          // N packed by pack_screen (the last sample did a Stokes step)
    R dl, pdl;           // affine length of the open step's pieces, and of the previous piece
    R I, tau, Ij;
    R tau_c, Ij_c;       // compensation terms of the two sums
    int nsamp, nrec;
    R pys[kQC], pyb[kQC];   // previous piece: sample and boundary (x, y, z, k_x, k_y, k_z)
    Coh<R> N;
    BlockCache bc;       // the last block table entry (used by the FP64 polarized walk)
    // averaged quantities (their own pass): for q = rho, n_e, p, Theta_e, B,
    // sigma, beta^-1, the sums of q dlambda and q dI_j and the tau-relaxed <q>
    R av_l[7], av_j[7], av_t[7];
};

template <typename R>
__device__ __forceinline__ void begin_ray(RayWalk<R> &w, const double *rec, int n_acc, double kt, double den,
                                          const TransferParams &tp) {
    // n = nu / den (camera_pixel), so nu_cam / n = den
    w.rec = rec;
    w.kt = (R)kt;
    w.n_norm = (R)(tp.nu_cam / den);
    w.L = (R)tp.L;
    w.lj = (R)(tp.L * den * den * den);
    // the last step sampled against the grid (stored with the final state);
    // the vacuum steps beyond it count one record each and are not walked
    const int last = (int)rec[(long long)n_acc * kRecDoubles + 23];
    w.st = last;
    w.p = -1;
    w.nsub = 0;
    w.inv_nsub = 1.0;
    w.inb = false;
    w.started = false;
    w.fresh = false;
    w.dl = w.pdl = R(0);
    w.I = w.tau = w.Ij = w.tau_c = w.Ij_c = R(0);
    w.nsamp = 0;
    w.nrec = n_acc - 1 - last;
    w.bc.cell = -1;
#pragma unroll
    for (int m = 0; m < 7; ++m) w.av_l[m] = w.av_j[m] = w.av_t[m] = R(0);
#pragma unroll
    for (int m = 0; m < 10; ++m) w.N.r[m] = R(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) w.N.i[m] = R(0);
}

// Kahan-compensated s += x
template <typename R>
__device__ __forceinline__ void csum(R &s, R &c, R x) {
    R y = x - c;
    R t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ __forceinline__ void load_state7(const double *r, double y[7]) {
#pragma unroll
    for (int m = 0; m < 7; ++m) y[m] = r[m];
}

// Open step w.st: the sampling decision and number of pieces stored with the
// record, the node and (for more than one piece) the quartic into LDS.  The
// FP32 form reads the quartic's coefficients from the record (the
// FP32-quartic layout); the FP64 form forms them from y0, y1, f0, f1 and y_mid.
template <typename R>
__device__ __forceinline__ void next_step(RayWalk<R> &w, QuartLds<R> &s_q, int lane) {
    const double *r = w.rec + (long long)w.st * kRecDoubles;
    double y0[7];
    load_state7(r, y0);
    const double h = r[7], code = r[23];
    w.inb = code > 0.0;
    const int nsub = w.inb ? (int)code : 1;
#pragma unroll
    for (int m = 1; m < 7; ++m) s_q.y0[(m - 1) * 64 + lane] = y0[m];
    if (nsub > 1) {
        if constexpr (sizeof(R) == 4) {
            // float 7 j + m of the record holds c_{j+1} of state component m
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 *cv = reinterpret_cast<const f4 *>(r + 8);
            f4 v[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] = cv[k];
#pragma unroll
            for (int i = 0; i < 28; ++i)
                if (i % 7 != 0) s_q.c[(kQC * (i / 7) + i % 7 - 1) * 64 + lane] = v[i / 4][i % 4];
        } else {
            double ym[7], y1[7], f0[7], f1[7];
            load_state7(r + 8, ym);
            load_state7(r + kRecDoubles, y1);
            load_state7(r + 16, f0);
            load_state7(r + kRecDoubles + 16, f1);
#pragma unroll
            for (int m = 1; m < 7; ++m) {
                const double A = y1[m] - y0[m] - h * f0[m];
                const double B = h * (f1[m] - f0[m]);
                const double C = 16.0 * (ym[m] - y0[m]) - 8.0 * h * f0[m];
                s_q.c[(m - 1) * 64 + lane] = (R)(h * f0[m]);
                s_q.c[(kQC + m - 1) * 64 + lane] = (R)(-5.0 * A + B + C);
                s_q.c[(2 * kQC + m - 1) * 64 + lane] = (R)(14.0 * A - 3.0 * B - 2.0 * C);
                s_q.c[(3 * kQC + m - 1) * 64 + lane] = (R)(-8.0 * A + 2.0 * B + C);
            }
        }
    }
    w.nsub = nsub;
    w.inv_nsub = 1.0 / (double)nsub;
    w.dl = (R)(fabs(h) * w.inv_nsub);
    w.nrec += nsub;
    w.p = nsub - 1;
    --w.st;
}

// State (t, x, y, z, k_t, k_x, k_y, k_z) at theta of the open step; t is not
// formed (set to 0).
template <typename R>
__device__ __forceinline__ void quartic_at(const QuartLds<R> &s_q, int off, double th, double y[8], double kt) {
    const R t = (R)th;
#pragma unroll
    for (int m = 0; m < kQC; ++m) {
        const int q = m < 3 ? m + 1 : m + 2;
        R v = s_q.c[(3 * kQC + m) * 64 + off];
        v = s_q.c[(2 * kQC + m) * 64 + off] + t * v;
        v = s_q.c[(kQC + m) * 64 + off] + t * v;
        v = s_q.c[m * 64 + off] + t * v;
        y[q] = s_q.y0[m * 64 + off] + th * (double)v;
    }
    y[0] = 0.0;
    y[4] = kt;
}

template <typename R>
__device__ __forceinline__ void to_state_r(const R p6[kQC], R kt, R y[8]) {
    y[0] = R(0); y[1] = p6[0]; y[2] = p6[1]; y[3] = p6[2];
    y[4] = kt; y[5] = p6[3]; y[6] = p6[4]; y[7] = p6[5];
}

// Averaged quantities at a plasma sample (paper section 4.6, Auxiliary
// Images): sums of q dlambda and q dI_j, and <q>_tau relaxed towards q over
// the sample's depth dtau, <q> += (q - <q>)(1 - e^-dtau).
template <typename R>
__device__ __forceinline__ void accumulate_averages(RayWalk<R> &w, const Sample<R> &smp, R dl, R dj, R dtau) {
    const R q[7] = {smp.rho, smp.ne, smp.p, smp.th, smp.B, smp.sigma, smp.binv};
    const R wt = -fexpm1(-dtau);
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        w.av_l[k] += q[k] * dl;
        w.av_j[k] += q[k] * dj;
        w.av_t[k] += (q[k] - w.av_t[k]) * wt;
    }
}

// Process piece w.p of the open step (AVG: the unpolarized walk of the
// averages pass).
template <bool POL, typename R, bool CUTS = false, bool AVG = false, bool NTH = false>
__device__ __forceinline__ void piece(RayWalk<R> &w, const GeoParams &P, const DevGrid &g, const PlasmaParams &pp,
                                      const QuartLds<R> &s_q, int lane) {
    const int flat = P.flat;
    int off = lane;
    asm volatile("" : "+v"(off));   // keep the LDS reads here
    const int p = w.p;
    double ys[8], yb[8];
    if (w.nsub == 1) {
        const double *rr = w.rec + (long long)(w.st + 1) * kRecDoubles + 8;
        ys[0] = rr[0]; ys[1] = rr[1]; ys[2] = rr[2]; ys[3] = rr[3];
        ys[5] = rr[4]; ys[6] = rr[5]; ys[7] = rr[6];
        ys[4] = (double)w.kt;
    } else {
        quartic_at(s_q, off, ((double)p + 0.5) * w.inv_nsub, ys, (double)w.kt);
    }
    if (p == 0) {
#pragma unroll
        for (int m = 0; m < kQC; ++m) yb[m < 3 ? m + 1 : m + 2] = s_q.y0[m * 64 + off];
        yb[0] = 0.0;
        yb[4] = (double)w.kt;
    } else {
        quartic_at(s_q, off, (double)p * w.inv_nsub, yb, (double)w.kt);
    }
    w.p = p - 1;
    Sample<R> smp;
    smp.plasma = false;
    if (w.inb) sample_point<R, CUTS, NTH, POL && sizeof(R) == 8>(P.a, flat, g, pp, ys, (double)w.n_norm, smp, &w.bc);
    R c[8];
    if (smp.plasma) {
        R lt = w.L * w.dl * smp.omega;
        R ljw = fdiv(w.lj * w.dl, smp.omega * smp.omega);
#pragma unroll
        for (int m = 0; m < 3; ++m) c[m] = smp.co[m] * ljw;
#pragma unroll
        for (int m = 3; m < 8; ++m) c[m] = smp.co[m] * lt;
    }
    if (!POL) {
        if (smp.plasma) {
            ++w.nsamp;
            w.I = unpol_segment<R>(w.I, c[0], c[3]);
            csum(w.tau, w.tau_c, c[3]);
            csum(w.Ij, w.Ij_c, c[0]);
            if constexpr (AVG) accumulate_averages(w, smp, w.dl, c[0], c[3]);
        }
        return;
    }
    if (!w.started && !smp.plasma) return;
    const R ktr = (R)w.kt;
    const R ar = (R)P.a;
    bool stk = false;   // a Stokes step at this sample
    if (smp.plasma) {
        ++w.nsamp;
        csum(w.tau, w.tau_c, c[3]);
        csum(w.Ij, w.Ij_c, c[0]);
#pragma unroll
        for (int m = 0; m < 8; ++m) stk = stk || (c[m] != R(0));
    }
    const R dlt = R(0.5) * (w.pdl + w.dl);
    R ya[8], yc[8];
    to_state_r(w.pys, ktr, ya);
    to_state_r(w.pyb, ktr, yc);
    const R kc[4] = {(R)ys[4], (R)ys[5], (R)ys[6], (R)ys[7]};
    R S[4] = {R(0), R(0), R(0), R(0)};
    R e1[4], e2[4], pc[4], qc[4], e3[4];
    // A lane that does a Stokes step here from a packed state (or from
    // nothing, at the first sample of its walk) needs only the screen
    // projection of the transported N.  The choice is the lane's own, so a
    // ray's arithmetic does not depend on the rays that share its wave.
    if (stk && (w.fresh || !w.started)) {
        screen_basis(smp.k, smp.u, kc, smp.b, e1, e2, pc, qc, e3);
        if (w.started) {
            R F[2][4], pt[4], qt[4];
            if (flat) {
#pragma unroll
                for (int m = 0; m < 4; ++m) F[0][m] = F[1][m] = pt[m] = qt[m] = R(0);
            } else {
                ConnF<R> cn;
                conn_geom(ar, flat, ya, ya + 4, cn);
                conn_vec(cn, w.N.r, F[0]);
                conn_vec(cn, w.N.r + 4, F[1]);
                conn_geom(ar, flat, yc, yc + 4, cn);
                conn_covec(cn, pc, pt);
                conn_covec(cn, qc, qt);
            }
            screen_transport_stokes(w.N, F, pt, qt, pc, qc, dlt, S);
        }
    } else {
        if (w.started) {
            if (w.fresh) {
                unpack_screen(w.N);
                w.fresh = false;
            }
            transport_step<R>(ar, flat, ya, yc, dlt, w.N);
        }
        if (stk) {
            screen_basis(smp.k, smp.u, kc, smp.b, e1, e2, pc, qc, e3);
            coh_to_stokes(pc, qc, w.N, S);
        }
    }
    if (stk) {
        if constexpr (NTH && sizeof(R) == 4) stokes_step_nth(c, S);
        else if constexpr (NTH) stokes_step_general(c, S);
        else stokes_step(c, S);
        pack_screen(e1, e2, S, w.N);
        w.fresh = true;
    }
    w.started = true;
#pragma unroll
    for (int m = 0; m < kQC; ++m) {
        w.pys[m] = (R)ys[m < 3 ? m + 1 : m + 2];
        w.pyb[m] = (R)yb[m < 3 ? m + 1 : m + 2];
    }
    w.pdl = w.dl;
}

// Close the ray at the pixel: final half transport, camera Stokes basis.
template <bool POL, typename R>
__device__ __forceinline__ void finish_ray(RayWalk<R> &w, const GeoParams &P, const double upix[4],
                                           const double Hv[4], TransferOut &o) {
    o.tau = (double)w.tau;
    o.Ij = (double)w.Ij;
    o.nsamp = w.nsamp;
    o.nrec = w.nrec;
    o.S[0] = o.S[1] = o.S[2] = o.S[3] = 0.0;
    if (!POL) {
        o.S[0] = (double)w.I;
        return;
    }
    if (!w.started) return;
    if (w.fresh) unpack_screen(w.N);
    const double *rec = w.rec;
    const R ktr = (R)w.kt, ar = (R)P.a;
    R y0[8];
    y0[0] = (R)rec[0]; y0[1] = (R)rec[1]; y0[2] = (R)rec[2]; y0[3] = (R)rec[3];
    y0[4] = ktr; y0[5] = (R)rec[4]; y0[6] = (R)rec[5]; y0[7] = (R)rec[6];
    R ya[8];
    to_state_r(w.pys, ktr, ya);
    transport_step<R>(ar, P.flat, ya, y0, R(0.5) * w.pdl, w.N);
    KS<R> k = ks_point<R>(ar, P.flat, y0[1], y0[2], y0[3]);
    R mH[4] = {(R)-Hv[0], (R)-Hv[1], (R)-Hv[2], (R)-Hv[3]};
    R up[4] = {(R)upix[0], (R)upix[1], (R)upix[2], (R)upix[3]};
    R e1[4], e2[4], p[4], q[4], e3[4];
    screen_basis(k, up, y0 + 4, mH, e1, e2, p, q, e3);
    R S[4];
    coh_to_stokes(p, q, w.N, S);
    for (int m = 0; m < 4; ++m) o.S[m] = (double)S[m];
}

// A polarized ray's state at the end of its walk, handed from the persistent
// transfer kernel to the finishing kernel so that the final transport and
// projection (a few hundred operations for one lane) run converged over all
// rays instead of with the rest of a wave waiting: kRayEnd values of R per ray,
// N (16, packed or full), the previous sample (6), pdl, tau, Ij, k_t, then
// nsamp, nrec, started and the packed flag as integers stored bit for bit.
constexpr int kRayEnd = 32;

template <typename R>
__device__ __forceinline__ int as_int(R v) {
    if constexpr (sizeof(R) == 4) return __builtin_bit_cast(int, v);
    else return (int)__builtin_bit_cast(long long, v);
}
template <typename R>
__device__ __forceinline__ R from_int(int i) {
    if constexpr (sizeof(R) == 4) return __builtin_bit_cast(float, i);
    else return __builtin_bit_cast(double, (long long)i);
}

template <typename R>
__device__ __forceinline__ void store_ray_end(const RayWalk<R> &w, R *e) {
    R v[kRayEnd];
#pragma unroll
    for (int m = 0; m < 10; ++m) v[m] = w.N.r[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) v[10 + m] = w.N.i[m];
#pragma unroll
    for (int m = 0; m < kQC; ++m) v[16 + m] = w.pys[m];
    v[22] = w.pdl;
    v[23] = w.tau;
    v[24] = w.Ij;
    v[25] = w.kt;
    v[26] = from_int<R>(w.nsamp);
    v[27] = from_int<R>(w.nrec);
    v[28] = from_int<R>(w.started ? 1 : 0);
    v[29] = from_int<R>(w.fresh ? 1 : 0);
    v[30] = v[31] = R(0);
    typedef R rv __attribute__((ext_vector_type(16 / sizeof(R))));
    constexpr int NE = 16 / sizeof(R);
    rv *d = reinterpret_cast<rv *>(e);
#pragma unroll
    for (int k = 0; k < kRayEnd / NE; ++k) {
        rv t;
#pragma unroll
        for (int q = 0; q < NE; ++q) t[q] = v[NE * k + q];
        d[k] = t;
    }
}

template <typename R>
__device__ __forceinline__ void load_ray_end(RayWalk<R> &w, const R *e, const double *rec) {
    w.rec = rec;
#pragma unroll
    for (int m = 0; m < 10; ++m) w.N.r[m] = e[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) w.N.i[m] = e[10 + m];
#pragma unroll
    for (int m = 0; m < kQC; ++m) w.pys[m] = e[16 + m];
    w.pdl = e[22];
    w.tau = e[23];
    w.Ij = e[24];
    w.kt = e[25];
    w.nsamp = as_int(e[26]);
    w.nrec = as_int(e[27]);
    w.started = as_int(e[28]) != 0;
    w.fresh = as_int(e[29]) != 0;
}

// The 21 averaged-quantity maps of a finished ray of the averages pass:
// <q>_lambda = sum q dlambda / lambda (lambda the ray's affine length),
// <q>_Ij = sum q dI_j / I_j (0 without emission), <q>_tau.
template <typename R>
__device__ __forceinline__ void write_averages(const RayWalk<R> &w, double lambda, long long NN, long long pix,
                                               double *avg) {
    const double Ij = (double)w.Ij;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        avg[k * NN + pix] = (double)w.av_l[k] / lambda;
        avg[(7 + k) * NN + pix] = Ij > 0.0 ? (double)w.av_j[k] / Ij : 0.0;
        avg[(14 + k) * NN + pix] = (double)w.av_t[k];
    }
}

// Whole ray by one lane (used where rays are not interleaved).
template <bool POL, typename R, bool CUTS = false, bool AVG = false, bool NTH = false>
__device__ __forceinline__ void transfer_ray(const GeoParams &P, const DevGrid &g, const PlasmaParams &pp,
                                             const TransferParams &tp, const double *rec, int n_acc, double kt,
                                             double den, const double upix[4], const double Hv[4],
                                             TransferOut &o, double *avg = nullptr, double lambda = 0.0,
                                             long long NN = 0, long long pix = 0) {
    __shared__ QuartLds<R> s_q;
    const int lane = threadIdx.x;
    RayWalk<R> w;
    begin_ray(w, rec, n_acc, kt, den, tp);
    while (w.st >= 0 || w.p >= 0) {
        if (w.p < 0) next_step(w, s_q, lane);
        piece<POL, R, CUTS, AVG, NTH>(w, P, g, pp, s_q, lane);
    }
    finish_ray<POL, R>(w, P, upix, Hv, o);
    if constexpr (AVG) write_averages(w, lambda, NN, pix, avg);
}

}  // namespace bl
