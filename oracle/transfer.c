/*
 * transfer.c -- radiative-transfer building blocks (oracle).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 *  - eq. (unpolarized): exact segment solution with Delta tau_max = 100;
 *  - eq. (polarized_s): the plasma terms dS/dlambda = J - M S with constant
 *    coefficients, solved exactly as the exponential of the augmented 5x5
 *    matrix [[-M, J], [0, 0]] (scaling and squaring of the Taylor series);
 *  - eq. (polarized_n): the coordinate terms, read as parallel transport of
 *    the rank-2 tensor, dN^ab/dlambda = -k^c (Gamma^a_cd N^db + Gamma^b_cd N^ad)
 *    (the printed minus between the two terms is taken as a typesetting
 *    slip: parallel transport of a tensor carries the same sign on both).
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

double or_unpol_segment(double I, double j, double alpha, double dl)
{
    if (alpha > 0.0) {
        double dtau = alpha * dl;
        if (dtau < 100.0) return exp(-dtau) * (I + expm1(dtau) * j / alpha);
        return j / alpha;
    }
    return I + j * dl;
}

static void matmul5(const double A[5][5], const double B[5][5], double C[5][5])
{
    int i, j, k;
    for (i = 0; i < 5; ++i)
        for (j = 0; j < 5; ++j) {
            double s = 0.0;
            for (k = 0; k < 5; ++k) s += A[i][k] * B[k][j];
            C[i][j] = s;
        }
}

/* exp(A) by scaling and squaring of the Taylor series */
static void expm5(const double A[5][5], double E[5][5])
{
    double X[5][5], T[5][5], P[5][5], nrm = 0.0;
    int i, j, k, sq = 0;
    for (i = 0; i < 5; ++i) {
        double rs = 0.0;
        for (j = 0; j < 5; ++j) rs += fabs(A[i][j]);
        if (rs > nrm) nrm = rs;
    }
    while (nrm > 0.25) { nrm *= 0.5; ++sq; }
    for (i = 0; i < 5; ++i)
        for (j = 0; j < 5; ++j) {
            X[i][j] = ldexp(A[i][j], -sq);
            E[i][j] = (i == j) ? 1.0 : 0.0;
            T[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (k = 1; k <= 30; ++k) {
        matmul5(T, X, P);
        for (i = 0; i < 5; ++i)
            for (j = 0; j < 5; ++j) {
                T[i][j] = P[i][j] / k;
                E[i][j] += T[i][j];
            }
    }
    for (k = 0; k < sq; ++k) {
        matmul5(E, E, P);
        memcpy(E, P, sizeof(P));
    }
}

void or_stokes_exact(const double S0[4], const double J[4], const double M[16],
                     double s, double S1[4])
{
    double A[5][5], E[5][5];
    int i, j;
    memset(A, 0, sizeof(A));
    for (i = 0; i < 4; ++i) {
        for (j = 0; j < 4; ++j) A[i][j] = -M[4 * i + j] * s;
        A[i][4] = J[i] * s;
    }
    expm5(A, E);
    for (i = 0; i < 4; ++i) {
        double v = E[i][4];
        for (j = 0; j < 4; ++j) v += E[i][j] * S0[j];
        S1[i] = v;
    }
}

/* x = M^-1 J by Gaussian elimination with partial pivoting */
void or_solve4(const double M[16], const double J[4], double x[4])
{
    double A[4][5];
    int i, j, k;
    for (i = 0; i < 4; ++i) {
        for (j = 0; j < 4; ++j) A[i][j] = M[4 * i + j];
        A[i][4] = J[i];
    }
    for (k = 0; k < 4; ++k) {
        int piv = k;
        for (i = k + 1; i < 4; ++i)
            if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (piv != k)
            for (j = 0; j < 5; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
        for (i = k + 1; i < 4; ++i) {
            double f = A[i][k] / A[k][k];
            for (j = k; j < 5; ++j) A[i][j] -= f * A[k][j];
        }
    }
    for (i = 3; i >= 0; --i) {
        double s = A[i][4];
        for (j = i + 1; j < 4; ++j) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
}

/* dN/dlambda for the real and imaginary parts of the Hermitian coherency
   tensor N^{ab} at state y (x^a, k_a):
   dN^{ab} = -(G^a_d N^{db} + G^b_d N^{ad}),  G^a_d = Gamma^a_{cd} k^c. */
void or_transport_rhs(double a, int flat, const double y[8],
                      const double Nre[16], const double Nim[16],
                      double dRe[16], double dIm[16])
{
    double g[16], gi[16], gam[64], ku[4], G[16];
    int al, be, ga, de;
    or_metric(a, flat, y, g, gi);
    or_christoffel(a, flat, y, gam);
    for (al = 0; al < 4; ++al) {
        ku[al] = 0.0;
        for (be = 0; be < 4; ++be) ku[al] += gi[4 * al + be] * y[4 + be];
    }
    for (al = 0; al < 4; ++al)
        for (de = 0; de < 4; ++de) {
            double s = 0.0;
            for (ga = 0; ga < 4; ++ga) s += gam[16 * al + 4 * ga + de] * ku[ga];
            G[4 * al + de] = s;
        }
    for (al = 0; al < 4; ++al)
        for (be = 0; be < 4; ++be) {
            double sr = 0.0, si = 0.0;
            for (de = 0; de < 4; ++de) {
                sr += G[4 * al + de] * Nre[4 * de + be] + G[4 * be + de] * Nre[4 * al + de];
                si += G[4 * al + de] * Nim[4 * de + be] + G[4 * be + de] * Nim[4 * al + de];
            }
            dRe[4 * al + be] = -sr;
            dIm[4 * al + be] = -si;
        }
}
