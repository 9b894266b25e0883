// blgpu.hip -- kernels and C ABI of libblgpu (declarations in include/blgpu.h).
//
// Work layout: one ray per lane.  For an image the pixels are processed in
// chunks; per chunk one kernel integrates the geodesics and writes 128-byte
// step records (one cache line each, per-ray contiguous so the backward walk
// of the transfer reads whole lines), then a second kernel walks each ray's
// records from source to camera.  Rays that need more records than the
// per-ray slot holds are queued and finished by a single-wave kernel that
// traces and transfers them one by one with a private record buffer sized
// for max_steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/blgpu.h"
#include "bl_transfer.hpp"
#include "bl_geodesic.hpp"

using namespace bl;

// ============================================================ camera frame
// Camera frame of the paper's section 2.1 (single lane, once per image):
// centre from spherical KS, covariant k_a = (J^-1)^i_a k_i, k_t from the null
// condition (future directed), camera-frame metric g_a'b' and g^a'b', K from
// k_a - (u_a/u_t) k_t normalised by g^a'b', v from U = z (y on the polar
// axis) by Gram-Schmidt, h = D^-1/2 [abc] v_b' K_c', rotation by psi, and the
// return to coordinate components A^t = u^t A^t' - (u_a/u_t) A^a',
// A^a = A^a' + u^a A^t'.  One block per image, the frame of image b is
// written into B.imgs[b].fr.
__global__ void k_camera_frame(Batch bt) {
    if (threadIdx.x != 0 || (int)blockIdx.x >= bt.n_img) return;
    ImgDev &im = bt.imgs[blockIdx.x];
    const CamParams cp = im.cp;
    const double a = im.a;
    const int flat = im.flat;
    Frame fr;
    double st = sin(cp.theta), ct = cos(cp.theta), sp = sin(cp.phi), cph = cos(cp.phi);
    double r = cp.r;
    fr.xc[0] = 0.0;
    fr.xc[1] = st * (r * cph - a * sp);
    fr.xc[2] = st * (r * sp + a * cph);
    fr.xc[3] = r * ct;
    double J[3][3] = {{st * cph, ct * (r * cph - a * sp), st * (-r * sp - a * cph)},
                      {st * sp, ct * (r * sp + a * cph), st * (r * cph - a * sp)},
                      {ct, -r * st, 0.0}};
#pragma unroll
    for (int i = 0; i < 3; ++i) fr.ut[i] = J[i][0] * cp.u_normal[0] + J[i][1] * cp.u_normal[1] + J[i][2] * cp.u_normal[2];
    // covariant spatial k: solve J^T k = k_sph
    double kl[4];
    if (st != 0.0) {
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = J[j][i];
        double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                     M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        for (int c = 0; c < 3; ++c) {
            double T[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) T[i][j] = (j == c) ? cp.k_cov[i] : M[i][j];
            kl[1 + c] = (T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1]) - T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0]) +
                         T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0])) / det;
        }
    } else {
        double w0 = J[0][1], w1 = J[1][1], ww = w0 * w0 + w1 * w1;
        kl[3] = cp.k_cov[0] / J[2][0];
        kl[1] = ww > 0.0 ? cp.k_cov[1] * w0 / ww : 0.0;
        kl[2] = ww > 0.0 ? cp.k_cov[1] * w1 / ww : 0.0;
    }
    auto k = ks_point(a, flat, fr.xc[1], fr.xc[2], fr.xc[3]);
    double g[4][4], gi[4][4];
    double ll[4] = {1.0, k.l[0], k.l[1], k.l[2]}, lu[4] = {-1.0, k.l[0], k.l[1], k.l[2]};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double eta = (i == j) ? (i == 0 ? -1.0 : 1.0) : 0.0;
            g[i][j] = eta + k.f * ll[i] * ll[j];
            gi[i][j] = eta - k.f * lu[i] * lu[j];
        }
    velocity_from_normal(k, fr.ut, fr.u);
    double ul[4];
    lower(k, fr.u, ul);
    double A = gi[0][0], B = gi[0][1] * kl[1] + gi[0][2] * kl[2] + gi[0][3] * kl[3], C = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C += gi[1 + i][1 + j] * kl[1 + i] * kl[1 + j];
    kl[0] = (-B + sqrt(B * B - A * C)) / A;
    double gp[3][3], gpi[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            gp[i][j] = g[1 + i][1 + j] - ul[1 + i] / ul[0] * g[0][1 + j] - ul[1 + j] / ul[0] * g[0][1 + i] +
                       ul[1 + i] * ul[1 + j] * g[0][0] / (ul[0] * ul[0]);
            gpi[i][j] = gi[1 + i][1 + j] + fr.u[1 + i] * fr.u[1 + j];
        }
    double Kl[3], Ku[3], Kt = 0.0, nrm = 0.0;
    for (int i = 0; i < 3; ++i) Kl[i] = kl[1 + i] - ul[1 + i] / ul[0] * kl[0];
    for (int i = 0; i < 4; ++i) Kt -= fr.u[i] * kl[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nrm += gpi[i][j] * Kl[i] * Kl[j];
    nrm = 1.0 / sqrt(nrm);
    for (int i = 0; i < 3; ++i) Kl[i] *= nrm;
    Kt *= nrm;
    for (int i = 0; i < 3; ++i) Ku[i] = gpi[i][0] * Kl[0] + gpi[i][1] * Kl[1] + gpi[i][2] * Kl[2];
    double U[3] = {0.0, 0.0, 1.0};
    if (fr.xc[1] == 0.0 && fr.xc[2] == 0.0) {
        U[1] = 1.0;
        U[2] = 0.0;
    }
    double UK = U[0] * Kl[0] + U[1] * Kl[1] + U[2] * Kl[2];
    double vu[3], vl[3];
    for (int i = 0; i < 3; ++i) vu[i] = U[i] - UK * Ku[i];
    for (int i = 0; i < 3; ++i) vl[i] = gp[i][0] * vu[0] + gp[i][1] * vu[1] + gp[i][2] * vu[2];
    nrm = 1.0 / sqrt(vl[0] * vu[0] + vl[1] * vu[1] + vl[2] * vu[2]);
    for (int i = 0; i < 3; ++i) {
        vu[i] *= nrm;
        vl[i] *= nrm;
    }
    double D = gp[0][0] * (gp[1][1] * gp[2][2] - gp[1][2] * gp[2][1]) - gp[0][1] * (gp[1][0] * gp[2][2] - gp[1][2] * gp[2][0]) +
               gp[0][2] * (gp[1][0] * gp[2][1] - gp[1][1] * gp[2][0]);
    double isd = 1.0 / sqrt(D);
    double hu[3] = {(vl[1] * Kl[2] - vl[2] * Kl[1]) * isd, (vl[2] * Kl[0] - vl[0] * Kl[2]) * isd,
                    (vl[0] * Kl[1] - vl[1] * Kl[0]) * isd};
    double cps = cos(cp.psi), sps = sin(cp.psi);
    double Hp[3], Vp[3];
    for (int i = 0; i < 3; ++i) {
        Hp[i] = hu[i] * cps - vu[i] * sps;
        Vp[i] = vu[i] * cps + hu[i] * sps;
    }
    fr.K[0] = fr.u[0] * Kt;
    fr.H[0] = 0.0;
    fr.V[0] = 0.0;
    for (int b = 0; b < 3; ++b) {
        fr.K[0] -= ul[1 + b] / ul[0] * Ku[b];
        fr.H[0] -= ul[1 + b] / ul[0] * Hp[b];
        fr.V[0] -= ul[1 + b] / ul[0] * Vp[b];
    }
    for (int i = 0; i < 3; ++i) {
        fr.K[1 + i] = Ku[i] + fr.u[1 + i] * Kt;
        fr.H[1 + i] = Hp[i];
        fr.V[1 + i] = Vp[i];
    }
    fr.pad = 0.0;
    im.fr = fr;
}

__global__ void k_camera_rays(const ImgDev *__restrict__ imp, double *__restrict__ state_out,
                              double *__restrict__ norm_out) {
    const ImgDev &im = *imp;
    const CamParams &cp = im.cp;
    long long NN = (long long)cp.n * cp.n;
    long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= NN) return;
    double y[8], den;
    camera_pixel(im.fr, cp, im.a, im.flat, (int)(pix % cp.n), (int)(pix / cp.n), y, den);
    for (int m = 0; m < 8; ++m) state_out[pix * 8 + m] = y[m];
    norm_out[pix] = cp.nu / den;
}

__global__ void k_fill_int(int *p, int v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ============================================================ geodesics
// Per-image parameters of a lane: in a batch they are read from the image's
// descriptor, for a single image the kernel arguments already hold them.
template <bool BATCH>
__device__ __forceinline__ GeoParams lane_params(const GeoParams &P, const ImgDev &im) {
    if (!BATCH) return P;
    GeoParams Q = P;
    Q.a = im.a;
    Q.r_in = im.r_in;
    Q.r_cam = im.cp.r;
    Q.flat = im.flat;
    Q.n = im.cp.n;
    return Q;
}

// One lane per ray id of the chunk [start, start + count).  With WREC the step
// records are written into the lane's slot (moving to an extension slot of X
// when it fills); rays that outgrow that too are queued on ovf_list; ids of
// tile pixels outside their image get nacc = -2.
template <bool WREC, bool BATCH>
__global__ void __launch_bounds__(64, 2) k_geodesic(GeoParams P, Batch B, long long start, int count,
                                                 double *__restrict__ rec, double *__restrict__ meta,
                                                 int *__restrict__ nacc_out, int *__restrict__ work_out, ExtQueue X,
                                                 int *__restrict__ ovf_count,
                                                 int *__restrict__ ovf_list, double *__restrict__ state_out) {
    int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= count) return;
    const long long gid = start + slot;
    const int img = BATCH ? find_image(B, gid) : 0;
    const ImgDev &im = B.imgs[img];
    int pi, pj;
    if (!ray_pixel(B, im.cp.n, gid - (BATCH ? B.ray0[img] : 0), pi, pj)) {
        if (WREC) nacc_out[slot] = work_out[slot] = -2;
        return;
    }
    const GeoParams Q = lane_params<BATCH>(P, im);
    const long long NN = (long long)im.cp.n * im.cp.n;
    const long long pix = (long long)pj * im.cp.n + pi;
    double *aux = im.aux;
    double y8[8], den;
    camera_pixel(im.fr, im.cp, Q.a, Q.flat, pi, pj, y8, den);
    double y[7] = {y8[0], y8[1], y8[2], y8[3], y8[5], y8[6], y8[7]};
    double kt = y8[4];
    TraceOut o;
    trace_ray<WREC>(Q, y, kt, WREC ? rec + (long long)slot * Q.cap * kRecDoubles : nullptr, Q.cap, o,
                    StepLog{nullptr, 0, nullptr}, &X, slot);
    if (WREC) {
        meta[2 * slot] = kt;
        meta[2 * slot + 1] = den;
        if (o.status == kRayOverflow) {
            nacc_out[slot] = work_out[slot] = -1;
            int idx = atomicAdd(ovf_count, 1);
            ovf_list[idx] = (int)gid;
            return;
        }
        nacc_out[slot] = o.n_acc;
        work_out[slot] = o.work;
    }
    aux[BL_AUX_DT * NN + pix] = o.dt;
    aux[BL_AUX_S * NN + pix] = o.s;
    aux[BL_AUX_LAMBDA * NN + pix] = o.lambda;
    aux[BL_AUX_NACC * NN + pix] = (double)o.n_acc;
    aux[BL_AUX_NREJ * NN + pix] = (double)o.n_rej;
    aux[BL_AUX_STATUS * NN + pix] = (double)o.status;
    if (!WREC) {
        aux[BL_AUX_TAU * NN + pix] = 0.0;
        aux[BL_AUX_IJ * NN + pix] = 0.0;
        aux[BL_AUX_NSAMP * NN + pix] = 0.0;
        aux[BL_AUX_NREC * NN + pix] = 0.0;
        if (state_out) {
            state_out[pix * 8 + 0] = y[0];
            state_out[pix * 8 + 1] = y[1];
            state_out[pix * 8 + 2] = y[2];
            state_out[pix * 8 + 3] = y[3];
            state_out[pix * 8 + 4] = kt;
            state_out[pix * 8 + 5] = y[4];
            state_out[pix * 8 + 6] = y[5];
            state_out[pix * 8 + 7] = y[6];
        }
    }
}

// Transfer results are already in camera units (I_nu = nu^3 I).
__device__ __forceinline__ void write_pixel(const TransferOut &t, long long NN, long long pix, double *image,
                                            double *aux) {
    for (int q = 0; q < 4; ++q) image[q * NN + pix] = t.S[q];
    aux[BL_AUX_TAU * NN + pix] = t.tau;
    aux[BL_AUX_IJ * NN + pix] = t.Ij;
    aux[BL_AUX_NSAMP * NN + pix] = (double)t.nsamp;
    aux[BL_AUX_NREC * NN + pix] = (double)t.nrec;
}

__device__ __forceinline__ void pixel_observer(const Frame &fr, const GeoParams &P, const double *rec0, double upix[4]) {
    auto k = ks_point(P.a, P.flat, rec0[1], rec0[2], rec0[3]);
    velocity_from_normal(k, fr.ut, upix);
}

// Persistent transfer: each wave keeps its 64 lanes busy by giving a lane
// that finished its ray the next ray of the chunk (one atomic per wave for all
// lanes that need one), so the per-piece work always runs on full waves even
// though rays hold from tens to thousands of pieces.  A wave takes new rays
// once at least refill_min lanes are idle, or when none holds a ray.  Every
// lane leaves the loop once the queue is exhausted and its ray is written.
// ------------------------------------------------------------- ray order
// The transfer takes the rays of a chunk longest first, by the number of
// walk iterations the geodesic kernel counted for each (the pieces of the
// steps from the last sampled one to the camera), so that the few very long
// rays near the photon ring start early and their serial walks overlap the
// bulk instead of trailing it: a counting sort on kOrderBins bins of
// work / 32 (the last bin open-ended), in descending bin order.  Each block
// of 256 rays counts and ranks its rays in LDS and makes one global atomic
// per non-empty bin.  Slots without a ray for the transfer (work < 0) go
// last.  The order within a bin is not deterministic; results do not depend
// on it.
constexpr int kOrderBins = 64;

__device__ __forceinline__ int order_key(int work) { return work < 0 ? 0 : min(work >> 5, kOrderBins - 1); }

__global__ void __launch_bounds__(256) k_order_hist(const int *__restrict__ work, int count, int *__restrict__ hist) {
    __shared__ int lh[kOrderBins];
    if (threadIdx.x < kOrderBins) lh[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) atomicAdd(lh + order_key(work[i]), 1);
    __syncthreads();
    if (threadIdx.x < kOrderBins && lh[threadIdx.x]) atomicAdd(hist + threadIdx.x, lh[threadIdx.x]);
}

// Exclusive offsets in descending bin order (one block of kOrderBins threads).
__global__ void __launch_bounds__(kOrderBins) k_order_scan(int *__restrict__ hist) {
    __shared__ int sc[kOrderBins];
    const int t = threadIdx.x;
    const int key = kOrderBins - 1 - t;   // position t in descending order
    const int own = hist[key];
    sc[t] = own;
    __syncthreads();
    for (int off = 1; off < kOrderBins; off <<= 1) {
        int v = t >= off ? sc[t - off] : 0;
        __syncthreads();
        sc[t] += v;
        __syncthreads();
    }
    hist[key] = sc[t] - own;
}

__global__ void __launch_bounds__(256) k_order_scatter(const int *__restrict__ work, int count, int *__restrict__ offs,
                                                       int *__restrict__ order) {
    __shared__ int lh[kOrderBins], lb[kOrderBins];
    if (threadIdx.x < kOrderBins) lh[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int key = i < count ? order_key(work[i]) : 0;
    const int rank = i < count ? atomicAdd(lh + key, 1) : 0;
    __syncthreads();
    if (threadIdx.x < kOrderBins) lb[threadIdx.x] = lh[threadIdx.x] ? atomicAdd(offs + threadIdx.x, lh[threadIdx.x]) : 0;
    __syncthreads();
    if (i < count) order[lb[key] + rank] = i;
}

// Resident waves per SIMD the transfer kernels are compiled for (the register
// budget: 168 VGPRs for three, 128 for four, 256 for two); the polarized FP64
// kernel keeps the compiler's choice (one).
template <bool POL, typename R, bool AVG>
constexpr int transfer_waves() { return sizeof(R) == 4 ? (POL || AVG ? 3 : 4) : (POL ? 1 : 2); }

template <bool POL, typename R, bool BATCH, bool CUTS, bool AVG = false, bool NTH = false>
__global__ void __launch_bounds__(64, (transfer_waves<POL, R, AVG>())) k_transfer(GeoParams P, Batch B, DevGrid g,
                                                                             PlasmaParams pp, TransferParams tp,
                                                 long long start, int count, int refill_min,
                                                 const double *__restrict__ rec, const double *__restrict__ meta,
                                                 const int *__restrict__ nacc, const int *__restrict__ order,
                                                 ExtQueue X, int *__restrict__ queue, R *__restrict__ ends) {
    __shared__ QuartLds<R> s_q;
    const int lane = threadIdx.x;
    RayWalk<R> w;
    int slot = -1, img = 0;
    double a_l = P.a;
    int flat_l = P.flat;
    bool done = false;
    for (;;) {
        unsigned long long need = __ballot(slot < 0 && !done);
        if (need && (__popcll(need) >= refill_min || __ballot(slot >= 0) == 0)) {
            int leader = __ffsll((long long)need) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(queue, __popcll(need));
            base = __shfl(base, leader);
            if (slot < 0 && !done) {
                const int pos = base + __popcll(need & ((1ull << lane) - 1ull));
                if (pos >= count) {
                    done = true;
                } else {
                    const int id = order[pos];
                    int na = nacc[id];
                    if (na >= 0) {   // -1: finished by the overflow kernel, -2: no pixel
                        slot = id;
                        TransferParams tl = tp;
                        if (BATCH) {
                            img = find_image(B, start + id);
                            const ImgDev &im = B.imgs[img];
                            a_l = im.a;
                            flat_l = im.flat;
                            tl.L = im.L;
                            tl.nu_cam = im.cp.nu;
                        }
                        const int e = X.of[id];
                        const double *rp = e >= 0 ? X.rec + (long long)e * X.cap_rec * kRecDoubles
                                                  : rec + (long long)id * P.cap * kRecDoubles;
                        begin_ray(w, rp, na, meta[2 * id], meta[2 * id + 1], tl);
                    }
                }
            }
        }
        if (__ballot(slot >= 0 || !done) == 0) break;
        GeoParams Pl = P;
        if (BATCH) {
            Pl.a = a_l;
            Pl.flat = flat_l;
        }
        if (slot >= 0 && w.p < 0) {
            if (w.st < 0 && POL) {
                // finished by k_finish
                store_ray_end(w, ends + (long long)slot * kRayEnd);
                slot = -1;
            } else if (w.st < 0) {
                const ImgDev &im = B.imgs[img];
                const long long gid = start + slot;
                int pi = 0, pj = 0;
                ray_pixel(B, im.cp.n, gid - (BATCH ? B.ray0[img] : 0), pi, pj);
                double upix[4];
                pixel_observer(im.fr, Pl, w.rec, upix);
                TransferOut t;
                finish_ray<POL, R>(w, Pl, upix, im.fr.H, t);
                const long long NN = (long long)im.cp.n * im.cp.n, pix = (long long)pj * im.cp.n + pi;
                if constexpr (AVG) write_averages(w, im.aux[BL_AUX_LAMBDA * NN + pix], NN, pix, im.avg);
                else write_pixel(t, NN, pix, im.image, im.aux);
                slot = -1;
            } else {
                next_step(w, s_q, lane);
            }
        }
        if (slot >= 0) piece<POL, R, CUTS, AVG, NTH>(w, Pl, g, pp, s_q, lane);
    }
}

// Final transport to the pixel and projection on the camera's Stokes basis
// for the polarized rays of a chunk, from the end states the transfer kernel
// stored (one lane per ray slot).
template <typename R, bool BATCH>
__global__ void __launch_bounds__(64) k_finish(GeoParams P, Batch B, long long start, int count,
                                               const double *__restrict__ rec, const int *__restrict__ nacc,
                                               ExtQueue X, const R *__restrict__ ends) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= count || nacc[id] < 0) return;   // -1: finished by the overflow kernel, -2: no pixel
    const int img = BATCH ? find_image(B, start + id) : 0;
    const ImgDev &im = B.imgs[img];
    GeoParams Pl = P;
    if (BATCH) {
        Pl.a = im.a;
        Pl.flat = im.flat;
    }
    const int e = X.of[id];
    const double *rp = e >= 0 ? X.rec + (long long)e * X.cap_rec * kRecDoubles : rec + (long long)id * P.cap * kRecDoubles;
    RayWalk<R> w;
    load_ray_end(w, ends + (long long)id * kRayEnd, rp);
    int pi = 0, pj = 0;
    ray_pixel(B, im.cp.n, start + id - (BATCH ? B.ray0[img] : 0), pi, pj);
    double upix[4];
    pixel_observer(im.fr, Pl, rp, upix);
    TransferOut t;
    finish_ray<true, R>(w, Pl, upix, im.fr.H, t);
    write_pixel(t, (long long)im.cp.n * im.cp.n, (long long)pj * im.cp.n + pi, im.image, im.aux);
}

// Rays queued by k_geodesic: one wave, each lane traces and transfers its
// rays in turn with a private buffer of big_cap records.
template <bool POL, typename R, bool CUTS, bool AVG = false, bool NTH = false>
__global__ void __launch_bounds__(64) k_overflow(GeoParams P, Batch B, DevGrid g, PlasmaParams pp, TransferParams tp,
                                                 const int *__restrict__ ovf_count, const int *__restrict__ ovf_list,
                                                 double *__restrict__ big_rec, int big_cap) {
    int lane = threadIdx.x;
    int total = *ovf_count;
    double *r = big_rec + (long long)lane * big_cap * kRecDoubles;
    for (int idx = lane; idx < total; idx += blockDim.x) {
        const long long gid = ovf_list[idx];
        const int img = find_image(B, gid);
        const ImgDev &im = B.imgs[img];
        int pi, pj;
        ray_pixel(B, im.cp.n, gid - B.ray0[img], pi, pj);
        GeoParams Q = lane_params<true>(P, im);
        Q.cap = big_cap;
        TransferParams tl = tp;
        tl.L = im.L;
        tl.nu_cam = im.cp.nu;
        const long long NN = (long long)im.cp.n * im.cp.n, pix = (long long)pj * im.cp.n + pi;
        double *aux = im.aux;
        double y8[8], den;
        camera_pixel(im.fr, im.cp, Q.a, Q.flat, pi, pj, y8, den);
        double y[7] = {y8[0], y8[1], y8[2], y8[3], y8[5], y8[6], y8[7]};
        double kt = y8[4];
        TraceOut o;
        trace_ray<true>(Q, y, kt, r, big_cap, o);
        double upix[4];
        pixel_observer(im.fr, Q, r, upix);
        TransferOut t;
        if constexpr (AVG) {
            transfer_ray<POL, R, CUTS, true>(Q, g, pp, tl, r, o.n_acc, kt, den, upix, im.fr.H, t, im.avg, o.lambda,
                                             NN, pix);
        } else {
            aux[BL_AUX_DT * NN + pix] = o.dt;
            aux[BL_AUX_S * NN + pix] = o.s;
            aux[BL_AUX_LAMBDA * NN + pix] = o.lambda;
            aux[BL_AUX_NACC * NN + pix] = (double)o.n_acc;
            aux[BL_AUX_NREJ * NN + pix] = (double)o.n_rej;
            aux[BL_AUX_STATUS * NN + pix] = (double)o.status;
            transfer_ray<POL, R, CUTS, false, NTH>(Q, g, pp, tl, r, o.n_acc, kt, den, upix, im.fr.H, t);
            write_pixel(t, NN, pix, im.image, aux);
        }
    }
}

// ============================================================ learned step
// Geodesics with learned step proposals: blocks of four waves share the
// packed network (forward fragments and FP32 tail) in LDS; each wave has its
// own staging rows.  Lanes without a ray still take part in the network calls.
template <bool WREC, bool BATCH>
__global__ void __launch_bounds__(256, 2) k_geodesic_learned(GeoParams P, Batch B, long long start, int count,
                                                          const u32x4 *__restrict__ pk_g,
                                                          const float *__restrict__ tail_g, double *__restrict__ rec,
                                                          double *__restrict__ meta, int *__restrict__ nacc_out,
                                                          int *__restrict__ work_out, ExtQueue X,
                                                          int *__restrict__ ovf_count,
                                                          int *__restrict__ ovf_list) {
    __shared__ u32x4 s_pk[kPkFwd];
    __shared__ float s_tail[kTailN];
    __shared__ u32x4 s_stage[4][64 * 4];
    for (int i = threadIdx.x; i < kPkFwd; i += blockDim.x) s_pk[i] = pk_g[i];
    for (int i = threadIdx.x; i < kTailN; i += blockDim.x) s_tail[i] = tail_g[i];
    __syncthreads();
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    const long long gid = start + slot;
    bool active = slot < count;
    int img = 0, pi = 0, pj = 0;
    if (active) {
        img = BATCH ? find_image(B, gid) : 0;
        active = ray_pixel(B, B.imgs[img].cp.n, gid - (BATCH ? B.ray0[img] : 0), pi, pj);
        if (!active && WREC) nacc_out[slot] = work_out[slot] = -2;
    }
    const ImgDev &im = B.imgs[img];
    const GeoParams Q = lane_params<BATCH>(P, im);
    double y8[8] = {0, 0, 0, 0, -1, 0, 0, 0}, den = 1.0;
    if (active) camera_pixel(im.fr, im.cp, Q.a, Q.flat, pi, pj, y8, den);
    double y[7] = {y8[0], y8[1], y8[2], y8[3], y8[5], y8[6], y8[7]};
    const double kt = y8[4];
    TraceOut o;
    trace_ray_learned<WREC>(Q, active, y, kt, WREC && active ? rec + (long long)slot * Q.cap * kRecDoubles : nullptr,
                            Q.cap, o, s_pk, s_tail, s_stage[threadIdx.x >> 6], &X, slot);
    if (!active) return;
    const long long NN = (long long)im.cp.n * im.cp.n, pix = (long long)pj * im.cp.n + pi;
    double *aux = im.aux;
    if (WREC) {
        meta[2 * slot] = kt;
        meta[2 * slot + 1] = den;
        if (o.status == kRayOverflow) {
            nacc_out[slot] = work_out[slot] = -1;
            int idx = atomicAdd(ovf_count, 1);
            ovf_list[idx] = (int)gid;
            return;
        }
        nacc_out[slot] = o.n_acc;
        work_out[slot] = o.work;
    }
    aux[BL_AUX_DT * NN + pix] = o.dt;
    aux[BL_AUX_S * NN + pix] = o.s;
    aux[BL_AUX_LAMBDA * NN + pix] = o.lambda;
    aux[BL_AUX_NACC * NN + pix] = (double)o.n_acc;
    aux[BL_AUX_NREJ * NN + pix] = (double)o.n_rej;
    aux[BL_AUX_STATUS * NN + pix] = (double)o.status;
}

// Step log of the plain integrator over the rays of a batch (no records);
// geodesic auxiliary maps are written as by bl_trace_geodesics.
__global__ void __launch_bounds__(64) k_steplog(GeoParams P, Batch B, long long start, int count, StepLog lg) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= count) return;
    const long long gid = start + slot;
    const int img = find_image(B, gid);
    const ImgDev &im = B.imgs[img];
    int pi, pj;
    if (!ray_pixel(B, im.cp.n, gid - B.ray0[img], pi, pj)) return;
    const GeoParams Q = lane_params<true>(P, im);
    double y8[8], den;
    camera_pixel(im.fr, im.cp, Q.a, Q.flat, pi, pj, y8, den);
    double y[7] = {y8[0], y8[1], y8[2], y8[3], y8[5], y8[6], y8[7]};
    TraceOut o;
    trace_ray<false, true>(Q, y, y8[4], nullptr, 0, o, lg);
    const long long NN = (long long)im.cp.n * im.cp.n, pix = (long long)pj * im.cp.n + pi;
    double *aux = im.aux;
    aux[BL_AUX_DT * NN + pix] = o.dt;
    aux[BL_AUX_S * NN + pix] = o.s;
    aux[BL_AUX_LAMBDA * NN + pix] = o.lambda;
    aux[BL_AUX_TAU * NN + pix] = 0.0;
    aux[BL_AUX_IJ * NN + pix] = 0.0;
    aux[BL_AUX_NACC * NN + pix] = (double)o.n_acc;
    aux[BL_AUX_NREJ * NN + pix] = (double)o.n_rej;
    aux[BL_AUX_STATUS * NN + pix] = (double)o.status;
    aux[BL_AUX_NSAMP * NN + pix] = 0.0;
    aux[BL_AUX_NREC * NN + pix] = 0.0;
}

// ------------------------------------------------------------- the network
// Packed A-operand fragments and the FP32 tail from the FP32 model.
__global__ void k_mlp_pack(const float *__restrict__ model, u32x4 *__restrict__ pk, float *__restrict__ tail) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kPkAll) {
        const int lane = t & 63, slot = t >> 6, g = lane >> 4, i = lane & 15;
        float v[8];
        for (int e = 0; e < 8; ++e) {
            if (slot < 4) {   // forward layer 1: W1[16 mt + i][8 g + e]
                const int k = 8 * g + e;
                v[e] = k < kMlpIn ? model[kW1 + (16 * slot + i) * kMlpIn + k] : 0.0f;
            } else {
                const int q = (slot - 4) % 8, mt = q / 2, kk = q % 2, k = hid_k(kk, g, e), u = 16 * mt + i;
                const int base = slot < 12 ? kW2 : slot < 20 ? kW3 : slot < 28 ? kW2 : kW3;
                v[e] = slot < 20 ? model[base + u * kMlpH + k]      // forward: W[u][k]
                                 : model[base + k * kMlpH + u];     // backward: W^T[u][k] = W[k][u]
            }
        }
        pk[t] = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
    }
    if (t < kTailN) {
        float v = 0.0f;
        if (t < 64) v = model[kB1 + t];
        else if (t < 128) v = model[kB2 + t - 64];
        else if (t < 192) v = model[kB3 + t - 128];
        else if (t < 256) v = model[kW4 + t - 192];
        else if (t == kTB4) v = model[kB4];
        else if (t < kTISig) v = model[kMu + t - kTMu];
        else if (t < kTISig + kMlpIn) v = 1.0f / model[kSig + t - kTISig];
        tail[t] = v;
    }
}

// Per-block sums and sums of squares (double) of the 12 record columns.
__global__ void __launch_bounds__(256) k_mlp_stats(const float *__restrict__ rec, long long n,
                                                   double *__restrict__ part) {
    __shared__ double sh[256][2];
    for (int c = 0; c < kLogRec; ++c) {
        double s = 0.0, q = 0.0;
        for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (long long)gridDim.x * blockDim.x) {
            double v = rec[r * kLogRec + c];
            s += v;
            q += v * v;
        }
        sh[threadIdx.x][0] = s;
        sh[threadIdx.x][1] = q;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                sh[threadIdx.x][0] += sh[threadIdx.x + w][0];
                sh[threadIdx.x][1] += sh[threadIdx.x + w][1];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[(blockIdx.x * kLogRec + c) * 2] = sh[0][0];
            part[(blockIdx.x * kLogRec + c) * 2 + 1] = sh[0][1];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double splitmix_u01(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

// Initial model: feature mean and standard deviation from the statistics
// (fixed summation order), LeCun-uniform weights U(-sqrt(3/fan_in),
// sqrt(3/fan_in)) from a counter-based generator, zero hidden biases and the
// output bias at the mean target.
__global__ void k_mlp_init(const double *__restrict__ part, int nblk, long long n, unsigned long long seed,
                           float *__restrict__ model) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kMlpNModel) return;
    auto col = [&](int c, double &mean, double &sd) {
        double s = 0.0, q = 0.0;
        for (int b = 0; b < nblk; ++b) {
            s += part[(b * kLogRec + c) * 2];
            q += part[(b * kLogRec + c) * 2 + 1];
        }
        mean = s / (double)n;
        double var = fmax(0.0, q / (double)n - mean * mean);
        sd = sqrt(var);
        if (!(sd > 1e-6 * (1.0 + fabs(mean)))) sd = 1.0;
    };
    float v = 0.0f;
    if (t >= kMu) {
        double m, sd;
        col((t - kMu) % kMlpIn, m, sd);
        v = (float)(t < kSig ? m : sd);
    } else if (t == kB4) {
        double m, sd;
        col(kMlpIn, m, sd);
        v = (float)m;
    } else {
        int fan = 0;
        if (t < kB1) fan = kMlpIn;
        else if ((t >= kW2 && t < kB2) || (t >= kW3 && t < kB3) || (t >= kW4 && t < kB4)) fan = kMlpH;
        if (fan) v = (float)((2.0 * splitmix_u01(seed * 0x100000001B3ull + (unsigned long long)t) - 1.0) *
                             sqrt(3.0 / fan));
    }
    model[t] = v;
}

// Forward and backward pass over tiles of 64 records, one tile per wave:
// rows r = tile 64 + lane < n_rows are records idx(r) = (mul (offset + r) +
// add) mod n_mod (an affine permutation of the training set; mul = 1, add =
// 0 for the plain order).  Writes the per-tile partial gradient of
// sum (y - target)^2 * inv_n (all kMlpNParam entries) and the per-tile
// partial sum of (y - target)^2; y_out (optional) receives the outputs.
// BF16 operands on the matrix cores: normalised inputs, weights, hidden
// activations and backpropagated pre-activation gradients; everything else
// FP32.
__global__ void __launch_bounds__(64) k_mlp_fwdbwd(const u32x4 *__restrict__ pk, const float *__restrict__ tail,
                                                   const float *__restrict__ rec, long long n_rows, long long offset,
                                                   long long mul, long long add, long long n_mod, float inv_n,
                                                   int want_grad, float *__restrict__ grad_part,
                                                   float *__restrict__ loss_part, float *__restrict__ y_out) {
    __shared__ u32x4 s_stage[64 * 4];
    __shared__ __attribute__((aligned(16))) unsigned short s_xt[32 * 64];       // inputs, [feature][ray]
    __shared__ __attribute__((aligned(16))) unsigned short s_h1[64 * 64];       // BF16 h1, [unit][ray]
    __shared__ __attribute__((aligned(16))) unsigned short s_h2[64 * 64];
    __shared__ __attribute__((aligned(16))) unsigned short s_dz[64 * 64];       // BF16 dz of the current layer, [unit][ray]
    __shared__ f32x4 s_z1[16 * 64], s_z2[16 * 64], s_z3[16 * 64]; // pre-activations, [mt * 4 + nt][lane]
    const int lane = threadIdx.x, g = lane >> 4, j = lane & 15;
    const long long row = (long long)blockIdx.x * 64 + lane;
    const bool valid = row < n_rows;
    float x[kMlpIn], target = 0.0f;
    if (valid) {
        const long long idx = (long long)(((unsigned long long)mul * (unsigned long long)(offset + row) + (unsigned long long)add) %
                                          (unsigned long long)n_mod);
        const float *q = rec + idx * kLogRec;
        #pragma unroll
        for (int m = 0; m < kMlpIn; ++m) x[m] = q[m];
        target = q[kMlpIn];
    } else {
        #pragma unroll
        for (int m = 0; m < kMlpIn; ++m) x[m] = tail[kTMu + m];
    }
    // ---- forward
    stage_input(tail, x, s_stage, lane);
    #pragma unroll
    for (int f = 0; f < 32; ++f)
        s_xt[f * 64 + lane] = f < kMlpIn ? (unsigned short)(pack2((x[f] - tail[kTMu + f]) * tail[kTISig + f], 0.0f) & 0xffffu) : 0;
    wave_lds_sync();
    u32x4 b1[4][1];
    input_bfrag(s_stage, b1, lane);
    f32x4 h[4][4];
    u32x4 bq[4][2];
    mm_layer<1>(pk + kPkL1, b1, h, lane);
    #pragma unroll
    for (int L = 1; L <= 3; ++L) {
        const float *bias = tail + (L == 1 ? kTB1 : L == 2 ? kTB2 : kTB3);
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float bb = bias[16 * mt + 4 * g + e];
                #pragma unroll
                for (int nt = 0; nt < 4; ++nt) h[mt][nt][e] += bb;
            }
        if (L < 3) {
            f32x4 *zs = L == 1 ? s_z1 : s_z2;
            unsigned short *hs = L == 1 ? s_h1 : s_h2;
            #pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                #pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    zs[(mt * 4 + nt) * 64 + lane] = h[mt][nt];
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        h[mt][nt][e] = silu(h[mt][nt][e]);
                        hs[(16 * mt + 4 * g + e) * 64 + 16 * nt + j] = (unsigned short)(pack2(h[mt][nt][e], 0.0f) & 0xffffu);
                    }
                }
            to_bfrag(h, bq);
            mm_layer<2>(pk + (L == 1 ? kPkL2 : kPkL3), bq, h, lane);
        }
    }
    // h now holds z3: keep z3 in LDS (for the backward pass) and turn h into h3
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            s_z3[(mt * 4 + nt) * 64 + lane] = h[mt][nt];
#pragma unroll
            for (int e = 0; e < 4; ++e) h[mt][nt][e] = silu(h[mt][nt][e]);
        }
    const float y = out_layer(h, tail, lane);
    if (valid && y_out) y_out[row] = y;
    const float diff = valid ? y - target : 0.0f;
    float lsum = diff * diff;
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
    if (lane == 0) loss_part[blockIdx.x] = lsum;
    if (!want_grad) return;
    float *gp = grad_part + (long long)blockIdx.x * kMlpNParam;
    // ---- backward
    const float dy = 2.0f * diff * inv_n;
    float dyn[4];
    #pragma unroll
    for (int nt = 0; nt < 4; ++nt) dyn[nt] = __shfl(dy, 16 * nt + j);
    float db4 = dy;
    for (int o = 32; o > 0; o >>= 1) db4 += __shfl_xor(db4, o);
    if (lane == 0) gp[kB4] = db4;
    // w4 and dz3 (h holds h3, z3 comes back from LDS)
    f32x4 dz[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * mt + 4 * g + e;
            const float w = tail[kTW4 + u];
            float gw = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                gw += h[mt][nt][e] * dyn[nt];
                dz[mt][nt][e] = w * dyn[nt] * dsilu(s_z3[(mt * 4 + nt) * 64 + lane][e]);
            }
            for (int o = 1; o < 16; o <<= 1) gw += __shfl_xor(gw, o);
            if (j == 0) gp[kW4 + u] = gw;
        }
    #pragma unroll
    for (int L = 3; L >= 1; --L) {
        // bias gradient: sum over the rays of dz
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int e = 0; e < 4; ++e) {
                float sb = dz[mt][0][e] + dz[mt][1][e] + dz[mt][2][e] + dz[mt][3][e];
                for (int o = 1; o < 16; o <<= 1) sb += __shfl_xor(sb, o);
                if (j == 0) gp[(L == 3 ? kB3 : L == 2 ? kB2 : kB1) + 16 * mt + 4 * g + e] = sb;
            }
        // weight gradient dW = dz h_prev^T (K = the 64 rays), through LDS
        wave_lds_sync();
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                #pragma unroll
                for (int e = 0; e < 4; ++e)
                    s_dz[(16 * mt + 4 * g + e) * 64 + 16 * nt + j] = (unsigned short)(pack2(dz[mt][nt][e], 0.0f) & 0xffffu);
        wave_lds_sync();
        const unsigned short *hp = L == 3 ? s_h2 : L == 2 ? s_h1 : s_xt;
        const int ntn = L == 1 ? 2 : 4;   // input features of layer 1: 32 (11 used)
        f32x4 gw[4][4];
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int nt = 0; nt < ntn; ++nt) gw[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        #pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            u32x4 bB[4];
            #pragma unroll
            for (int nt = 0; nt < ntn; ++nt)
                bB[nt] = *(const u32x4 *)(hp + (16 * nt + j) * 64 + 32 * kk + 8 * g);
            #pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const u32x4 aA = *(const u32x4 *)(s_dz + (16 * mt + j) * 64 + 32 * kk + 8 * g);
                #pragma unroll
                for (int nt = 0; nt < ntn; ++nt) gw[mt][nt] = mma(aA, bB[nt], gw[mt][nt]);
            }
        }
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int nt = 0; nt < ntn; ++nt)
                #pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int o = 16 * mt + 4 * g + e, i = 16 * nt + j;
                    if (L == 1) {
                        if (i < kMlpIn) gp[kW1 + o * kMlpIn + i] = gw[mt][nt][e];
                    } else {
                        gp[(L == 3 ? kW3 : kW2) + o * kMlpH + i] = gw[mt][nt][e];
                    }
                }
        if (L == 1) break;
        // dh_prev = W^T dz, then dz_prev = dh_prev silu'(z_prev)
        to_bfrag(dz, bq);
        mm_layer<2>(pk + (L == 3 ? kPkB3 : kPkB2), bq, h, lane);
        const f32x4 *zs = L == 3 ? s_z2 : s_z1;
        #pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            #pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const f32x4 zz = zs[(mt * 4 + nt) * 64 + lane];
                #pragma unroll
                for (int e = 0; e < 4; ++e) dz[mt][nt][e] = h[mt][nt][e] * dsilu(zz[e]);
            }
    }
}

// The gradient partials and losses of the tiles summed in two stages, each
// in a fixed order: slice y of the grid sums tiles [kMlpSlice y,
// kMlpSlice (y + 1)) into slice_sum[y] and slice_loss[y] (many threads at
// once, instead of one thread per parameter walking every tile), then
// grad[p] = the sum over the slices in order and loss_acc[0] += the sum of
// the slice losses (launches in stream order).
constexpr int kMlpSlice = 16;
__global__ void k_mlp_reduce_slices(const float *__restrict__ part, const float *__restrict__ loss_part, int n_tiles,
                                    int want_grad, double *__restrict__ slice_sum, double *__restrict__ slice_loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int t0 = blockIdx.y * kMlpSlice, t1 = min(n_tiles, t0 + kMlpSlice);
    if (p == 0) {
        double l = 0.0;
        for (int t = t0; t < t1; ++t) l += loss_part[t];
        slice_loss[blockIdx.y] = l;
    }
    if (!want_grad || p >= kMlpNParam) return;
    double s = 0.0;
    for (int t = t0; t < t1; ++t) s += part[(long long)t * kMlpNParam + p];
    slice_sum[(long long)blockIdx.y * kMlpNParam + p] = s;
}
__global__ void k_mlp_reduce(const double *__restrict__ slice_sum, const double *__restrict__ slice_loss,
                             int n_slices, float *__restrict__ grad, double *__restrict__ loss_acc, int want_grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (want_grad && p < kMlpNParam) {
        double s = 0.0;
        for (int y = 0; y < n_slices; ++y) s += slice_sum[(long long)y * kMlpNParam + p];
        grad[p] = (float)s;
    }
    if (p == 0) {
        double l = 0.0;
        for (int y = 0; y < n_slices; ++y) l += slice_loss[y];
        loss_acc[0] += l;
    }
}

// Adam on the FP32 master weights (bias-corrected moments).
__global__ void k_mlp_adam(float *__restrict__ model, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ grad, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpNParam) return;
    const float gr = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * gr;
    const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    model[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_mlp_store_loss(double *__restrict__ acc, double denom, float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = (float)(acc[0] / denom);
        acc[0] = 0.0;
    }
}

// dst[i] = src[(mul i + add) mod n] for record rows.
__global__ void k_gather_rows(const float *__restrict__ src, float *__restrict__ dst, long long n, long long mul,
                              long long add) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long j = (long long)(((unsigned long long)mul * (unsigned long long)i + (unsigned long long)add) %
                                    (unsigned long long)n);
#pragma unroll
    for (int c = 0; c < kLogRec; ++c) dst[i * kLogRec + c] = src[j * kLogRec + c];
}

__global__ void k_fill_f64(double *p, double v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float *p, float v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ============================================================ per-sample check
__global__ void k_eval_samples(double a, int flat, DevGrid g, PlasmaParams pp, long long n,
                               const double *__restrict__ states, const double *__restrict__ norms,
                               double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[8];
    for (int m = 0; m < 8; ++m) y[m] = states[i * 8 + m];
    double *o = out + i * BL_NSAMPLE_OUT;
    for (int m = 0; m < BL_NSAMPLE_OUT; ++m) o[m] = 0.0;
    double y7[7] = {y[0], y[1], y[2], y[3], y[5], y[6], y[7]}, dy[7];
    geo_rhs(a, flat, y7, y[4], dy);
    o[0] = dy[0]; o[1] = dy[1]; o[2] = dy[2]; o[3] = dy[3];
    o[4] = 0.0; o[5] = dy[4]; o[6] = dy[5]; o[7] = dy[6];
    double G[16];
    conn_k(a, flat, y, y + 4, G);
    for (int m = 0; m < 16; ++m) o[8 + m] = G[m];
    Sample<double> s;
    sample_point<double, true, true>(a, flat, g, pp, y, norms[i], s);
    o[53] = s.sigma;
    if (!s.plasma) return;
    // invariants: j/nu^2, alpha nu, rho nu at the fluid-frame frequency
    for (int m = 0; m < 3; ++m) o[24 + m] = s.co[m] / (s.nu_fl * s.nu_fl);
    for (int m = 3; m < 8; ++m) o[24 + m] = s.co[m] * s.nu_fl;
    o[32] = s.ne; o[33] = s.th; o[34] = s.B; o[35] = s.nu_fl;
    auto k = ks_point(a, flat, y[1], y[2], y[3]);
    double e[4][4];
    tetrad(k, s.u, y + 4, s.b, e);
    for (int q = 0; q < 4; ++q)
        for (int m = 0; m < 4; ++m) o[36 + 4 * q + m] = e[q][m];
    o[52] = 1.0;
}

// The fluid-frame coefficients alone, for checking: rows in [n][5] = n_e,
// Theta_e, B (gauss), nu (Hz), cos theta_B; out [n][8], in the arithmetic
// type R (thermal electrons, or the populations of nth when it is given).
template <typename R>
__global__ void k_eval_coeffs(long long n, const double *__restrict__ in, int polarized, const NthParams *nth,
                              double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *r = in + i * 5;
    R co[8];
    if (nth) {
        thermal_coeffs<R>((R)r[0] * (R)nth->frac[0], (R)r[1], (R)r[2], (R)r[3], (R)r[4], polarized, co);
        nonthermal_coeffs<R>(*nth, (R)r[0], (R)r[2], (R)r[3], (R)r[4], polarized, co);
    } else {
        thermal_coeffs<R>((R)r[0], (R)r[1], (R)r[2], (R)r[3], (R)r[4], polarized, co);
    }
    for (int m = 0; m < 8; ++m) out[i * 8 + m] = (double)co[m];
}

// The plasma substep alone, for checking: coefficient sets c [n][8] (jI, jQ,
// jV, aI, aQ, aV, rQ, rV, the segment length folded in) and states S0
// [n][4], in the arithmetic type R; GENERAL selects the substep of the
// nonthermal kernels (any source vector) over the thermal closed form.
template <typename R, bool GENERAL>
__global__ void k_eval_stokes(long long n, const double *__restrict__ c8, const double *__restrict__ s4,
                              double *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R c[8], S[4];
    for (int m = 0; m < 8; ++m) c[m] = (R)c8[i * 8 + m];
    for (int m = 0; m < 4; ++m) S[m] = (R)s4[i * 4 + m];
    if constexpr (!GENERAL) stokes_step(c, S);
    else if constexpr (sizeof(R) == 4) stokes_step_nth(c, S);
    else stokes_step_general(c, S);
    for (int m = 0; m < 4; ++m) out[i * 4 + m] = (double)S[m];
}

// ============================================================ host side
// Scratch of the allocation-free render (bl_render_noalloc): one static
// device array, which every GPU the library runs on holds (its own copy, at
// its own address) until the process ends.  Host code must not pass the
// array's name to a kernel or a copy (on the host it is only a stand-in):
// the device address comes from hipGetSymbolAddress at context creation.
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr long long kNoAllocMaxSteps = 4095;   // bounds the overflow kernel's private buffer
constexpr int kNoAllocExtSlots = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device workspace of a render: grown on demand by ensure() (hipMalloc), or
// carved from the library's static scratch array by the allocation-free entry
// point, which swaps in an empty set for the duration of its call.
struct RenderBuffers {
    // image descriptors of the current render; the host copies stay alive
    // until the upload that read them has completed (upload_done)
    ImgDev *d_imgs = nullptr;
    size_t imgs_bytes = 0;
    long long *d_ray0 = nullptr;
    size_t ray0_bytes = 0;
    double *d_rec = nullptr;
    size_t rec_bytes = 0;
    double *d_meta = nullptr;
    int *d_nacc = nullptr;
    int *d_work = nullptr;               // transfer iterations per ray slot (the ray order's key)
    size_t work_bytes = 0;
    ExtQueue ext{};                      // extension slots of the current chunk
    size_t ext_rec_bytes = 0, ext_of_bytes = 0;
    int *d_order = nullptr;              // processing order of the chunk's slots
    size_t order_bytes = 0;
    int *d_hist = nullptr;               // counting-sort bins
    size_t slot_cap = 0;
    int *d_ovf_count = nullptr;
    int *d_ovf_list = nullptr;
    size_t ovf_cap = 0;
    double *d_big = nullptr;
    size_t big_bytes = 0;
    int *d_queue = nullptr;              // per-chunk work counters of the persistent kernels
    size_t queue_bytes = 0;
    char *d_ends = nullptr;              // polarized rays' end states, kRayEnd reals per ray slot
    size_t ends_bytes = 0;
    CutParams *d_cuts = nullptr;         // device copy of the data cuts, uploaded with each render
    size_t cuts_bytes = 0;
    NthParams *d_nth = nullptr;          // device copy of the nonthermal populations' constants
    size_t nth_bytes = 0;
};

// Bump allocator over the static scratch array (allocation-free renders).
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};

struct bl_context {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    RenderBuffers rb;
    Arena *arena = nullptr;              // set only during an allocation-free render
    void *scratch = nullptr;             // this device's copy of the static scratch array
    std::vector<ImgDev> h_imgs;
    std::vector<long long> h_ray0;
    hipEvent_t upload_done = nullptr;
    bl_tuning tuning = {8, 8, 0, 4, 0, 0, 0};   // the autotuner's choice for the 1024^2 SMR image
    size_t ws_limit = (size_t)128 << 30;   // bytes of step records per chunk (set at creation)
    int cus = 0;
    int blocks_tr[14] = {0};              // resident waves per CU of k_transfer<pol, R, batch>:
                                         // [4 batch + 2 pol + (R == float)]; [8 + (R == float)]:
                                         // the averages instantiation; [10 + 2 pol + (R == float)]:
                                         // the nonthermal one
    // step-proposal network installed by bl_set_step_model (packed form)
    u32x4 *d_step_pk = nullptr;
    float *d_step_tail = nullptr;
    bool has_step_model = false;
    bl_cuts cuts{};          // data cuts for the following renders (bl_set_cuts)
    bool has_cuts = false;
    int *d_refine = nullptr;       // refinement flags of an adaptive level
    size_t refine_bytes = 0;
    // network training workspace
    u32x4 *d_mlp_pk = nullptr;
    float *d_mlp_tail = nullptr;
    float *d_mlp_gpart = nullptr;
    size_t mlp_gpart_bytes = 0;
    double *d_mlp_slices = nullptr;   // per-slice gradient sums of a pass
    size_t mlp_slices_bytes = 0;
    double *d_mlp_sloss = nullptr;    // per-slice loss sums
    size_t mlp_sloss_bytes = 0;
    float *d_mlp_lpart = nullptr;
    size_t mlp_lpart_bytes = 0;
    float *d_mlp_grad = nullptr, *d_mlp_m = nullptr, *d_mlp_v = nullptr;
    double *d_mlp_acc = nullptr;
    double *d_mlp_stats = nullptr;
    float *d_mlp_rows = nullptr;     // the records in shuffled order
    size_t mlp_rows_bytes = 0;
    unsigned long long *d_log_count = nullptr;
    bool prof = false;
    struct Timed {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
};

struct bl_grid {
    bl_context *ctx = nullptr;
    DevGrid g{};
    double *d_table = nullptr;
};

// ---------------------------------------------------------------- adaptive
// Refinement criteria of one block of an adaptive level (paper section 4.4,
// Adaptive Ray Tracing), on Stokes I of the block's B x B pixels alone:
// central differences inside the block, one-sided ones at its edges (the
// gradient: the two-point difference; the Laplacian: the second difference
// of the nearest interior pixel), none along a direction of one pixel (two
// for the Laplacian); the relative forms divide by the 1-2-1 weighted sum
// (the pair sum / 2 for a one-sided gradient) and are 0 where that is 0.
// Evaluated without contraction so that a decision depends only on the
// intensities and the thresholds.
struct RefineParams {
    int b, level, n_root, n_regions;
    int use[5], pad;
    double thr[5];
    double frac, width;
    double region[8][5];   // x0, x1, y0, y1, minimum level
};

__device__ double crit_grad(const double *v, int stride, int n, int k, bool rel) {
#pragma clang fp contract(off)
    if (n < 2) return 0.0;
    if (k > 0 && k < n - 1) {
        const double a = v[(k - 1) * stride], b = v[k * stride], c = v[(k + 1) * stride];
        if (rel) {
            const double sw = a + 2.0 * b + c;
            return sw == 0.0 ? 0.0 : 2.0 * (c - a) / sw;
        }
        return 0.5 * (c - a);
    }
    const double lo = k == 0 ? v[0] : v[(n - 2) * stride], hi = k == 0 ? v[stride] : v[(n - 1) * stride];
    if (rel) {
        const double sw = lo + hi;
        return sw == 0.0 ? 0.0 : 2.0 * (hi - lo) / sw;
    }
    return hi - lo;
}

__device__ double crit_lap(const double *v, int stride, int n, int k, bool rel) {
#pragma clang fp contract(off)
    if (n < 3) return 0.0;
    const int m = k < 1 ? 1 : (k > n - 2 ? n - 2 : k);
    const double a = v[(m - 1) * stride], b = v[m * stride], c = v[(m + 1) * stride];
    const double d2 = a - 2.0 * b + c;
    if (rel) {
        const double sw = a + 2.0 * b + c;
        return sw == 0.0 ? 0.0 : 4.0 * d2 / sw;
    }
    return d2;
}

// One wave per block: flags[k] = 1 if block k of the level refines.
// blocks: [n_blocks][3] (level, bx, by); img: the level's images, block k at
// img + k 4 B^2, Stokes I first.  Launched with exactly n_blocks groups.
__global__ void __launch_bounds__(64) k_refine(RefineParams rp, const int *__restrict__ blocks,
                                               const double *__restrict__ img, int n_blocks,
                                               int *__restrict__ flags) {
#pragma clang fp contract(off)
    const int k = blockIdx.x;
    if (k >= n_blocks) return;
    const int lane = threadIdx.x, b = rp.b, bb = b * b;
    const double *I = img + (size_t)k * 4 * bb;
    int cnt[5] = {0, 0, 0, 0, 0};
    for (int p = lane; p < bb; p += 64) {
        const int j = p / b, i = p - j * b;
        const double *row = I + (size_t)j * b, *col = I + i;
        double v[5];
        v[0] = I[p];
        double gi = crit_grad(row, 1, b, i, false), gj = crit_grad(col, b, b, j, false);
        v[1] = sqrt(gi * gi + gj * gj);
        gi = crit_grad(row, 1, b, i, true);
        gj = crit_grad(col, b, b, j, true);
        v[2] = sqrt(gi * gi + gj * gj);
        v[3] = fabs(crit_lap(row, 1, b, i, false) + crit_lap(col, b, b, j, false));
        v[4] = fabs(crit_lap(row, 1, b, i, true) + crit_lap(col, b, b, j, true));
#pragma unroll
        for (int c = 0; c < 5; ++c) cnt[c] += (rp.use[c] && v[c] > rp.thr[c]) ? 1 : 0;
    }
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt[c] += __shfl_xor(cnt[c], o);
    if (lane != 0) return;
    bool ref = false;
    const double need = rp.frac * (double)bb;
#pragma unroll
    for (int c = 0; c < 5; ++c) ref = ref || (rp.use[c] && (double)cnt[c] >= need);
    const int bx = blocks[3 * k + 1], by = blocks[3 * k + 2];
    const double nl = (double)rp.n_root * (double)(1LL << rp.level);
    const double cx = ((double)bx * b + 0.5 * b - 0.5 * nl) * rp.width / nl;
    const double cy = ((double)by * b + 0.5 * b - 0.5 * nl) * rp.width / nl;
    for (int r = 0; r < rp.n_regions; ++r) {
        const double *g = rp.region[r];
        if (g[0] <= cx && cx <= g[1] && g[2] <= cy && cy <= g[3] && (double)rp.level < g[4]) ref = true;
    }
    flags[k] = ref ? 1 : 0;
}

namespace {

bl_status fail(bl_context *ctx, bl_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, e_ == hipErrorOutOfMemory ? BL_E_OOM : BL_E_DEVICE,                   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)

bl_status check_camera(bl_context *ctx, const bl_camera *cam) {
    if (!cam) return fail(ctx, BL_E_INVALID_ARG, "camera is NULL");
    if (cam->n < 1 || cam->n > 16384) return fail(ctx, BL_E_INVALID_ARG, "camera n must be in 1..16384");
    if (!(cam->width > 0.0) || !(cam->r > 0.0) || !(cam->nu_hz > 0.0))
        return fail(ctx, BL_E_INVALID_ARG, "camera width, r and nu_hz must be positive");
    if (cam->freq_mode != 0 && cam->freq_mode != 1) return fail(ctx, BL_E_INVALID_ARG, "freq_mode must be 0 or 1");
    if (cam->kind != 0)
        return fail(ctx, BL_E_UNSUPPORTED, "only the plane-parallel camera (kind 0) is built");
    return BL_OK;
}

bl_status check_spacetime(bl_context *ctx, const bl_spacetime *st) {
    if (!st) return fail(ctx, BL_E_INVALID_ARG, "spacetime is NULL");
    if (!(std::fabs(st->a) < 1.0)) return fail(ctx, BL_E_INVALID_ARG, "spin must satisfy |a| < 1");
    if (!(st->mass_msun > 0.0)) return fail(ctx, BL_E_INVALID_ARG, "mass_msun must be positive");
    if (!(st->r_in >= 0.0)) return fail(ctx, BL_E_INVALID_ARG, "r_in must be >= 0");
    return BL_OK;
}

bl_status check_integrator(bl_context *ctx, const bl_integrator *in) {
    if (!in) return fail(ctx, BL_E_INVALID_ARG, "integrator is NULL");
    if (!(in->f_abs >= 0.0) || !(in->f_rel >= 0.0) || !(in->ds_max >= 0.0) || !(in->h0_frac > 0.0))
        return fail(ctx, BL_E_INVALID_ARG, "tolerances and ds_max must be >= 0, h0_frac > 0");
    if (in->max_steps < 1 || in->max_steps > (int64_t)1 << 30)
        return fail(ctx, BL_E_INVALID_ARG, "max_steps must be in 1..2^30");
    if (in->record_cap < 0 || in->record_cap == 1) return fail(ctx, BL_E_INVALID_ARG, "record_cap must be 0 or >= 2");
    return BL_OK;
}

CamParams cam_params(const bl_camera *c) {
    CamParams p;
    p.r = c->r;
    p.theta = c->theta;
    p.phi = c->phi;
    for (int i = 0; i < 3; ++i) {
        p.u_normal[i] = c->u_normal[i];
        p.k_cov[i] = c->k_cov[i];
    }
    p.width = c->width;
    p.psi = c->psi;
    p.nu = c->nu_hz;
    p.n = c->n;
    p.nf = c->n;
    p.i0 = p.j0 = p.pad_c = 0;
    p.freq_mode = c->freq_mode;
    return p;
}

// Step records per ray slot by default: 512 records (98 KB) hold all but about
// one ray in 30000 even in strongly lensed images (high spin, edge-on: up to
// 9 % of rays pass 256 steps there); those move to the 2048-record extension
// slots as they grow.
constexpr int kDefaultRecordCap = 512;

GeoParams geo_params(const bl_camera *c, const bl_spacetime *st, const bl_integrator *in) {
    GeoParams P;
    P.a = st->a;
    P.r_in = st->r_in;
    P.r_cam = c->r;
    P.f_abs = in ? in->f_abs : 1e-8;
    P.f_rel = in ? in->f_rel : 1e-8;
    P.h0_frac = in ? in->h0_frac : 0.01;
    P.max_steps = in ? in->max_steps : 100000;
    P.flat = st->flat ? 1 : 0;
    P.cap = (in && in->record_cap > 0) ? in->record_cap : kDefaultRecordCap;
    P.n = c->n;
    // no records are sampled unless a render sets the grid box, the piece
    // length and the record layout (record_layout)
    P.rec_quart32 = 0;
    P.net_every = 1;
    for (int d = 0; d < 6; ++d) P.bb[d] = 0.0;
    P.ds_max = 0.0;
    return P;
}

PlasmaParams plasma_params(const bl_context *ctx, const bl_plasma *plasma, const DevGrid &g, double mass_msun) {
    PlasmaParams pp;
    pp.mu = plasma->mu;
    pp.ne_ni = plasma->ne_ni;
    pp.r_high = plasma->r_high;
    pp.r_low = plasma->r_low;
    pp.sigma_max = plasma->sigma_max;
    pp.mass_msun = mass_msun;
    pp.polarized = plasma->polarized ? 1 : 0;
    pp.interp = plasma->interp ? 1 : 0;
    pp.ne_per_rho = g.rho_unit / (pp.mu * kMp) / (1.0 + 1.0 / pp.ne_ni);
    pp.th_per_pr = pp.mu * kMp / kMe;
    pp.gauss_per_b = kC * sqrt(4.0 * kPi * g.rho_unit);
    pp.cuts = ctx->has_cuts ? 1 : 0;
    pp.cut = ctx->rb.d_cuts;
    pp.nonthermal = 0;
    pp.nth = ctx->rb.d_nth;
    return pp;
}

// A device buffer of at least need_bytes in *p (have: its current size).
template <typename T>
bl_status ensure(bl_context *ctx, T **p, size_t &have, size_t need_bytes) {
    if (ctx->arena) {
        // allocation-free render: the next 256-byte aligned piece of the
        // static scratch array (never hipMalloc)
        Arena &A = *ctx->arena;
        const size_t off = (A.used + 255) & ~(size_t)255;
        if (need_bytes > A.cap || off > A.cap - need_bytes)
            return fail(ctx, BL_E_UNSUPPORTED,
                        "the allocation-free render needs more than the " + std::to_string(A.cap) +
                            " bytes of its static scratch: lower record_cap, max_steps or the image size");
        *p = reinterpret_cast<T *>(A.base + off);
        have = need_bytes;
        A.used = off + need_bytes;
        return BL_OK;
    }
    if (have >= need_bytes && *p) return BL_OK;
    if (*p) {
        HIPCHK(ctx, hipFree(*p));
        *p = nullptr;
        have = 0;
    }
    hipError_t e = hipMalloc((void **)p, need_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // do not leave the failure for the next launch check
        *p = nullptr;
        return fail(ctx, e == hipErrorOutOfMemory ? BL_E_OOM : BL_E_DEVICE,
                    std::string("hipMalloc of ") + std::to_string(need_bytes) + " bytes: " + hipGetErrorString(e));
    }
    have = need_bytes;
    return BL_OK;
}

// Device copy of the context's data cuts for the launches that follow on the
// stream (the copy is ordered with them).
bl_status upload_cuts(bl_context *ctx) {
    if (!ctx->has_cuts) return BL_OK;
    bl_status s;
    if ((s = ensure(ctx, &ctx->rb.d_cuts, ctx->rb.cuts_bytes, sizeof(CutParams))) != BL_OK) return s;
    const bl_cuts &c = ctx->cuts;
    CutParams h{};
    const double *lims[8] = {c.rho, c.ne, c.p, c.theta_e, c.b, c.sigma, c.beta_inv, c.r};
    for (int k = 0; k < 8; ++k) {
        h.lo[k] = lims[k][0];
        h.hi[k] = lims[k][1];
        h.lo_f[k] = (float)h.lo[k];
        h.hi_f[k] = (float)h.hi[k];
    }
    for (int i = 0; i < 3; ++i) {
        h.x0[i] = c.plane_origin[i];
        h.n[i] = c.plane_normal[i];
    }
    h.plane = c.plane;
    HIPCHK(ctx, hipMemcpyAsync(ctx->rb.d_cuts, &h, sizeof(CutParams), hipMemcpyHostToDevice, ctx->stream));
    // the host struct is a local: wait for the copy to have read it
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return BL_OK;
}

// Electron populations of a plasma (paper sections 2.6 and 4.5): validation
// and the fractions (all zero: thermal electrons only).
bl_status nth_fractions(bl_context *ctx, const bl_plasma *pl, double fr[3]) {
    fr[0] = pl->fractions[0];
    fr[1] = pl->fractions[1];
    fr[2] = pl->fractions[2];
    if (fr[0] == 0.0 && fr[1] == 0.0 && fr[2] == 0.0) fr[0] = 1.0;
    if (!(fr[0] >= 0.0) || !(fr[1] >= 0.0) || !(fr[2] >= 0.0) || !(fabs(fr[0] + fr[1] + fr[2] - 1.0) <= 1e-9))
        return fail(ctx, BL_E_INVALID_ARG, "electron fractions must be non-negative and sum to 1");
    if (fr[1] > 0.0 && !(pl->pl_p > 1.0 && pl->pl_gamma_min >= 1.0 && pl->pl_gamma_max > pl->pl_gamma_min &&
                         std::isfinite(pl->pl_gamma_max)))
        return fail(ctx, BL_E_INVALID_ARG, "power law needs p > 1 and 1 <= gamma_min < gamma_max < inf");
    if (fr[2] > 0.0 && !(pl->kappa >= 2.5 && std::isfinite(pl->kappa) && pl->kappa_w > 0.0 &&
                         std::isfinite(pl->kappa_w)))
        return fail(ctx, BL_E_INVALID_ARG, "kappa distribution needs kappa >= 2.5 and w > 0");
    return BL_OK;
}

// int_1^inf gamma^s gamma sqrt(gamma^2 - 1) (1 + (gamma - 1)/(kappa w))^-(kappa+1) dgamma
// by the trapezoid rule in v = ln(gamma - 1) over [-80, 100] (the integrand
// times e^v decays exponentially at both ends for kappa >= 2.5, s <= 0),
// each term formed from its logarithm.
double kappa_moment(double kap, double w, double s) {
    const double h = 0.0025, kw = kap * w;
    double sum = 0.0;
    for (int i = 0; i <= 72000; ++i) {
        const double v = -80.0 + i * h;
        const double t = exp(v), lg = log1p(t);
        const double lf = lg * (1.0 + s) + 0.5 * (v + log(2.0 + t)) - (kap + 1.0) * log1p(t / kw) + v;
        sum += exp(lf);
    }
    return sum * h;
}

// The power-law terms of NthParams for dn/dgamma = n_e C gamma^-p.
void nth_powerlaw_terms(NthParams &q, int k, double p, double C) {
    q.lhj[k] = log(C) + 0.5 * p * log(3.0) - log(2.0 * (p + 1.0)) + lgamma((3.0 * p - 1.0) / 12.0) +
               lgamma((3.0 * p + 19.0) / 12.0);
    q.ej[k] = -0.5 * (p - 1.0);
    q.lhjq[k] = log((p + 1.0) / (p + 7.0 / 3.0));
    q.lha[k] = log(C) + 0.5 * (p + 1.0) * log(3.0) - log(4.0) + lgamma((3.0 * p + 2.0) / 12.0) +
               lgamma((3.0 * p + 22.0) / 12.0);
    q.ea[k] = -0.5 * (p + 2.0);
    q.lhaq[k] = log((p + 2.0) / (p + 10.0 / 3.0));
}

// Host constants of a plasma's electron populations; active: a nonthermal
// population is present.
bl_status nth_params(bl_context *ctx, const bl_plasma *pl, NthParams &q, bool &active) {
    double fr[3];
    bl_status s;
    if ((s = nth_fractions(ctx, pl, fr)) != BL_OK) return s;
    active = fr[1] > 0.0 || fr[2] > 0.0;
    q = NthParams{};
    if (!active) return BL_OK;
    for (int k = 0; k < 3; ++k) q.frac[k] = fr[k];
    if (fr[1] > 0.0) {
        const double p = pl->pl_p;
        nth_powerlaw_terms(q, 0, p, (p - 1.0) / (pow(pl->pl_gamma_min, 1.0 - p) - pow(pl->pl_gamma_max, 1.0 - p)));
    }
    if (fr[2] > 0.0) {
        const double kap = pl->kappa, w = pl->kappa_w, kw = kap * w;
        const double z0 = kappa_moment(kap, w, 0.0);
        nth_powerlaw_terms(q, 1, kap - 1.0, pow(kw, kap + 1.0) / z0);
        // F(x) ~ (4 pi/(sqrt3 Gamma(1/3))) (x/2)^1/3 for small x, x/2 = X/(3 gamma^2)
        const double g13 = tgamma(1.0 / 3.0);
        q.llj = log(2.0 * kPi / g13) - log(3.0) / 3.0 + log(kappa_moment(kap, w, -2.0 / 3.0) / z0);
        q.lla = log(4.0 * kPi / (3.0 * g13)) - log(3.0) / 3.0 + log(kappa_moment(kap, w, -5.0 / 3.0) / z0);
    }
    return BL_OK;
}

// Device copies of the populations' constants of n plasmas for the launches
// that follow, one slot each (uploaded only when one of them has a nonthermal
// population), and each plasma's PlasmaParams pointed at its slot.
bl_status upload_nth(bl_context *ctx, int n, const bl_plasma *const *pls, PlasmaParams *pps) {
    // no host allocation for one plasma (the allocation-free render)
    NthParams q1{};
    std::vector<NthParams> qv;
    NthParams *q = &q1;
    if (n > 1) {
        qv.resize(n);
        q = qv.data();
    }
    bool any = false;
    bl_status s;
    for (int f = 0; f < n; ++f) {
        bool a = false;
        if ((s = nth_params(ctx, pls[f], q[f], a)) != BL_OK) return s;
        pps[f].nonthermal = a ? 1 : 0;
        any = any || a;
    }
    if (!any) return BL_OK;
    if ((s = ensure(ctx, &ctx->rb.d_nth, ctx->rb.nth_bytes, (size_t)n * sizeof(NthParams))) != BL_OK) return s;
    HIPCHK(ctx, hipMemcpyAsync(ctx->rb.d_nth, q, (size_t)n * sizeof(NthParams), hipMemcpyHostToDevice, ctx->stream));
    // the host structs are locals: wait for the copy to have read them
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int f = 0; f < n; ++f) pps[f].nth = ctx->rb.d_nth + f;
    return BL_OK;
}

// What the geodesic kernels store with each record for the transfer: the grid
// box and piece length for the sampling decision, and the FP32-quartic layout
// for the mixed form (whose transfer kernels read it).
void record_layout(GeoParams &P, const DevGrid &g, const bl_integrator *in, bool mixed) {
    for (int d = 0; d < 6; ++d) P.bb[d] = g.bb[d];
    P.ds_max = in->ds_max;
    P.rec_quart32 = mixed ? 1 : 0;
}


// Event pair around one launch when timing is on.
struct TimedLaunch {
    bl_context *ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(bl_context *c, int k) : ctx(c), kind(k) {
        if (!ctx->prof) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, ctx->stream);
    }
    ~TimedLaunch() {
        if (!a) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->timed.push_back({kind, a, b});
    }
};

// Waves per CU of each persistent transfer kernel that fit at once.
bl_status persistent_waves(bl_context *ctx) {
    if (ctx->cus > 0) return BL_OK;
    int cus = 0, b[14] = {0};
    HIPCHK(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[0], k_transfer<false, double, false, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[1], k_transfer<false, float, false, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[2], k_transfer<true, double, false, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[3], k_transfer<true, float, false, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[4], k_transfer<false, double, true, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[5], k_transfer<false, float, true, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[6], k_transfer<true, double, true, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[7], k_transfer<true, float, true, false>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[8], k_transfer<false, double, false, false, true>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[9], k_transfer<false, float, false, false, true>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[10], k_transfer<false, double, false, false, false, true>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[11], k_transfer<false, float, false, false, false, true>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[12], k_transfer<true, double, false, false, false, true>, 64, 0));
    HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[13], k_transfer<true, float, false, false, false, true>, 64, 0));
    for (int k = 0; k < 14; ++k) ctx->blocks_tr[k] = std::max(1, b[k]);
    ctx->cus = std::max(1, cus);
    return BL_OK;
}

bl_status check_tuning(bl_context *ctx, const bl_tuning *t) {
    if (!t) return fail(ctx, BL_E_INVALID_ARG, "tuning is NULL");
    bool rowmajor = t->tile_w == 0 && t->tile_h == 0;
    if (!rowmajor && !(t->tile_w > 0 && t->tile_h > 0 && t->tile_w * t->tile_h == 64))
        return fail(ctx, BL_E_INVALID_ARG, "tile_w * tile_h must be 64 (or both 0)");
    if (t->transfer_waves_per_cu < 0 || t->transfer_waves_per_cu > 64)
        return fail(ctx, BL_E_INVALID_ARG, "transfer_waves_per_cu must be in 0..64");
    if (t->refill_min < 1 || t->refill_min > 64) return fail(ctx, BL_E_INVALID_ARG, "refill_min must be in 1..64");
    if (t->chunk_rays < 0 || t->chunk_rays % 64 != 0 || t->chunk_rays > (1LL << 30))
        return fail(ctx, BL_E_INVALID_ARG, "chunk_rays must be a multiple of 64 in 0..2^30");
    if (t->order != 0 && t->order != 1) return fail(ctx, BL_E_INVALID_ARG, "order must be 0 or 1");
    if (t->reserved != 0) return fail(ctx, BL_E_INVALID_ARG, "reserved must be 0");
    return BL_OK;
}

// Ray ids owned by an image of side n under the tuning's pixel order.
long long image_rays(int n, const bl_tuning &t) {
    if (t.tile_w <= 0) return (long long)n * n;
    long long ntx = (n + t.tile_w - 1) / t.tile_w, nty = (n + t.tile_h - 1) / t.tile_h;
    return ntx * nty * 64;
}

// Build and upload the image table (in placement order: given, or largest
// first) and launch the camera-frame kernel.  Returns the batch view and the
// total ray-id count.
// Image table of n entries.  With shared_rays every entry describes the
// same rays (the same camera at the frequencies of a multi-frequency render:
// ray ids start at 0 for each and the render has one image's rays).
bl_status upload_images(bl_context *ctx, int n, const bl_camera *const *cams, const bl_spacetime *const *sts,
                        double *const *images, double *const *auxs, const bl_tuning &t, Batch &B,
                        long long &total, bool shared_rays = false, double *const *avgs = nullptr,
                        const int *sub = nullptr) {
    // placement order (no host allocation for a single image: the context
    // reserved room for one descriptor at creation)
    int perm1 = 0;
    std::vector<int> permv;
    int *perm = &perm1;
    if (n > 1) {
        permv.resize(n);
        for (int k = 0; k < n; ++k) permv[k] = k;
        if (t.order == 1)
            std::stable_sort(permv.begin(), permv.end(), [&](int x, int y) { return cams[x]->n > cams[y]->n; });
        perm = permv.data();
    }
    HIPCHK(ctx, hipEventSynchronize(ctx->upload_done));
    ctx->h_imgs.assign(n, ImgDev{});
    ctx->h_ray0.assign(n, 0);
    long long r = 0;
    for (int q = 0; q < n; ++q) {
        const int k = perm[q];
        ImgDev &im = ctx->h_imgs[q];
        im.cp = cam_params(cams[k]);
        if (sub) {   // a block of a finer image: (nf, i0, j0) per image
            im.cp.nf = sub[3 * k];
            im.cp.i0 = sub[3 * k + 1];
            im.cp.j0 = sub[3 * k + 2];
        }
        im.a = sts[k]->a;
        im.r_in = sts[k]->r_in;
        im.flat = sts[k]->flat ? 1 : 0;
        im.L = kG * sts[k]->mass_msun * kMsun / (kC * kC);
        im.image = images[k];
        im.aux = auxs[k];
        im.avg = avgs ? avgs[k] : nullptr;
        im.ray0 = shared_rays ? 0 : r;
        im.nray = image_rays(cams[k]->n, t);
        ctx->h_ray0[q] = im.ray0;
        if (!shared_rays || q == 0) r += im.nray;
    }
    if (r >= (1LL << 31)) return fail(ctx, BL_E_UNSUPPORTED, "more than 2^31 - 1 ray ids in one render");
    bl_status s;
    if ((s = ensure(ctx, &ctx->rb.d_imgs, ctx->rb.imgs_bytes, (size_t)n * sizeof(ImgDev))) != BL_OK) return s;
    if ((s = ensure(ctx, &ctx->rb.d_ray0, ctx->rb.ray0_bytes, (size_t)n * sizeof(long long))) != BL_OK) return s;
    HIPCHK(ctx, hipMemcpyAsync(ctx->rb.d_imgs, ctx->h_imgs.data(), (size_t)n * sizeof(ImgDev), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->rb.d_ray0, ctx->h_ray0.data(), (size_t)n * sizeof(long long),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
    B.imgs = ctx->rb.d_imgs;
    B.ray0 = ctx->rb.d_ray0;
    B.n_img = n;   // every entry gets its camera frame
    B.tw = t.tile_w;
    B.th = t.tile_h;
    B.pad = 0;
    {
        TimedLaunch tl(ctx, BL_K_SETUP);
        hipLaunchKernelGGL(k_camera_frame, dim3((unsigned)n), dim3(64), 0, ctx->stream, B);
    }
    HIPCHK(ctx, hipGetLastError());
    if (shared_rays) B.n_img = 1;   // the entries describe one image's rays
    total = r;
    return BL_OK;
}

bl_status upload_one(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st, double *image, double *aux,
                     const bl_tuning &t, Batch &B, long long &total) {
    return upload_images(ctx, 1, &cam, &st, &image, &aux, t, B, total);
}

template <bool POL, typename R, bool BATCH, bool CUTS, bool AVG = false, bool NTH = false>
void launch_transfer(bl_context *ctx, dim3 grd, const GeoParams &P, const Batch &B, const DevGrid &g,
                     const PlasmaParams &pp, const TransferParams &tp, long long start, int count, int refill,
                     int *q) {
    R *ends = reinterpret_cast<R *>(ctx->rb.d_ends);
    hipLaunchKernelGGL((k_transfer<POL, R, BATCH, CUTS, AVG, NTH>), grd, dim3(64), 0, ctx->stream, P, B, g, pp, tp, start, count,
                       refill, ctx->rb.d_rec, ctx->rb.d_meta, ctx->rb.d_nacc, ctx->rb.d_order, ctx->rb.ext, q, ends);
    if (POL)
        hipLaunchKernelGGL((k_finish<R, BATCH>), dim3((count + 63) / 64), dim3(64), 0, ctx->stream, P, B, start, count,
                           ctx->rb.d_rec, ctx->rb.d_nacc, ctx->rb.ext, (const R *)ends);
}

template <bool POL, typename R, bool CUTS, bool AVG = false, bool NTH = false>
void launch_overflow(bl_context *ctx, const GeoParams &P, const Batch &B, const DevGrid &g, const PlasmaParams &pp,
                     const TransferParams &tp, int big_cap) {
    hipLaunchKernelGGL((k_overflow<POL, R, CUTS, AVG, NTH>), dim3(1), dim3(64), 0, ctx->stream, P, B, g, pp, tp, ctx->rb.d_ovf_count,
                       ctx->rb.d_ovf_list, ctx->rb.d_big, big_cap);
}

// The render of n images (a batch of one for bl_render).  With batch = false
// there is one image and the kernels take its parameters as wave-uniform
// values.
// With n_freq > 0 (one image, batch = false) the cameras cams[0..n_freq) are
// one camera at the frequencies of a multi-frequency render: the geodesics
// are traced once per chunk and the transfer runs once per frequency on the
// same step records, each writing its own image and aux.
// The overflow kernel over the rays queued so far, once per output (frequency
// and plasma): rays longer than the extension slots are traced again for each.
bl_status overflow_all(bl_context *ctx, const Batch &B, const GeoParams &P, const bl_grid *grid,
                       const PlasmaParams *pps, const TransferParams &tp, const bl_camera *const *cams, int n_tr,
                       bool mixed, int big_cap) {
    for (int f = 0; f < n_tr; ++f) {
        Batch Bf = B;
        Bf.imgs = B.imgs + f;
        TransferParams tpf = tp;
        tpf.nu_cam = cams[f]->nu_hz;
        const PlasmaParams &pp = pps[f];
        TimedLaunch tl(ctx, BL_K_OVERFLOW);
        switch (2 * pp.polarized + (mixed ? 1 : 0) + (pp.nonthermal ? 8 : (pp.cuts ? 4 : 0))) {
        case 8: launch_overflow<false, double, false, false, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 9: launch_overflow<false, float, false, false, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 10: launch_overflow<true, double, false, false, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 11: launch_overflow<true, float, false, false, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 0: launch_overflow<false, double, false>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 1: launch_overflow<false, float, false>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 2: launch_overflow<true, double, false>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 3: launch_overflow<true, float, false>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 4: launch_overflow<false, double, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 5: launch_overflow<false, float, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        case 6: launch_overflow<true, double, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        default: launch_overflow<true, float, true>(ctx, P, Bf, grid->g, pp, tpf, big_cap); break;
        }
        HIPCHK(ctx, hipGetLastError());
    }
    return BL_OK;
}

// Options of the allocation-free render: extension slots per chunk, and the
// overflow kernel run after every chunk (so its ray list holds one chunk's
// rays, not the whole image's).
struct RenderOpts {
    int ext_slots = 1024;
    bool per_chunk_overflow = false;
};

bl_status render_images(bl_context *ctx, int n, const bl_camera *const *cams, const bl_spacetime *const *sts,
                        double *const *images, double *const *auxs, const bl_integrator *integ, const bl_grid *grid,
                        const bl_plasma *plasma, const bl_mode *mode, const bl_tuning &t, bool batch,
                        int n_freq = 0, double *avg = nullptr, const int *sub = nullptr,
                        const RenderOpts &opt = RenderOpts(), const bl_plasma *const *tr_plasmas = nullptr) {
    bl_status s;
    if ((s = check_integrator(ctx, integ)) != BL_OK || (s = check_tuning(ctx, &t)) != BL_OK) return s;
    if (n_freq > 0 && (n != 1 || batch)) return fail(ctx, BL_E_INVALID_ARG, "a multi-frequency render has one image");
    if (avg && (n != 1 || batch || n_freq > 0)) return fail(ctx, BL_E_INVALID_ARG, "averages are for one image");
    const int n_tr = n_freq > 0 ? n_freq : 1;   // transfers per chunk
    const int n_q = n_tr + (avg ? 1 : 0);        // queue counters per chunk (the averages pass has its own)
    for (int k = 0; k < (n_freq > 0 ? n_freq : n); ++k) {
        if ((s = check_camera(ctx, cams[k])) != BL_OK || (s = check_spacetime(ctx, sts[k])) != BL_OK) return s;
        if (!images[k] || !auxs[k]) return fail(ctx, BL_E_INVALID_ARG, "image and aux outputs must be non-NULL");
    }
    if (!grid || !plasma) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    if (tr_plasmas && n_freq < 1) return fail(ctx, BL_E_INVALID_ARG, "per-output plasmas need a multi-output render");
    if (mode && (mode->precision < 0 || mode->precision > 1))
        return fail(ctx, BL_E_INVALID_ARG, "precision must be 0 (FP64) or 1 (mixed)");
    if (mode && (mode->step_model < 0 || mode->step_model > 64))
        return fail(ctx, BL_E_INVALID_ARG, "step_model must be 0 (controller) or 1..64 (learned)");
    const bool learned = mode && mode->step_model >= 1;
    if (learned && !ctx->has_step_model)
        return fail(ctx, BL_E_STATE, "learned step proposals need a network installed with bl_set_step_model");
    if (grid && grid->ctx != ctx) return fail(ctx, BL_E_STATE, "the grid belongs to another context");
    const bool mixed = mode && mode->precision == 1;
    if (grid->g.dtype != 0 && !mixed) return fail(ctx, BL_E_UNSUPPORTED, "float32 grids need precision 1");
    // the plasma of each output (the same one unless the caller gives one per
    // output of a multi-output render)
    const bl_plasma *pl1 = plasma;
    const bl_plasma *const *pls = tr_plasmas ? tr_plasmas : &pl1;
    for (int f = 0; f < (tr_plasmas ? n_tr : 1); ++f) {
        const bl_plasma *pl = pls[f];
        if (!pl) return fail(ctx, BL_E_INVALID_ARG, "NULL plasma");
        if (!(pl->mu > 0.0) || !(pl->ne_ni > 0.0) || !(pl->sigma_max >= 0.0))
            return fail(ctx, BL_E_INVALID_ARG, "plasma mu, ne_ni must be positive and sigma_max >= 0");
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if ((s = persistent_waves(ctx)) != BL_OK) return s;
    Batch B;
    long long total = 0;
    if ((s = upload_images(ctx, n_freq > 0 ? n_freq : n, cams, sts, images, auxs, t, B, total, n_freq > 0,
                           avg ? &avg : nullptr, sub)) != BL_OK)
        return s;
    GeoParams P = geo_params(cams[0], sts[0], integ);
    record_layout(P, grid->g, integ, mixed);
    if (learned) P.net_every = mode->step_model;
    size_t rec_per_ray = (size_t)P.cap * kRecDoubles * sizeof(double);
    long long chunk = t.chunk_rays > 0 ? t.chunk_rays : (long long)(ctx->ws_limit / rec_per_ray);
    chunk = std::max(64LL, chunk - chunk % 64);
    chunk = std::min(chunk, (total + 63) / 64 * 64);
    if ((s = ensure(ctx, &ctx->rb.d_rec, ctx->rb.rec_bytes, (size_t)chunk * rec_per_ray)) != BL_OK) return s;
    size_t have_meta = ctx->rb.slot_cap * 2 * sizeof(double), have_nacc = ctx->rb.slot_cap * sizeof(int);
    if ((s = ensure(ctx, &ctx->rb.d_meta, have_meta, (size_t)chunk * 2 * sizeof(double))) != BL_OK) return s;
    if ((s = ensure(ctx, &ctx->rb.d_nacc, have_nacc, (size_t)chunk * sizeof(int))) != BL_OK) return s;
    ctx->rb.slot_cap = std::min(have_meta / (2 * sizeof(double)), have_nacc / sizeof(int));
    if ((s = ensure(ctx, &ctx->rb.d_order, ctx->rb.order_bytes, (size_t)chunk * sizeof(int))) != BL_OK) return s;
    if ((s = ensure(ctx, &ctx->rb.d_work, ctx->rb.work_bytes, (size_t)chunk * sizeof(int))) != BL_OK) return s;
    if ((s = ensure(ctx, &ctx->rb.d_ends, ctx->rb.ends_bytes,
                    (size_t)chunk * kRayEnd * (mixed ? sizeof(float) : sizeof(double)))) != BL_OK)
        return s;
    // extension slots for rays longer than a record slot: 1024 per chunk of
    // 2048 records (or max_steps + 1 if less), when that is more than a slot;
    // a ray that finds no free extension slot is finished by the single-wave
    // overflow kernel
    {
        ExtQueue &X = ctx->rb.ext;
        const int cap_rec = (int)std::min<long long>(2048, P.max_steps + 1);
        X.cap_rays = cap_rec > P.cap ? opt.ext_slots : 0;
        X.cap_rec = cap_rec;
        size_t have = X.count ? sizeof(int) : 0;
        if ((s = ensure(ctx, &X.count, have, sizeof(int))) != BL_OK) return s;
        if ((s = ensure(ctx, &X.of, ctx->rb.ext_of_bytes, (size_t)chunk * sizeof(int))) != BL_OK) return s;
        if (X.cap_rays > 0 &&
            (s = ensure(ctx, &X.rec, ctx->rb.ext_rec_bytes,
                        (size_t)X.cap_rays * X.cap_rec * kRecDoubles * sizeof(double))) != BL_OK)
            return s;
    }
    {
        size_t have_hist = ctx->rb.d_hist ? (size_t)kOrderBins * sizeof(int) : 0;
        if ((s = ensure(ctx, &ctx->rb.d_hist, have_hist, (size_t)kOrderBins * sizeof(int))) != BL_OK) return s;
    }
    size_t one = sizeof(int);
    size_t have_cnt = ctx->rb.d_ovf_count ? one : 0;
    if ((s = ensure(ctx, &ctx->rb.d_ovf_count, have_cnt, one)) != BL_OK) return s;
    if ((s = ensure(ctx, &ctx->rb.d_ovf_list, ctx->rb.ovf_cap,
                    (size_t)(opt.per_chunk_overflow ? chunk : total) * sizeof(int))) != BL_OK)
        return s;
    int big_cap = (int)std::min<long long>(P.max_steps + 1, 1LL << 30);
    if ((s = ensure(ctx, &ctx->rb.d_big, ctx->rb.big_bytes, (size_t)64 * big_cap * kRecDoubles * sizeof(double))) != BL_OK)
        return s;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, ctx->rb.d_ovf_count, 0, 1);
    HIPCHK(ctx, hipGetLastError());
    if ((s = upload_cuts(ctx)) != BL_OK) return s;
    // each output's plasma constants (no host allocation for one output)
    PlasmaParams pp1;
    std::vector<PlasmaParams> ppv;
    PlasmaParams *pps = &pp1;
    if (tr_plasmas && n_tr > 1) {
        ppv.resize(n_tr);
        pps = ppv.data();
    }
    const int n_pl = tr_plasmas ? n_tr : 1;
    for (int f = 0; f < n_pl; ++f) pps[f] = plasma_params(ctx, pls[f], grid->g, sts[0]->mass_msun);
    if ((s = upload_nth(ctx, n_pl, pls, pps)) != BL_OK) return s;
    bool nth = false;
    for (int f = 0; f < n_pl; ++f) nth = nth || pps[f].nonthermal;
    if (nth && (batch || ctx->has_cuts || avg))
        return fail(ctx, BL_E_UNSUPPORTED,
                    "nonthermal electrons are rendered by single-image renders without data cuts or averages");
    if (!tr_plasmas && n_tr > 1) {
        ppv.assign(n_tr, pp1);
        pps = ppv.data();
    }
    const PlasmaParams &pp = pps[0];
    TransferParams tp;
    tp.ds_max = integ->ds_max;
    tp.L = kG * sts[0]->mass_msun * kMsun / (kC * kC);
    tp.nu_cam = cams[0]->nu_hz;
    long long nchunk = (total + chunk - 1) / chunk;
    const long long nqueue = 2 * nchunk * n_q;   // one counter (padded to two ints) per transfer launch
    if ((s = ensure(ctx, &ctx->rb.d_queue, ctx->rb.queue_bytes, (size_t)nqueue * sizeof(int))) != BL_OK) return s;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((nqueue + 63) / 64)), dim3(64), 0, ctx->stream, ctx->rb.d_queue, 0,
                       (int)nqueue);
    HIPCHK(ctx, hipGetLastError());
    // the transfer kernel of a plasma (its index in the launch switch) and
    // the waves of it that fit at once
    auto kernel_of = [&](const PlasmaParams &q) {
        const int k = 4 * (batch ? 1 : 0) + 2 * q.polarized + (mixed ? 1 : 0);
        return q.nonthermal ? 16 + k : k + (q.cuts ? 8 : 0);
    };
    auto resident_of = [&](const PlasmaParams &q) {
        const int k = 2 * q.polarized + (mixed ? 1 : 0);
        int per_cu = ctx->blocks_tr[q.nonthermal ? 10 + k : 4 * (batch ? 1 : 0) + k];
        if (t.transfer_waves_per_cu > 0) per_cu = std::min(per_cu, t.transfer_waves_per_cu);
        return per_cu * ctx->cus;
    };
    long long ichunk = 0;
    for (long long start = 0; start < total; start += chunk, ++ichunk) {
        int count = (int)std::min(chunk, total - start);
        dim3 grd((count + 63) / 64), blk(64);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, ctx->rb.ext.count, 0, 1);
        hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, ctx->stream, ctx->rb.ext.of, -1,
                           count);
        if (opt.per_chunk_overflow && start > 0)
            hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, ctx->rb.d_ovf_count, 0, 1);
        {
            TimedLaunch tl(ctx, BL_K_GEODESIC);
            if (learned) {
                dim3 lg((count + 255) / 256), lb(256);
                if (batch)
                    hipLaunchKernelGGL((k_geodesic_learned<true, true>), lg, lb, 0, ctx->stream, P, B, start, count,
                                       ctx->d_step_pk, ctx->d_step_tail, ctx->rb.d_rec, ctx->rb.d_meta, ctx->rb.d_nacc,
                                       ctx->rb.d_work, ctx->rb.ext, ctx->rb.d_ovf_count, ctx->rb.d_ovf_list);
                else
                    hipLaunchKernelGGL((k_geodesic_learned<true, false>), lg, lb, 0, ctx->stream, P, B, start, count,
                                       ctx->d_step_pk, ctx->d_step_tail, ctx->rb.d_rec, ctx->rb.d_meta, ctx->rb.d_nacc,
                                       ctx->rb.d_work, ctx->rb.ext, ctx->rb.d_ovf_count, ctx->rb.d_ovf_list);
            } else if (batch) {
                hipLaunchKernelGGL((k_geodesic<true, true>), grd, blk, 0, ctx->stream, P, B, start, count, ctx->rb.d_rec,
                                   ctx->rb.d_meta, ctx->rb.d_nacc, ctx->rb.d_work, ctx->rb.ext, ctx->rb.d_ovf_count, ctx->rb.d_ovf_list,
                                   nullptr);
            } else {
                hipLaunchKernelGGL((k_geodesic<true, false>), grd, blk, 0, ctx->stream, P, B, start, count,
                                   ctx->rb.d_rec, ctx->rb.d_meta, ctx->rb.d_nacc, ctx->rb.d_work, ctx->rb.ext, ctx->rb.d_ovf_count,
                                   ctx->rb.d_ovf_list,
                                   nullptr);
            }
        }
        HIPCHK(ctx, hipGetLastError());
        {
            TimedLaunch tl(ctx, BL_K_SETUP);
            const unsigned nb = (unsigned)((count + 255) / 256);
            hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(kOrderBins), 0, ctx->stream, ctx->rb.d_hist, 0, kOrderBins);
            hipLaunchKernelGGL(k_order_hist, dim3(nb), dim3(256), 0, ctx->stream, ctx->rb.d_work, count, ctx->rb.d_hist);
            hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBins), 0, ctx->stream, ctx->rb.d_hist);
            hipLaunchKernelGGL(k_order_scatter, dim3(nb), dim3(256), 0, ctx->stream, ctx->rb.d_work, count, ctx->rb.d_hist,
                               ctx->rb.d_order);
        }
        HIPCHK(ctx, hipGetLastError());
        for (int f = 0; f < n_tr; ++f) {
            // output f of a multi-output render: its image table entry
            // (outputs, camera frequency), its plasma and its own queue counter
            Batch Bf = B;
            Bf.imgs = B.imgs + f;
            TransferParams tpf = tp;
            tpf.nu_cam = cams[f]->nu_hz;
            const PlasmaParams &pp = pps[f];
            TimedLaunch tl(ctx, BL_K_TRANSFER);
            int *q = ctx->rb.d_queue + 2 * (ichunk * n_q + f);
            dim3 pg(std::min<int>(grd.x, resident_of(pp)));
            switch (kernel_of(pp)) {
            case 16: launch_transfer<false, double, false, false, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 17: launch_transfer<false, float, false, false, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 18: launch_transfer<true, double, false, false, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 19: launch_transfer<true, float, false, false, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 0: launch_transfer<false, double, false, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 1: launch_transfer<false, float, false, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 2: launch_transfer<true, double, false, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 3: launch_transfer<true, float, false, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 4: launch_transfer<false, double, true, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 5: launch_transfer<false, float, true, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 6: launch_transfer<true, double, true, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 7: launch_transfer<true, float, true, false>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 8: launch_transfer<false, double, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 9: launch_transfer<false, float, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 10: launch_transfer<true, double, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 11: launch_transfer<true, float, false, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 12: launch_transfer<false, double, true, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 13: launch_transfer<false, float, true, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            case 14: launch_transfer<true, double, true, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            default: launch_transfer<true, float, true, true>(ctx, pg, P, Bf, grid->g, pp, tpf, start, count, t.refill_min, q); break;
            }
            HIPCHK(ctx, hipGetLastError());
        }
        if (avg) {
            // the averages pass: the unpolarized walk over the same records
            // (j_I and alpha_I are those of the polarized coefficients)
            PlasmaParams pa = pp;
            pa.polarized = 0;
            TimedLaunch tl(ctx, BL_K_TRANSFER);
            int *q = ctx->rb.d_queue + 2 * (ichunk * n_q + n_tr);
            dim3 pg(std::min<int>(grd.x, ctx->blocks_tr[mixed ? 9 : 8] * ctx->cus));
            switch ((mixed ? 1 : 0) + (pp.cuts ? 2 : 0)) {
            case 0: launch_transfer<false, double, false, false, true>(ctx, pg, P, B, grid->g, pa, tp, start, count, t.refill_min, q); break;
            case 1: launch_transfer<false, float, false, false, true>(ctx, pg, P, B, grid->g, pa, tp, start, count, t.refill_min, q); break;
            case 2: launch_transfer<false, double, false, true, true>(ctx, pg, P, B, grid->g, pa, tp, start, count, t.refill_min, q); break;
            default: launch_transfer<false, float, false, true, true>(ctx, pg, P, B, grid->g, pa, tp, start, count, t.refill_min, q); break;
            }
            HIPCHK(ctx, hipGetLastError());
        }
        if (opt.per_chunk_overflow)
            if ((s = overflow_all(ctx, B, P, grid, pps, tp, cams, n_tr, mixed, big_cap)) != BL_OK) return s;
    }
    if (avg) {
        PlasmaParams pa = pp;
        pa.polarized = 0;
        TimedLaunch tl(ctx, BL_K_OVERFLOW);
        switch ((mixed ? 1 : 0) + (pp.cuts ? 2 : 0)) {
        case 0: launch_overflow<false, double, false, true>(ctx, P, B, grid->g, pa, tp, big_cap); break;
        case 1: launch_overflow<false, float, false, true>(ctx, P, B, grid->g, pa, tp, big_cap); break;
        case 2: launch_overflow<false, double, true, true>(ctx, P, B, grid->g, pa, tp, big_cap); break;
        default: launch_overflow<false, float, true, true>(ctx, P, B, grid->g, pa, tp, big_cap); break;
        }
        HIPCHK(ctx, hipGetLastError());
    }
    if (!opt.per_chunk_overflow)
        if ((s = overflow_all(ctx, B, P, grid, pps, tp, cams, n_tr, mixed, big_cap)) != BL_OK) return s;
    if (n_freq > 1) {
        // the geodesic maps (dt, s, lambda and n_acc, n_rej, status) were
        // written into the first frequency's aux
        const size_t NN = (size_t)cams[0]->n * cams[0]->n;
        for (int f = 1; f < n_freq; ++f) {
            HIPCHK(ctx, hipMemcpyAsync(auxs[f] + BL_AUX_DT * NN, auxs[0] + BL_AUX_DT * NN, 3 * NN * sizeof(double),
                                       hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(auxs[f] + BL_AUX_NACC * NN, auxs[0] + BL_AUX_NACC * NN,
                                       3 * NN * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    return BL_OK;
}

// Adaptive render: the root level's blocks, then level by level the children
// of the blocks the criteria flag, each level as one batched render of its
// blocks (every block a B x B sub-image of the level's N 2^l image).
bl_status adaptive_impl(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st, const bl_integrator *integ,
                        const bl_grid *grid, const bl_plasma *plasma, const bl_mode *mode, const bl_adaptive *ad,
                        int32_t max_blocks, int32_t *blocks_out, double *image_out, double *aux_out,
                        int32_t *counts_out) {
    bl_status s;
    if ((s = check_camera(ctx, cam)) != BL_OK) return s;
    const int B = ad->block_n, N = cam->n;
    if (B < 1 || N % B != 0) return fail(ctx, BL_E_INVALID_ARG, "block_n must divide the camera's n");
    if (ad->max_level < 0 || ad->max_level > 20 || ((long long)N << ad->max_level) > (1LL << 20))
        return fail(ctx, BL_E_INVALID_ARG, "need 0 <= max_level and n 2^max_level <= 2^20");
    if (ad->n_regions < 0 || ad->n_regions > BL_ADAPT_MAX_REGIONS)
        return fail(ctx, BL_E_INVALID_ARG, "n_regions must be 0 .. BL_ADAPT_MAX_REGIONS");
    if (!(ad->frac > 0.0 && ad->frac <= 1.0)) return fail(ctx, BL_E_INVALID_ARG, "frac must lie in (0, 1]");
    for (int c = 0; c < 5; ++c) {
        if (ad->use[c] != 0 && ad->use[c] != 1) return fail(ctx, BL_E_INVALID_ARG, "use[] entries must be 0 or 1");
        if (ad->use[c] && std::isnan(ad->thr[c])) return fail(ctx, BL_E_INVALID_ARG, "NaN threshold");
    }
    for (int r = 0; r < ad->n_regions; ++r)
        for (int q = 0; q < 5; ++q)
            if (std::isnan(ad->region[r][q])) return fail(ctx, BL_E_INVALID_ARG, "NaN region bound");
    if (max_blocks < 1 || !blocks_out || !image_out || !aux_out || !counts_out)
        return fail(ctx, BL_E_INVALID_ARG, "need max_blocks >= 1 and non-NULL outputs");
    for (int l = 0; l <= ad->max_level; ++l) counts_out[l] = 0;
    bl_tuning t = ctx->tuning;
    if (t.tile_w > 0 && (B % t.tile_w != 0 || B % t.tile_h != 0)) t.tile_w = t.tile_h = 0;   // row-major blocks
    RefineParams rp{};
    rp.b = B;
    rp.n_root = N;
    rp.n_regions = ad->n_regions;
    for (int c = 0; c < 5; ++c) {
        rp.use[c] = ad->use[c];
        rp.thr[c] = ad->thr[c];
    }
    rp.frac = ad->frac;
    rp.width = cam->width;
    for (int r = 0; r < ad->n_regions; ++r)
        for (int q = 0; q < 5; ++q) rp.region[r][q] = ad->region[r][q];
    std::vector<int> blk;
    for (int by = 0; by < N / B; ++by)
        for (int bx = 0; bx < N / B; ++bx) blk.insert(blk.end(), {0, bx, by});
    const size_t img_sz = (size_t)4 * B * B, aux_sz = (size_t)BL_NAUX * B * B;
    long long off = 0;
    for (int level = 0; level <= ad->max_level && !blk.empty(); ++level) {
        const int nl = (int)(blk.size() / 3);
        if (off + nl > max_blocks)
            return fail(ctx, BL_E_UNSUPPORTED, "max_blocks is too small for level " + std::to_string(level));
        std::vector<bl_camera> cams(nl, *cam);
        std::vector<const bl_camera *> cp(nl);
        std::vector<const bl_spacetime *> sp(nl, st);
        std::vector<double *> ims(nl), axs(nl);
        std::vector<int> sub(3 * (size_t)nl);
        for (int k = 0; k < nl; ++k) {
            cams[k].n = B;
            cp[k] = &cams[k];
            ims[k] = image_out + (size_t)(off + k) * img_sz;
            axs[k] = aux_out + (size_t)(off + k) * aux_sz;
            sub[3 * k] = N << level;
            sub[3 * k + 1] = blk[3 * k + 1] * B;
            sub[3 * k + 2] = blk[3 * k + 2] * B;
        }
        if ((s = render_images(ctx, nl, cp.data(), sp.data(), ims.data(), axs.data(), integ, grid, plasma, mode, t,
                               true, 0, nullptr, sub.data())) != BL_OK)
            return s;
        // the level's block list; blk must stay alive until the stream has
        // passed this copy: the guard waits for the stream on every return
        // (the error returns included) and blk is only replaced after the
        // synchronisations below
        struct StreamWait {
            hipStream_t st;
            ~StreamWait() { (void)hipStreamSynchronize(st); }
        } wait_copy{ctx->stream};
        HIPCHK(ctx, hipMemcpyAsync(blocks_out + 3 * off, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice,
                                   ctx->stream));
        counts_out[level] = nl;
        if (level < ad->max_level) {
            if ((s = ensure(ctx, &ctx->d_refine, ctx->refine_bytes, (size_t)nl * sizeof(int))) != BL_OK) return s;
            rp.level = level;
            hipLaunchKernelGGL(k_refine, dim3((unsigned)nl), dim3(64), 0, ctx->stream, rp,
                               (const int *)(blocks_out + 3 * off), (const double *)ims[0], nl, ctx->d_refine);
            HIPCHK(ctx, hipGetLastError());
            std::vector<int> flags(nl);
            HIPCHK(ctx, hipMemcpyAsync(flags.data(), ctx->d_refine, (size_t)nl * sizeof(int), hipMemcpyDeviceToHost,
                                       ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            std::vector<int> next;
            for (int k = 0; k < nl; ++k)
                if (flags[k])
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx)
                            next.insert(next.end(), {level + 1, 2 * blk[3 * k + 1] + dx, 2 * blk[3 * k + 2] + dy});
            blk.swap(next);
        } else {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));   // the host block list was read by the copy
        }
        off += nl;
    }
    return BL_OK;
}

bl_status render_batch_impl(bl_context *ctx, int32_t n_images, const bl_image_desc *images,
                            const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                            const bl_mode *mode, const bl_tuning &t) {
    if (n_images < 1 || !images) return fail(ctx, BL_E_INVALID_ARG, "need n_images >= 1 and an image array");
    std::vector<const bl_camera *> cams(n_images);
    std::vector<const bl_spacetime *> sts(n_images);
    std::vector<double *> ims(n_images), auxs(n_images);
    for (int k = 0; k < n_images; ++k) {
        cams[k] = &images[k].cam;
        sts[k] = &images[k].st;
        ims[k] = images[k].image_out;
        auxs[k] = images[k].aux_out;
        if (images[k].st.mass_msun != images[0].st.mass_msun)
            return fail(ctx, BL_E_UNSUPPORTED, "all images of a batch must share mass_msun");
    }
    return render_images(ctx, n_images, cams.data(), sts.data(), ims.data(), auxs.data(), integ, grid, plasma, mode, t,
                         true);
}

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

int bl_abi_version(void) { return BLGPU_ABI_VERSION; }

bl_status bl_create(int device, void *hip_stream, bl_context **out) {
    if (!out) return BL_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return BL_E_DEVICE;
    bl_context *ctx = new (std::nothrow) bl_context();
    if (!ctx) return BL_E_OOM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return BL_E_DEVICE;
    }
    // step-record workspace per chunk: 128 GiB, at most half the free memory
    // (a 1024^2 image with 512-record slots, 103 GB, then runs as one chunk)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
        ctx->ws_limit = std::max<size_t>((size_t)64 << 20, std::min(ctx->ws_limit, free_b / 2));
    // what every render reuses: the upload event and room for one image
    // descriptor on the host (so that a single-image render allocates nothing
    // on the host once the context exists)
    if (hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming) != hipSuccess) {
        delete ctx;
        return BL_E_DEVICE;
    }
    ctx->h_imgs.reserve(1);
    ctx->h_ray0.reserve(1);
    // this device's address of the static scratch array, looked up once per
    // device with the device current (a failure leaves it NULL: only the
    // allocation-free render needs it, and it reports the failure)
    {
        static std::mutex mu;
        static std::vector<void *> addr;
        static std::vector<char> done;
        std::lock_guard<std::mutex> lock(mu);
        if ((int)addr.size() < ndev) {
            addr.resize(ndev, nullptr);
            done.resize(ndev, 0);
        }
        if (!done[device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) addr[device] = ptr;
            else (void)hipGetLastError();
            done[device] = 1;
        }
        ctx->scratch = addr[device];
    }
    *out = ctx;
    return BL_OK;
}

void bl_destroy(bl_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    (void)hipFree(ctx->rb.d_imgs);
    (void)hipFree(ctx->d_step_pk);
    (void)hipFree(ctx->d_step_tail);
    (void)hipFree(ctx->d_mlp_pk);
    (void)hipFree(ctx->d_mlp_tail);
    (void)hipFree(ctx->d_mlp_gpart);
    (void)hipFree(ctx->d_mlp_slices);
    (void)hipFree(ctx->d_mlp_sloss);
    (void)hipFree(ctx->d_mlp_lpart);
    (void)hipFree(ctx->d_mlp_grad);
    (void)hipFree(ctx->d_mlp_m);
    (void)hipFree(ctx->d_mlp_v);
    (void)hipFree(ctx->d_mlp_acc);
    (void)hipFree(ctx->d_mlp_stats);
    (void)hipFree(ctx->d_mlp_rows);
    (void)hipFree(ctx->d_log_count);
    (void)hipFree(ctx->rb.d_ray0);
    if (ctx->upload_done) (void)hipEventDestroy(ctx->upload_done);
    (void)hipFree(ctx->rb.d_rec);
    (void)hipFree(ctx->rb.d_meta);
    (void)hipFree(ctx->rb.d_nacc);
    (void)hipFree(ctx->rb.d_work);
    (void)hipFree(ctx->rb.d_order);
    (void)hipFree(ctx->rb.ext.count);
    (void)hipFree(ctx->rb.ext.of);
    (void)hipFree(ctx->rb.ext.rec);
    (void)hipFree(ctx->rb.d_hist);
    (void)hipFree(ctx->rb.d_ovf_count);
    (void)hipFree(ctx->rb.d_ovf_list);
    (void)hipFree(ctx->rb.d_big);
    (void)hipFree(ctx->rb.d_queue);
    (void)hipFree(ctx->rb.d_ends);
    (void)hipFree(ctx->rb.d_cuts);
    (void)hipFree(ctx->d_refine);
    delete ctx;
}

const char *bl_last_error(const bl_context *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

bl_status bl_grid_create(bl_context *ctx, const bl_grid_desc *d, bl_grid **out) {
    if (!ctx || !d || !out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (d->n_blocks < 1 || d->bnx < 2 || d->bny < 2 || d->bnz < 2)
        return fail(ctx, BL_E_INVALID_ARG, "need n_blocks >= 1 and at least 2 cells per block axis");
    if (!d->bounds || !d->prims) return fail(ctx, BL_E_INVALID_ARG, "bounds and prims must be non-NULL");
    if (d->dtype != 0 && d->dtype != 1) return fail(ctx, BL_E_INVALID_ARG, "dtype must be 0 (f64) or 1 (f32)");
    if (!(d->rho_unit > 0.0)) return fail(ctx, BL_E_INVALID_ARG, "rho_unit must be positive");
    if (((uintptr_t)d->prims & 15) != 0) return fail(ctx, BL_E_INVALID_ARG, "prims must be 16-byte aligned");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int nb = d->n_blocks;
    DevGrid g{};
    double bb[6] = {1e300, -1e300, 1e300, -1e300, 1e300, -1e300};
    double tb[3] = {1e300, 1e300, 1e300};
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < 3; ++c) {
            double lo = d->bounds[6 * b + 2 * c], hi = d->bounds[6 * b + 2 * c + 1];
            if (!(hi > lo)) return fail(ctx, BL_E_INVALID_ARG, "block bounds must satisfy x1 > x0");
            bb[2 * c] = std::min(bb[2 * c], lo);
            bb[2 * c + 1] = std::max(bb[2 * c + 1], hi);
            tb[c] = std::min(tb[c], hi - lo);
        }
    long long tn[3];
    for (int c = 0; c < 3; ++c) {
        double q = (bb[2 * c + 1] - bb[2 * c]) / tb[c];
        tn[c] = std::llround(q);
        if (std::fabs(q - (double)tn[c]) > 1e-9 * q || tn[c] < 1)
            return fail(ctx, BL_E_UNSUPPORTED, "blocks are not aligned to a lattice of the smallest block size");
    }
    if (tn[0] * tn[1] * tn[2] > (1LL << 24)) return fail(ctx, BL_E_UNSUPPORTED, "block lattice larger than 2^24 cells");
    // per lattice cell: origin, inverse cell sizes and first cell of the
    // covering block (slot 6; -1 = none), 8 doubles
    std::vector<double> table((size_t)(tn[0] * tn[1] * tn[2]) * 8, 0.0);
    for (size_t t = 0; t < table.size(); t += 8) table[t + 6] = -1.0;
    const int nn[3] = {d->bnx, d->bny, d->bnz};
    const double cells = (double)d->bnx * d->bny * d->bnz;
    for (int b = 0; b < nb; ++b) {
        long long lo[3], hi[3];
        double ent[8];
        for (int c = 0; c < 3; ++c) {
            double x0 = d->bounds[6 * b + 2 * c], x1 = d->bounds[6 * b + 2 * c + 1];
            double ql = (x0 - bb[2 * c]) / tb[c], qh = (x1 - bb[2 * c]) / tb[c];
            lo[c] = std::llround(ql);
            hi[c] = std::llround(qh);
            if (std::fabs(ql - lo[c]) > 1e-9 * (1.0 + ql) || std::fabs(qh - hi[c]) > 1e-9 * (1.0 + qh))
                return fail(ctx, BL_E_UNSUPPORTED, "block not aligned to the block lattice");
            ent[c] = x0;
            ent[3 + c] = nn[c] / (x1 - x0);
        }
        ent[6] = (double)b * cells;
        ent[7] = 0.0;
        for (long long k = lo[2]; k < hi[2]; ++k)
            for (long long j = lo[1]; j < hi[1]; ++j)
                for (long long i = lo[0]; i < hi[0]; ++i) {
                    double *t = &table[(size_t)((k * tn[1] + j) * tn[0] + i) * 8];
                    if (t[6] >= 0.0) return fail(ctx, BL_E_INVALID_ARG, "blocks overlap");
                    for (int m = 0; m < 8; ++m) t[m] = ent[m];
                }
    }
    bl_grid *gr = new (std::nothrow) bl_grid();
    if (!gr) return fail(ctx, BL_E_OOM, "host allocation failed");
    gr->ctx = ctx;
    if (hipMalloc((void **)&gr->d_table, table.size() * sizeof(double)) != hipSuccess) {
        delete gr;
        return fail(ctx, BL_E_OOM, "device allocation of the block table failed");
    }
    HIPCHK(ctx, hipMemcpy(gr->d_table, table.data(), table.size() * sizeof(double), hipMemcpyHostToDevice));
    g.prims = d->prims;
    g.table = gr->d_table;
    for (int c = 0; c < 6; ++c) g.bb[c] = bb[c];
    for (int c = 0; c < 3; ++c) {
        g.t0[c] = bb[2 * c];
        g.tb[c] = tb[c];
        g.itb[c] = 1.0 / tb[c];
        g.tn[c] = (int)tn[c];
    }
    g.nb = nb;
    g.bnx = d->bnx;
    g.bny = d->bny;
    g.bnz = d->bnz;
    g.dtype = d->dtype;
    g.rho_unit = d->rho_unit;
    gr->g = g;
    *out = gr;
    return BL_OK;
}

void bl_grid_destroy(bl_grid *gr) {
    if (!gr) return;
    if (gr->ctx) (void)hipSetDevice(gr->ctx->device);
    (void)hipFree(gr->d_table);
    delete gr;
}

bl_status bl_camera_rays(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st, double *state_out,
                         double *norm_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    bl_status s;
    if ((s = check_camera(ctx, cam)) != BL_OK || (s = check_spacetime(ctx, st)) != BL_OK) return s;
    if (!state_out || !norm_out) return fail(ctx, BL_E_INVALID_ARG, "output pointers must be non-NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_tuning t = ctx->tuning;
    t.tile_w = t.tile_h = 0;
    Batch B;
    long long total = 0;
    if ((s = upload_one(ctx, cam, st, nullptr, nullptr, t, B, total)) != BL_OK) return s;
    long long NN = (long long)cam->n * cam->n;
    hipLaunchKernelGGL(k_camera_rays, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, ctx->stream, ctx->rb.d_imgs,
                       state_out, norm_out);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_trace_geodesics(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, double *state_out, double *aux_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    bl_status s;
    if ((s = check_camera(ctx, cam)) != BL_OK || (s = check_spacetime(ctx, st)) != BL_OK ||
        (s = check_integrator(ctx, integ)) != BL_OK)
        return s;
    if (!state_out || !aux_out) return fail(ctx, BL_E_INVALID_ARG, "output pointers must be non-NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_tuning t = ctx->tuning;
    t.tile_w = t.tile_h = 0;
    Batch B;
    long long total = 0;
    if ((s = upload_one(ctx, cam, st, nullptr, aux_out, t, B, total)) != BL_OK) return s;
    GeoParams P = geo_params(cam, st, integ);
    const long long chunk = 1 << 20;
    for (long long start = 0; start < total; start += chunk) {
        int count = (int)std::min(chunk, total - start);
        TimedLaunch tl(ctx, BL_K_GEODESIC);
        hipLaunchKernelGGL((k_geodesic<false, false>), dim3((count + 63) / 64), dim3(64), 0, ctx->stream, P, B, start,
                           count, nullptr, nullptr, nullptr, nullptr, ExtQueue{}, nullptr, nullptr, state_out);
        HIPCHK(ctx, hipGetLastError());
    }
    return BL_OK;
}

bl_status bl_render(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st, const bl_integrator *integ,
                    const bl_grid *grid, const bl_plasma *plasma, const bl_mode *mode, double *image_out,
                    double *aux_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    return render_images(ctx, 1, &cam, &st, &image_out, &aux_out, integ, grid, plasma, mode, ctx->tuning, false);
}

bl_status bl_render_noalloc(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                            const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                            const bl_mode *mode, double *image_out, double *aux_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st || !integ || !grid || !plasma) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    if (!ctx->scratch) return fail(ctx, BL_E_DEVICE, "the static scratch array has no device address on this device");
    bl_status s;
    if ((s = check_camera(ctx, cam)) != BL_OK || (s = check_integrator(ctx, integ)) != BL_OK) return s;
    if (integ->max_steps > kNoAllocMaxSteps)
        return fail(ctx, BL_E_INVALID_ARG,
                    "the allocation-free render takes max_steps <= " + std::to_string(kNoAllocMaxSteps));
    const bool mixed = mode && mode->precision == 1;
    // every buffer the render needs, for a chunk of `chunk` rays: per ray the
    // record slot, order key, queue entry, end state and overflow entry; fixed:
    // the image descriptor, extension slots, sort bins, overflow buffer,
    // queue counters (two ints per chunk) and the cut limits, each rounded up
    // to 256 bytes
    GeoParams P = geo_params(cam, st, integ);
    const size_t rec_per_ray = (size_t)P.cap * kRecDoubles * sizeof(double);
    const size_t per_ray = rec_per_ray + 2 * sizeof(double) + 5 * sizeof(int) +
                           (size_t)kRayEnd * (mixed ? sizeof(float) : sizeof(double));
    const long long cap_rec = std::min<long long>(2048, P.max_steps + 1);
    const long long big_cap = P.max_steps + 1;
    const long long total = image_rays(cam->n, ctx->tuning);
    const size_t fixed = 20 * 256 + sizeof(ImgDev) + sizeof(long long) + sizeof(int) +
                         (cap_rec > P.cap ? (size_t)kNoAllocExtSlots * cap_rec * kRecDoubles * sizeof(double) : 0) +
                         (size_t)kOrderBins * sizeof(int) + sizeof(int) +
                         (size_t)64 * big_cap * kRecDoubles * sizeof(double) + sizeof(CutParams) +
                         (size_t)2 * ((total + 63) / 64 + 1) * sizeof(int);
    if (fixed + 64 * per_ray > kScratchBytes)
        return fail(ctx, BL_E_UNSUPPORTED,
                    "the allocation-free render's scratch (" + std::to_string(kScratchBytes) +
                        " bytes) does not hold one wave of rays: lower record_cap or max_steps");
    long long chunk = (long long)((kScratchBytes - fixed) / per_ray);
    chunk = std::min(chunk - chunk % 64, (total + 63) / 64 * 64);
    bl_tuning t = ctx->tuning;
    t.chunk_rays = chunk;
    RenderOpts opt;
    opt.ext_slots = kNoAllocExtSlots;
    opt.per_chunk_overflow = true;
    // swap in an empty buffer set carved from the scratch; no timing events
    Arena arena;
    arena.base = static_cast<char *>(ctx->scratch);
    arena.cap = kScratchBytes;
    RenderBuffers saved = ctx->rb;
    const bool prof = ctx->prof;
    ctx->rb = RenderBuffers{};
    ctx->arena = &arena;
    ctx->prof = false;
    s = render_images(ctx, 1, &cam, &st, &image_out, &aux_out, integ, grid, plasma, mode, t, false, 0, nullptr,
                      nullptr, opt);
    ctx->rb = saved;
    ctx->arena = nullptr;
    ctx->prof = prof;
    return s;
}

bl_status bl_render_averages(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                             const bl_mode *mode, double *image_out, double *aux_out, double *avg_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st || !avg_out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    return render_images(ctx, 1, &cam, &st, &image_out, &aux_out, integ, grid, plasma, mode, ctx->tuning, false, 0,
                         avg_out);
}

bl_status bl_render_adaptive(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                             const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                             const bl_mode *mode, const bl_adaptive *adaptive, int32_t max_blocks,
                             int32_t *blocks_out, double *image_out, double *aux_out, int32_t *level_counts_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st || !adaptive) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    return adaptive_impl(ctx, cam, st, integ, grid, plasma, mode, adaptive, max_blocks, blocks_out, image_out, aux_out,
                         level_counts_out);
}

bl_status bl_set_cuts(bl_context *ctx, const bl_cuts *cuts) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cuts) {
        ctx->has_cuts = false;
        return BL_OK;
    }
    const double *lims[8] = {cuts->rho, cuts->ne, cuts->p, cuts->theta_e, cuts->b, cuts->sigma, cuts->beta_inv,
                             cuts->r};
    for (int k = 0; k < 8; ++k)
        if (std::isnan(lims[k][0]) || std::isnan(lims[k][1]))
            return fail(ctx, BL_E_INVALID_ARG, "cut limits must not be NaN");
    if (cuts->plane < -1 || cuts->plane > 1) return fail(ctx, BL_E_INVALID_ARG, "plane must be -1, 0 or 1");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(cuts->plane_origin[i]) || !std::isfinite(cuts->plane_normal[i]))
            return fail(ctx, BL_E_INVALID_ARG, "plane origin and normal must be finite");
    ctx->cuts = *cuts;
    ctx->has_cuts = true;
    return BL_OK;
}

bl_status bl_render_multifreq(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st,
                              const bl_integrator *integ, const bl_grid *grid, const bl_plasma *plasma,
                              const bl_mode *mode, int32_t n_freq, const double *nu_hz, double *const *images_out,
                              double *const *aux_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st || !nu_hz || !images_out || !aux_out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    if (n_freq < 1 || n_freq > 4096) return fail(ctx, BL_E_INVALID_ARG, "need 1 <= n_freq <= 4096");
    std::vector<bl_camera> cams(n_freq, *cam);
    std::vector<const bl_camera *> cp(n_freq);
    std::vector<const bl_spacetime *> sp(n_freq, st);
    for (int f = 0; f < n_freq; ++f) {
        if (!(nu_hz[f] > 0.0) || !std::isfinite(nu_hz[f]))
            return fail(ctx, BL_E_INVALID_ARG, "frequencies must be positive and finite");
        cams[f].nu_hz = nu_hz[f];
        cp[f] = &cams[f];
    }
    return render_images(ctx, 1, cp.data(), sp.data(), images_out, aux_out, integ, grid, plasma, mode, ctx->tuning,
                         false, n_freq);
}

bl_status bl_render_models(bl_context *ctx, const bl_camera *cam, const bl_spacetime *st, const bl_integrator *integ,
                          const bl_grid *grid, int32_t n_out, const double *nu_hz, const bl_plasma *plasmas,
                          const bl_mode *mode, double *const *images_out, double *const *aux_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!cam || !st || !plasmas || !images_out || !aux_out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    if (n_out < 1 || n_out > 4096) return fail(ctx, BL_E_INVALID_ARG, "need 1 <= n_out <= 4096");
    std::vector<bl_camera> cams(n_out, *cam);
    std::vector<const bl_camera *> cp(n_out);
    std::vector<const bl_spacetime *> sp(n_out, st);
    std::vector<const bl_plasma *> pl(n_out);
    for (int f = 0; f < n_out; ++f) {
        if (nu_hz) {
            if (!(nu_hz[f] > 0.0) || !std::isfinite(nu_hz[f]))
                return fail(ctx, BL_E_INVALID_ARG, "frequencies must be positive and finite");
            cams[f].nu_hz = nu_hz[f];
        }
        cp[f] = &cams[f];
        pl[f] = &plasmas[f];
    }
    return render_images(ctx, 1, cp.data(), sp.data(), images_out, aux_out, integ, grid, &plasmas[0], mode,
                         ctx->tuning, false, n_out, nullptr, nullptr, RenderOpts(), pl.data());
}

bl_status bl_render_batch(bl_context *ctx, int32_t n_images, const bl_image_desc *images, const bl_integrator *integ,
                          const bl_grid *grid, const bl_plasma *plasma, const bl_mode *mode,
                          const bl_tuning *tuning) {
    if (!ctx) return BL_E_INVALID_ARG;
    return render_batch_impl(ctx, n_images, images, integ, grid, plasma, mode, tuning ? *tuning : ctx->tuning);
}

bl_status bl_set_tuning(bl_context *ctx, const bl_tuning *tuning) {
    if (!ctx) return BL_E_INVALID_ARG;
    bl_status s = check_tuning(ctx, tuning);
    if (s != BL_OK) return s;
    ctx->tuning = *tuning;
    return BL_OK;
}

bl_status bl_get_tuning(const bl_context *ctx, bl_tuning *tuning_out) {
    if (!ctx || !tuning_out) return BL_E_INVALID_ARG;
    *tuning_out = ctx->tuning;
    return BL_OK;
}

bl_status bl_autotune(bl_context *ctx, int32_t n_images, const bl_image_desc *images, const bl_integrator *integ,
                      const bl_grid *grid, const bl_plasma *plasma, const bl_mode *mode, int32_t max_trials,
                      bl_tuning *best_out, double *best_ms_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (max_trials < 1) return fail(ctx, BL_E_INVALID_ARG, "max_trials must be >= 1");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipEvent_t ea = nullptr, eb = nullptr;
    HIPCHK(ctx, hipEventCreate(&ea));
    if (hipEventCreate(&eb) != hipSuccess) {
        (void)hipEventDestroy(ea);
        return fail(ctx, BL_E_DEVICE, "hipEventCreate failed");
    }
    int trials = 0;
    bl_status err = BL_OK;
    // one untimed render (allocations, first-touch) and one timed render
    auto timed = [&](const bl_tuning &t, double &ms) -> bl_status {
        bl_status s = render_batch_impl(ctx, n_images, images, integ, grid, plasma, mode, t);
        if (s != BL_OK) return s;
        if (hipEventRecord(ea, ctx->stream) != hipSuccess) return fail(ctx, BL_E_DEVICE, "hipEventRecord failed");
        s = render_batch_impl(ctx, n_images, images, integ, grid, plasma, mode, t);
        if (s != BL_OK) return s;
        if (hipEventRecord(eb, ctx->stream) != hipSuccess || hipEventSynchronize(eb) != hipSuccess)
            return fail(ctx, BL_E_DEVICE, "event timing failed");
        float f = 0.0f;
        if (hipEventElapsedTime(&f, ea, eb) != hipSuccess) return fail(ctx, BL_E_DEVICE, "hipEventElapsedTime failed");
        ms = f;
        ++trials;
        return BL_OK;
    };
    bl_tuning best = ctx->tuning;
    double best_ms = 0.0;
    err = timed(best, best_ms);
    if (err == BL_OK) {
        size_t rec_per_ray = (size_t)((integ && integ->record_cap > 0) ? integ->record_cap : kDefaultRecordCap) * kRecDoubles *
                             sizeof(double);
        const long long base = (long long)(ctx->ws_limit / rec_per_ray) / 64 * 64;
        const int occ = std::max(1, ctx->blocks_tr[7]);
        // coordinate search: each knob in turn over its candidates, keeping
        // the rest at the best values so far; a change must gain 1 %
        for (int knob = 0; knob < 5 && err == BL_OK; ++knob) {
            std::vector<bl_tuning> cand;
            bl_tuning c = best;
            if (knob == 0) {
                const int tiles[4][2] = {{0, 0}, {64, 1}, {16, 4}, {8, 8}};
                for (auto &tl : tiles) {
                    c = best;
                    c.tile_w = tl[0];
                    c.tile_h = tl[1];
                    cand.push_back(c);
                }
            } else if (knob == 1) {
                for (int w : {0, std::max(1, occ / 2), 1}) {
                    c = best;
                    c.transfer_waves_per_cu = w;
                    cand.push_back(c);
                }
            } else if (knob == 2) {
                for (int r : {1, 4, 16}) {
                    c = best;
                    c.refill_min = r;
                    cand.push_back(c);
                }
            } else if (knob == 3) {
                for (long long m : {0LL, std::max(64LL, base / 2 / 64 * 64), 2 * base}) {
                    c = best;
                    c.chunk_rays = m;
                    cand.push_back(c);
                }
            } else {
                for (int o : {0, 1}) {
                    c = best;
                    c.order = o;
                    cand.push_back(c);
                }
            }
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                const bl_tuning &t = cand[ci];
                bool seen = std::memcmp(&t, &best, sizeof(bl_tuning)) == 0;
                for (size_t cj = 0; cj < ci && !seen; ++cj)
                    seen = std::memcmp(&t, &cand[cj], sizeof(bl_tuning)) == 0;
                if (seen) continue;
                if (trials >= max_trials) break;
                double ms = 0.0;
                err = timed(t, ms);
                if (err == BL_E_OOM) {   // a workspace this size does not fit: skip the candidate
                    err = BL_OK;
                    continue;
                }
                if (err != BL_OK) break;
                if (ms < 0.99 * best_ms) {
                    best = t;
                    best_ms = ms;
                }
            }
        }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (err != BL_OK) return err;
    ctx->tuning = best;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return BL_OK;
}

// ------------------------------------------------------------ step network
namespace {

bl_status mlp_buffers(bl_context *ctx) {
    bl_status s;
    size_t have = ctx->d_mlp_pk ? (size_t)kPkAll * sizeof(u32x4) : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_pk, have, (size_t)kPkAll * sizeof(u32x4))) != BL_OK) return s;
    have = ctx->d_mlp_tail ? (size_t)kTailN * sizeof(float) : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_tail, have, (size_t)kTailN * sizeof(float))) != BL_OK) return s;
    const size_t np = (size_t)kMlpNParam * sizeof(float);
    have = ctx->d_mlp_grad ? np : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_grad, have, np)) != BL_OK) return s;
    have = ctx->d_mlp_m ? np : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_m, have, np)) != BL_OK) return s;
    have = ctx->d_mlp_v ? np : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_v, have, np)) != BL_OK) return s;
    have = ctx->d_mlp_acc ? 2 * sizeof(double) : 0;
    if ((s = ensure(ctx, &ctx->d_mlp_acc, have, 2 * sizeof(double))) != BL_OK) return s;
    return BL_OK;
}

bl_status mlp_tiles(bl_context *ctx, long long tiles) {
    bl_status s;
    if ((s = ensure(ctx, &ctx->d_mlp_gpart, ctx->mlp_gpart_bytes, (size_t)tiles * kMlpNParam * sizeof(float))) != BL_OK)
        return s;
    const long long slices = (tiles + kMlpSlice - 1) / kMlpSlice;
    if ((s = ensure(ctx, &ctx->d_mlp_slices, ctx->mlp_slices_bytes, (size_t)slices * kMlpNParam * sizeof(double))) !=
        BL_OK)
        return s;
    if ((s = ensure(ctx, &ctx->d_mlp_sloss, ctx->mlp_sloss_bytes, (size_t)slices * sizeof(double))) != BL_OK) return s;
    return ensure(ctx, &ctx->d_mlp_lpart, ctx->mlp_lpart_bytes, (size_t)tiles * sizeof(float));
}

void mlp_pack(bl_context *ctx, const float *model, u32x4 *pk, float *tail) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((kPkAll + 255) / 256), dim3(256), 0, ctx->stream, model, pk, tail);
}

// One pass of k_mlp_fwdbwd + reduction over rows [offset, offset + n_rows) of
// the permutation; adds the summed squared error to d_mlp_acc[0].
bl_status mlp_pass(bl_context *ctx, const float *records, long long n_rows, long long offset, long long mul,
                   long long add, long long n_mod, float inv_n, bool want_grad, float *y_out) {
    const long long tiles = (n_rows + 63) / 64;
    bl_status s = mlp_tiles(ctx, tiles);
    if (s != BL_OK) return s;
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((unsigned)tiles), dim3(64), 0, ctx->stream, ctx->d_mlp_pk, ctx->d_mlp_tail,
                       records, n_rows, offset, mul, add, n_mod, inv_n, want_grad ? 1 : 0, ctx->d_mlp_gpart,
                       ctx->d_mlp_lpart, y_out);
    const int slices = (int)((tiles + kMlpSlice - 1) / kMlpSlice);
    hipLaunchKernelGGL(k_mlp_reduce_slices, dim3(want_grad ? (kMlpNParam + 255) / 256 : 1, (unsigned)slices), dim3(256),
                       0, ctx->stream, ctx->d_mlp_gpart, ctx->d_mlp_lpart, (int)tiles, want_grad ? 1 : 0,
                       ctx->d_mlp_slices, ctx->d_mlp_sloss);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpNParam + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_mlp_slices,
                       ctx->d_mlp_sloss, slices, ctx->d_mlp_grad, ctx->d_mlp_acc, want_grad ? 1 : 0);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bool coprime(unsigned long long a, unsigned long long b) {
    while (b) {
        unsigned long long t = a % b;
        a = b;
        b = t;
    }
    return a == 1;
}

}  // namespace

bl_status bl_steplog(bl_context *ctx, int32_t n_images, const bl_image_desc *images, const bl_integrator *integ,
                     float *records_out, int64_t capacity, int64_t *n_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    bl_status s;
    if ((s = check_integrator(ctx, integ)) != BL_OK) return s;
    if (n_images < 1 || !images || !records_out || capacity < 0 || !n_out)
        return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    std::vector<const bl_camera *> cams(n_images);
    std::vector<const bl_spacetime *> sts(n_images);
    std::vector<double *> ims(n_images), auxs(n_images);
    for (int k = 0; k < n_images; ++k) {
        cams[k] = &images[k].cam;
        sts[k] = &images[k].st;
        ims[k] = images[k].image_out;
        auxs[k] = images[k].aux_out;
        if ((s = check_camera(ctx, cams[k])) != BL_OK || (s = check_spacetime(ctx, sts[k])) != BL_OK) return s;
        if (!auxs[k]) return fail(ctx, BL_E_INVALID_ARG, "aux outputs must be non-NULL");
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_tuning t = ctx->tuning;
    t.order = 0;
    Batch B;
    long long total = 0;
    if ((s = upload_images(ctx, n_images, cams.data(), sts.data(), ims.data(), auxs.data(), t, B, total)) != BL_OK)
        return s;
    size_t have = ctx->d_log_count ? sizeof(unsigned long long) : 0;
    if ((s = ensure(ctx, &ctx->d_log_count, have, sizeof(unsigned long long))) != BL_OK) return s;
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, ctx->stream, (double *)ctx->d_log_count, 0.0, 1);
    GeoParams P = geo_params(cams[0], sts[0], integ);
    StepLog lg{records_out, capacity, ctx->d_log_count};
    const long long chunk = 1 << 20;
    for (long long start = 0; start < total; start += chunk) {
        int count = (int)std::min(chunk, total - start);
        TimedLaunch tl(ctx, BL_K_GEODESIC);
        hipLaunchKernelGGL(k_steplog, dim3((count + 63) / 64), dim3(64), 0, ctx->stream, P, B, start, count, lg);
        HIPCHK(ctx, hipGetLastError());
    }
    unsigned long long cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(&cnt, ctx->d_log_count, sizeof cnt, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *n_out = (int64_t)cnt;
    return BL_OK;
}

bl_status bl_mlp_init(bl_context *ctx, const float *records, int64_t n, int64_t seed, float *model_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!records || n < 1 || !model_out) return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int nblk = 256;
    size_t have = ctx->d_mlp_stats ? (size_t)nblk * kLogRec * 2 * sizeof(double) : 0;
    bl_status s;
    if ((s = ensure(ctx, &ctx->d_mlp_stats, have, (size_t)nblk * kLogRec * 2 * sizeof(double))) != BL_OK) return s;
    hipLaunchKernelGGL(k_mlp_stats, dim3(nblk), dim3(256), 0, ctx->stream, records, (long long)n, ctx->d_mlp_stats);
    hipLaunchKernelGGL(k_mlp_init, dim3((kMlpNModel + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_mlp_stats, nblk,
                       (long long)n, (unsigned long long)seed, model_out);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_mlp_forward_backward(bl_context *ctx, const float *model, const float *records, int64_t n, float *y_out,
                                  float *loss_out, float *grad_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!model || !records || n < 1 || !loss_out || !grad_out) return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_status s;
    if ((s = mlp_buffers(ctx)) != BL_OK) return s;
    mlp_pack(ctx, model, ctx->d_mlp_pk, ctx->d_mlp_tail);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, ctx->stream, ctx->d_mlp_acc, 0.0, 2);
    if ((s = mlp_pass(ctx, records, n, 0, 1, 0, n, 1.0f / (float)n, true, y_out)) != BL_OK) return s;
    HIPCHK(ctx, hipMemcpyAsync(grad_out, ctx->d_mlp_grad, (size_t)kMlpNParam * sizeof(float),
                               hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_mlp_store_loss, dim3(1), dim3(64), 0, ctx->stream, ctx->d_mlp_acc, (double)n, loss_out);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_mlp_train(bl_context *ctx, const float *records, int64_t n, const bl_mlp_hparams *hp, float *model,
                       float *loss_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!records || !hp || !model || !loss_out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    if (hp->epochs < 1 || hp->batch < 64 || hp->batch % 64 != 0 || hp->n_val < 0 || n - hp->n_val < hp->batch ||
        !(hp->lr > 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) || !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) ||
        !(hp->eps > 0.0f))
        return fail(ctx, BL_E_INVALID_ARG, "need epochs >= 1, batch a multiple of 64 with n - n_val >= batch, "
                                           "lr > 0, 0 <= beta < 1, eps > 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_status s;
    if ((s = mlp_buffers(ctx)) != BL_OK) return s;
    const long long n_train = n - hp->n_val, steps = n_train / hp->batch;
    hipLaunchKernelGGL(k_fill_f32, dim3((kMlpNParam + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_mlp_m, 0.0f,
                       kMlpNParam);
    hipLaunchKernelGGL(k_fill_f32, dim3((kMlpNParam + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_mlp_v, 0.0f,
                       kMlpNParam);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, ctx->stream, ctx->d_mlp_acc, 0.0, 2);
    unsigned long long rng = 0x9E3779B97F4A7C15ull ^ (unsigned long long)hp->seed;
    auto next = [&]() {
        rng += 0x9E3779B97F4A7C15ull;
        unsigned long long z = rng;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto affine = [&](unsigned long long m, unsigned long long &mul, unsigned long long &add) {
        mul = 1;
        add = 0;
        if (m > 1) {
            do mul = next() % m; while (mul == 0 || !coprime(mul, m));
            add = next() % m;
        }
    };
    // rows in a fixed pseudo-random order: the held-out rows are the last
    // n_val of it, a scattered subset of the log
    if ((s = ensure(ctx, &ctx->d_mlp_rows, ctx->mlp_rows_bytes, (size_t)n * kLogRec * sizeof(float))) != BL_OK)
        return s;
    {
        unsigned long long mul, add;
        affine((unsigned long long)n, mul, add);
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, records,
                           ctx->d_mlp_rows, (long long)n, (long long)mul, (long long)add);
        HIPCHK(ctx, hipGetLastError());
    }
    records = ctx->d_mlp_rows;
    long long t_step = 0;
    const float b1 = hp->beta1, b2 = hp->beta2;
    for (int ep = 0; ep < hp->epochs; ++ep) {
        // a fresh affine permutation of the training rows per epoch
        unsigned long long mul, add;
        affine((unsigned long long)n_train, mul, add);
        for (long long st = 0; st < steps; ++st) {
            mlp_pack(ctx, model, ctx->d_mlp_pk, ctx->d_mlp_tail);
            if ((s = mlp_pass(ctx, records, hp->batch, st * hp->batch, (long long)mul, (long long)add, n_train,
                              1.0f / (float)hp->batch, true, nullptr)) != BL_OK)
                return s;
            ++t_step;
            const float c1 = 1.0f - std::pow(b1, (float)t_step), c2 = 1.0f - std::pow(b2, (float)t_step);
            hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNParam + 255) / 256), dim3(256), 0, ctx->stream, model,
                               ctx->d_mlp_m, ctx->d_mlp_v, ctx->d_mlp_grad, hp->lr, b1, b2, hp->eps, c1, c2);
        }
        hipLaunchKernelGGL(k_mlp_store_loss, dim3(1), dim3(64), 0, ctx->stream, ctx->d_mlp_acc,
                           (double)(steps * hp->batch), loss_out + 2 * ep);
        if (hp->n_val > 0) {
            mlp_pack(ctx, model, ctx->d_mlp_pk, ctx->d_mlp_tail);
            if ((s = mlp_pass(ctx, records + n_train * kLogRec, hp->n_val, 0, 1, 0, hp->n_val, 1.0f, false,
                              nullptr)) != BL_OK)
                return s;
            hipLaunchKernelGGL(k_mlp_store_loss, dim3(1), dim3(64), 0, ctx->stream, ctx->d_mlp_acc,
                               (double)hp->n_val, loss_out + 2 * ep + 1);
        } else {
            hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, ctx->stream, loss_out + 2 * ep + 1, 0.0f, 1);
        }
        HIPCHK(ctx, hipGetLastError());
    }
    return BL_OK;
}

bl_status bl_set_step_model(bl_context *ctx, const float *model) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!model) return fail(ctx, BL_E_INVALID_ARG, "model is NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    bl_status s;
    size_t have = ctx->d_step_pk ? (size_t)kPkAll * sizeof(u32x4) : 0;
    if ((s = ensure(ctx, &ctx->d_step_pk, have, (size_t)kPkAll * sizeof(u32x4))) != BL_OK) return s;
    have = ctx->d_step_tail ? (size_t)kTailN * sizeof(float) : 0;
    if ((s = ensure(ctx, &ctx->d_step_tail, have, (size_t)kTailN * sizeof(float))) != BL_OK) return s;
    mlp_pack(ctx, model, ctx->d_step_pk, ctx->d_step_tail);
    HIPCHK(ctx, hipGetLastError());
    ctx->has_step_model = true;
    return BL_OK;
}

bl_status bl_eval_samples(bl_context *ctx, const bl_spacetime *st, const bl_grid *grid, const bl_plasma *plasma,
                          int64_t n, const double *states, const double *norms, double *out) {
    if (!ctx) return BL_E_INVALID_ARG;
    bl_status s;
    if ((s = check_spacetime(ctx, st)) != BL_OK) return s;
    if (!grid || !plasma || !states || !norms || !out || n < 0) return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    if (grid->g.dtype != 0) return fail(ctx, BL_E_UNSUPPORTED, "float32 grids need precision 1");
    if (n == 0) return BL_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if ((s = upload_cuts(ctx)) != BL_OK) return s;
    PlasmaParams pp = plasma_params(ctx, plasma, grid->g, st->mass_msun);
    if ((s = upload_nth(ctx, 1, &plasma, &pp)) != BL_OK) return s;
    hipLaunchKernelGGL(k_eval_samples, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, ctx->stream, st->a,
                       st->flat ? 1 : 0, grid->g, pp, (long long)n, states, norms, out);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_eval_coeffs(bl_context *ctx, int32_t precision, const bl_plasma *plasma, int64_t n, const double *in,
                         double *out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!plasma || !in || !out || n < 0) return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    if (precision != 0 && precision != 1) return fail(ctx, BL_E_INVALID_ARG, "precision must be 0 or 1");
    if (n == 0) return BL_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    PlasmaParams pp{};
    pp.nonthermal = 0;
    pp.nth = nullptr;
    bl_status s;
    if ((s = upload_nth(ctx, 1, &plasma, &pp)) != BL_OK) return s;
    const NthParams *nth = pp.nonthermal ? pp.nth : nullptr;
    const dim3 grd((unsigned)((n + 63) / 64)), blk(64);
    const int pol = plasma->polarized ? 1 : 0;
    if (precision == 0)
        hipLaunchKernelGGL(k_eval_coeffs<double>, grd, blk, 0, ctx->stream, (long long)n, in, pol, nth, out);
    else
        hipLaunchKernelGGL(k_eval_coeffs<float>, grd, blk, 0, ctx->stream, (long long)n, in, pol, nth, out);
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_eval_stokes(bl_context *ctx, int32_t precision, int32_t general, int64_t n, const double *coeffs,
                         const double *s0, double *s_out) {
    if (!ctx) return BL_E_INVALID_ARG;
    if (!coeffs || !s0 || !s_out || n < 0) return fail(ctx, BL_E_INVALID_ARG, "invalid argument");
    if ((precision != 0 && precision != 1) || (general != 0 && general != 1))
        return fail(ctx, BL_E_INVALID_ARG, "precision and general must be 0 or 1");
    if (n == 0) return BL_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const dim3 grd((unsigned)((n + 63) / 64)), blk(64);
    const long long nn = (long long)n;
    switch (2 * precision + general) {
    case 0: hipLaunchKernelGGL((k_eval_stokes<double, false>), grd, blk, 0, ctx->stream, nn, coeffs, s0, s_out); break;
    case 1: hipLaunchKernelGGL((k_eval_stokes<double, true>), grd, blk, 0, ctx->stream, nn, coeffs, s0, s_out); break;
    case 2: hipLaunchKernelGGL((k_eval_stokes<float, false>), grd, blk, 0, ctx->stream, nn, coeffs, s0, s_out); break;
    default: hipLaunchKernelGGL((k_eval_stokes<float, true>), grd, blk, 0, ctx->stream, nn, coeffs, s0, s_out); break;
    }
    HIPCHK(ctx, hipGetLastError());
    return BL_OK;
}

bl_status bl_profile_enable(bl_context *ctx, int enable) {
    if (!ctx) return BL_E_INVALID_ARG;
    ctx->prof = enable != 0;
    return BL_OK;
}

bl_status bl_profile_read(bl_context *ctx, double *ms_out, int64_t *launches_out) {
    if (!ctx || !ms_out || !launches_out) return fail(ctx, BL_E_INVALID_ARG, "NULL argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < BL_NKERNEL; ++k) {
        ms_out[k] = 0.0;
        launches_out[k] = 0;
    }
    bl_status s = BL_OK;
    for (auto &t : ctx->timed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) s = fail(ctx, BL_E_DEVICE, "hipEventElapsedTime failed");
        if (t.kind >= 0 && t.kind < BL_NKERNEL) {
            ms_out[t.kind] += ms;
            launches_out[t.kind] += 1;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    ctx->timed.clear();
    return s;
}

}  // extern "C"
