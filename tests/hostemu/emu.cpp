// Test-only host run of the library's render kernels (built against the
// host stand-in for the HIP runtime): the camera frames, the geodesic kernel
// lane by lane, the persistent transfer kernel as a one-lane wave over all
// rays (its refill, per-lane state machine and ray-end handoff), the overflow
// kernel, the finishing kernel and, when asked, the averages pass, for one
// image of a workload written by tests/test_host_emulation.py, or two images
// as one batch.  Data cuts (cuts.bin: a bl_cuts), nonthermal populations (in
// the plasma), a second image (cam2.bin, st2.bin) and the averages pass
// (avg.flag) select the kernel instantiations the library launches for them.
// Writes, per image, the image and its maps, then the averaged maps.
//   emu <dir> <precision 0|1> <polarized 0|1> [record cap] [extension slots]
#include "blgpu.hip"
#include <vector>
#include <xmmintrin.h>
static void *readall(const char *dir, const char *fn, size_t *n) {
    char p[1024];
    snprintf(p, sizeof p, "%s/%s", dir, fn);
    FILE *f = fopen(p, "rb");
    if (!f) { fprintf(stderr, "missing %s\n", p); exit(2); }
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *b = malloc(sz);
    if (fread(b, 1, sz, f) != (size_t)sz) exit(3);
    fclose(f);
    *n = sz;
    return b;
}
template <typename T>
static void readstruct(const char *dir, const char *fn, T &out) {
    size_t sz;
    void *b = readall(dir, fn, &sz);
    if (sz != sizeof out) { fprintf(stderr, "%s: %zu bytes, expected %zu\n", fn, sz, sizeof out); exit(4); }
    memcpy(&out, b, sz);
    free(b);
}
static bool has_file(const char *dir, const char *fn) {
    char p[1024];
    snprintf(p, sizeof p, "%s/%s", dir, fn);
    FILE *f = fopen(p, "rb");
    if (f) fclose(f);
    return f != nullptr;
}
template <bool POL, typename R, bool CUTS, bool NTH, bool BATCH, bool AVG>
static void run(const char *dir, int precision, int cap_override, int ext_rays) {
    const int n_img = BATCH ? 2 : 1;
    bl_camera cam[2]; bl_spacetime st[2]; bl_integrator integ; bl_plasma pl;
    readstruct(dir, "cam.bin", cam[0]);
    readstruct(dir, "st.bin", st[0]);
    if (BATCH) {
        readstruct(dir, "cam2.bin", cam[1]);
        readstruct(dir, "st2.bin", st[1]);
    }
    readstruct(dir, "integ.bin", integ);
    readstruct(dir, "plasma.bin", pl);
    char p[1024];
    snprintf(p, sizeof p, "%s/grid.txt", dir);
    FILE *f = fopen(p, "r");
    int nb, bnx, bny, bnz; double rho_unit;
    if (fscanf(f, "%d %d %d %d %lf", &nb, &bnx, &bny, &bnz, &rho_unit) != 5) exit(5);
    fclose(f);
    size_t sz;
    double *prims = (double *)readall(dir, "prims.bin", &sz);
    double *bounds = (double *)readall(dir, "bounds.bin", &sz);
    bl_context *ctx = nullptr;
    if (bl_create(0, nullptr, &ctx) != BL_OK) exit(6);
    bl_grid_desc d{};
    d.n_blocks = nb; d.bnx = bnx; d.bny = bny; d.bnz = bnz; d.bounds = bounds; d.prims = prims; d.dtype = 0;
    d.rho_unit = rho_unit;
    bl_grid *grid = nullptr;
    if (bl_grid_create(ctx, &d, &grid) != BL_OK) exit(7);
    if (CUTS) {
        bl_cuts cu;
        readstruct(dir, "cuts.bin", cu);
        if (bl_set_cuts(ctx, &cu) != BL_OK || upload_cuts(ctx) != BL_OK) exit(9);
    }
    PlasmaParams pps[1] = {plasma_params(ctx, &pl, grid->g, st[0].mass_msun)};
    const bl_plasma *pls[1] = {&pl};
    if (upload_nth(ctx, 1, pls, pps) != BL_OK) exit(8);
    const PlasmaParams pp = pps[0];
    if ((pp.nonthermal != 0) != NTH || (pp.cuts != 0) != CUTS) { fprintf(stderr, "instantiation mismatch\n"); exit(10); }
    // images: row-major tiles of 8 x 8 pixels, one wave's worth of ray ids each
    std::vector<std::vector<double>> image(n_img), aux(n_img), avg(n_img);
    ImgDev im[2] = {};
    long long ray0[2] = {0, 0};
    long long count = 0;
    for (int k = 0; k < n_img; ++k) {
        const int n = cam[k].n, tiles = (n + 7) / 8;
        image[k].assign(4 * (size_t)n * n, -7.0);
        aux[k].assign((size_t)BL_NAUX * n * n, -7.0);
        avg[k].assign(AVG ? 21 * (size_t)n * n : 1, -7.0);
        im[k].cp = cam_params(&cam[k]);
        im[k].a = st[k].a; im[k].r_in = st[k].r_in; im[k].flat = st[k].flat ? 1 : 0;
        im[k].L = kG * st[k].mass_msun * kMsun / (kC * kC);
        im[k].image = image[k].data(); im[k].aux = aux[k].data(); im[k].avg = AVG ? avg[k].data() : nullptr;
        im[k].ray0 = ray0[k] = count;
        im[k].nray = (long long)tiles * tiles * 64;
        count += im[k].nray;
    }
    Batch B; B.imgs = im; B.ray0 = ray0; B.n_img = n_img; B.tw = 8; B.th = 8; B.pad = 0;
    threadIdx.x = 0;
    for (int k = 0; k < n_img; ++k) {
        blockIdx.x = k;
        k_camera_frame(B);
    }
    GeoParams P = geo_params(&cam[0], &st[0], &integ);
    record_layout(P, grid->g, &integ, precision == 1);
    if (cap_override > 0) P.cap = cap_override;
    TransferParams tp;
    tp.ds_max = integ.ds_max; tp.L = im[0].L; tp.nu_cam = cam[0].nu_hz;
    std::vector<double> rec((size_t)count * P.cap * kRecDoubles), meta(2 * (size_t)count);
    std::vector<int> nacc(count), work(count), ovf_list(count), of(count, -1), order(count), queue(4, 0);
    int ovf_count = 0, ext_count = 0;
    ExtQueue X;
    X.count = &ext_count; X.of = of.data();
    X.cap_rec = (int)std::min<long long>(2048, P.max_steps + 1);
    X.cap_rays = X.cap_rec > P.cap ? ext_rays : 0;
    std::vector<double> xrec((size_t)std::max(1, X.cap_rays) * X.cap_rec * kRecDoubles);
    X.rec = xrec.data();
    blockDim.x = 64;
    for (long long s = 0; s < count; ++s) {
        blockIdx.x = (unsigned)(s / 64); threadIdx.x = (unsigned)(s % 64);
        k_geodesic<true, BATCH>(P, B, 0, (int)count, rec.data(), meta.data(), nacc.data(), work.data(), X, &ovf_count,
                                ovf_list.data(), nullptr);
    }
    for (long long s = 0; s < count; ++s) order[s] = (int)s;
    std::vector<R> ends((size_t)count * kRayEnd);
    blockIdx.x = 0; threadIdx.x = 0;
    k_transfer<POL, R, BATCH, CUTS, false, NTH>(P, B, grid->g, pp, tp, 0, (int)count, 1, rec.data(), meta.data(),
                                                nacc.data(), order.data(), X, queue.data(), ends.data());
    PlasmaParams pa = pp;
    pa.polarized = 0;
    if (AVG)   // the averages pass: the unpolarized walk over the same records
        k_transfer<false, R, false, CUTS, true, false>(P, B, grid->g, pa, tp, 0, (int)count, 1, rec.data(), meta.data(),
                                                       nacc.data(), order.data(), X, queue.data() + 2, ends.data());
    if (ovf_count > 0) {
        const int big_cap = (int)std::min<long long>(P.max_steps + 1, 200000);
        std::vector<double> big((size_t)big_cap * kRecDoubles);
        blockDim.x = 1; threadIdx.x = 0;
        k_overflow<POL, R, CUTS, false, NTH>(P, B, grid->g, pp, tp, &ovf_count, ovf_list.data(), big.data(), big_cap);
        if (AVG)
            k_overflow<false, R, CUTS, true, false>(P, B, grid->g, pa, tp, &ovf_count, ovf_list.data(), big.data(),
                                                    big_cap);
        blockDim.x = 64;
    }
    if (POL) {
        for (long long s = 0; s < count; ++s) {
            blockIdx.x = (unsigned)(s / 64); threadIdx.x = (unsigned)(s % 64);
            k_finish<R, BATCH>(P, B, 0, (int)count, rec.data(), nacc.data(), X, ends.data());
        }
    }
    snprintf(p, sizeof p, "%s/emu_out_%d.bin", dir, precision);
    f = fopen(p, "wb");
    for (int k = 0; k < n_img; ++k) {
        fwrite(image[k].data(), sizeof(double), image[k].size(), f);
        fwrite(aux[k].data(), sizeof(double), aux[k].size(), f);
    }
    if (AVG) fwrite(avg[0].data(), sizeof(double), avg[0].size(), f);
    fclose(f);
    printf("emulated %d image(s) of %dx%d, precision %d, polarized %d, cap %d, extension requests %d, "
           "overflow rays %d\n", n_img, cam[0].n, cam[0].n, precision, (int)POL, P.cap, ext_count, ovf_count);
    bl_grid_destroy(grid);
    bl_destroy(ctx);
    free(prims); free(bounds);
}
template <bool POL, typename R>
static void run_form(const char *dir, int precision, int cap, int ext) {
    size_t sz;
    bl_plasma pl;
    void *b = readall(dir, "plasma.bin", &sz);
    memcpy(&pl, b, sizeof pl);
    free(b);
    const bool cuts = has_file(dir, "cuts.bin"), batch = has_file(dir, "cam2.bin"), avg = has_file(dir, "avg.flag");
    const bool nth = pl.fractions[1] != 0.0 || pl.fractions[2] != 0.0;
    if (batch) run<POL, R, false, false, true, false>(dir, precision, cap, ext);
    else if (avg) run<POL, R, false, false, false, true>(dir, precision, cap, ext);
    else if (cuts) run<POL, R, true, false, false, false>(dir, precision, cap, ext);
    else if (nth) run<POL, R, false, true, false, false>(dir, precision, cap, ext);
    else run<POL, R, false, false, false, false>(dir, precision, cap, ext);
}
int main(int argc, char **argv) {
    const char *dir = argv[1];
    int precision = atoi(argv[2]), pol = atoi(argv[3]);
    int cap = argc > 4 ? atoi(argv[4]) : 0, ext = argc > 5 ? atoi(argv[5]) : 16;
    // the mixed form's library build flushes FP32 values below 2^-126 to zero
    // (inputs and results); on the host the same control word also flushes
    // FP64, which the mixed form uses only for positions and step data
    if (precision == 1) _mm_setcsr(_mm_getcsr() | 0x8040);   // flush-to-zero, denormals-are-zero
    if (precision == 0) {
        if (pol) run_form<true, double>(dir, 0, cap, ext);
        else run_form<false, double>(dir, 0, cap, ext);
    } else {
        if (pol) run_form<true, float>(dir, 1, cap, ext);
        else run_form<false, float>(dir, 1, cap, ext);
    }
    return 0;
}
