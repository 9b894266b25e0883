// Test-only host run of the library's render kernels (built against the
// host stand-in for the HIP runtime): the camera frame, the geodesic kernel
// lane by lane, the persistent transfer kernel as a one-lane wave over all
// rays (its refill, per-lane state machine and ray-end handoff), the overflow
// kernel and the finishing kernel, for one image of a workload written by
// tests/test_host_emulation.py.  Writes the image and its maps.
// Data cuts (cuts.bin: a bl_cuts) and nonthermal populations (in the plasma)
// select the transfer instantiations the library would launch for them.
//   emu <dir> <precision 0|1> <polarized 0|1> [record cap] [extension slots]
#include "blgpu.hip"
#include <vector>
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
static bool has_file(const char *dir, const char *fn) {
    char p[1024];
    snprintf(p, sizeof p, "%s/%s", dir, fn);
    FILE *f = fopen(p, "rb");
    if (f) fclose(f);
    return f != nullptr;
}
template <bool POL, typename R, bool CUTS, bool NTH>
static void run(const char *dir, int precision, int cap_override, int ext_rays) {
    size_t sz;
    bl_camera cam; bl_spacetime st; bl_integrator integ; bl_plasma pl;
    void *b;
    b = readall(dir, "cam.bin", &sz); memcpy(&cam, b, sz); free(b);
    b = readall(dir, "st.bin", &sz); memcpy(&st, b, sz); free(b);
    b = readall(dir, "integ.bin", &sz); memcpy(&integ, b, sz); free(b);
    b = readall(dir, "plasma.bin", &sz); memcpy(&pl, b, sz); free(b);
    char p[1024];
    snprintf(p, sizeof p, "%s/grid.txt", dir);
    FILE *f = fopen(p, "r");
    int nb, bnx, bny, bnz; double rho_unit;
    if (fscanf(f, "%d %d %d %d %lf", &nb, &bnx, &bny, &bnz, &rho_unit) != 5) exit(5);
    fclose(f);
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
        b = readall(dir, "cuts.bin", &sz);
        if (sz != sizeof cu) exit(4);
        memcpy(&cu, b, sz);
        free(b);
        if (bl_set_cuts(ctx, &cu) != BL_OK || upload_cuts(ctx) != BL_OK) exit(9);
    }
    PlasmaParams pps[1] = {plasma_params(ctx, &pl, grid->g, st.mass_msun)};
    const bl_plasma *pls[1] = {&pl};
    if (upload_nth(ctx, 1, pls, pps) != BL_OK) exit(8);
    const PlasmaParams pp = pps[0];
    if ((pp.nonthermal != 0) != NTH || (pp.cuts != 0) != CUTS) { fprintf(stderr, "instantiation mismatch\n"); exit(10); }
    const int n = cam.n;
    std::vector<double> image(4 * (size_t)n * n, -7.0), aux((size_t)BL_NAUX * n * n, -7.0);
    ImgDev im{};
    im.cp = cam_params(&cam);
    im.a = st.a; im.r_in = st.r_in; im.flat = st.flat ? 1 : 0;
    im.L = kG * st.mass_msun * kMsun / (kC * kC);
    im.image = image.data(); im.aux = aux.data(); im.avg = nullptr;
    const int tiles = (n + 7) / 8;
    const int count = tiles * tiles * 64;
    im.ray0 = 0; im.nray = count;
    long long ray0 = 0;
    Batch B; B.imgs = &im; B.ray0 = &ray0; B.n_img = 1; B.tw = 8; B.th = 8; B.pad = 0;
    threadIdx.x = 0; blockIdx.x = 0;
    k_camera_frame(B);
    GeoParams P = geo_params(&cam, &st, &integ);
    record_layout(P, grid->g, &integ, precision == 1);
    if (cap_override > 0) P.cap = cap_override;
    TransferParams tp;
    tp.ds_max = integ.ds_max; tp.L = im.L; tp.nu_cam = cam.nu_hz;
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
    for (int s = 0; s < count; ++s) {
        blockIdx.x = s / 64; threadIdx.x = s % 64;
        k_geodesic<true, false>(P, B, 0, count, rec.data(), meta.data(), nacc.data(), work.data(), X, &ovf_count,
                                ovf_list.data(), nullptr);
    }
    for (int s = 0; s < count; ++s) order[s] = s;
    std::vector<R> ends((size_t)count * kRayEnd);
    blockIdx.x = 0; threadIdx.x = 0;
    k_transfer<POL, R, false, CUTS, false, NTH>(P, B, grid->g, pp, tp, 0, count, 1, rec.data(), meta.data(),
                                                  nacc.data(), order.data(), X, queue.data(), ends.data());
    if (ovf_count > 0) {
        const int big_cap = (int)std::min<long long>(P.max_steps + 1, 200000);
        std::vector<double> big((size_t)big_cap * kRecDoubles);
        blockDim.x = 1; threadIdx.x = 0;
        k_overflow<POL, R, CUTS, false, NTH>(P, B, grid->g, pp, tp, &ovf_count, ovf_list.data(), big.data(), big_cap);
        blockDim.x = 64;
    }
    if (POL) {
        for (int s = 0; s < count; ++s) {
            blockIdx.x = s / 64; threadIdx.x = s % 64;
            k_finish<R, false>(P, B, 0, count, rec.data(), nacc.data(), X, ends.data());
        }
    }
    snprintf(p, sizeof p, "%s/emu_out_%d.bin", dir, precision);
    f = fopen(p, "wb");
    fwrite(image.data(), sizeof(double), image.size(), f);
    fwrite(aux.data(), sizeof(double), aux.size(), f);
    fclose(f);
    printf("emulated %dx%d image, precision %d, polarized %d, cap %d, extension requests %d, overflow rays %d\n",
           n, n, precision, (int)POL, P.cap, ext_count, ovf_count);
    bl_grid_destroy(grid);
    bl_destroy(ctx);
    free(prims); free(bounds);
}
template <bool POL, typename R>
static void run_form(const char *dir, int precision, int cap, int ext, bool cuts, bool nth) {
    if (cuts) run<POL, R, true, false>(dir, precision, cap, ext);
    else if (nth) run<POL, R, false, true>(dir, precision, cap, ext);
    else run<POL, R, false, false>(dir, precision, cap, ext);
}
int main(int argc, char **argv) {
    const char *dir = argv[1];
    int precision = atoi(argv[2]), pol = atoi(argv[3]);
    int cap = argc > 4 ? atoi(argv[4]) : 0, ext = argc > 5 ? atoi(argv[5]) : 16;
    const bool cuts = has_file(dir, "cuts.bin");
    size_t sz;
    bl_plasma pl;
    void *b = readall(dir, "plasma.bin", &sz);
    memcpy(&pl, b, sizeof pl);
    free(b);
    const bool nth = pl.fractions[1] != 0.0 || pl.fractions[2] != 0.0;
    if (precision == 0) {
        if (pol) run_form<true, double>(dir, 0, cap, ext, cuts, nth);
        else run_form<false, double>(dir, 0, cap, ext, cuts, nth);
    } else {
        if (pol) run_form<true, float>(dir, 1, cap, ext, cuts, nth);
        else run_form<false, float>(dir, 1, cap, ext, cuts, nth);
    }
    return 0;
}
