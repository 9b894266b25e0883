"""Seeded synthetic GRMHD-like fluid data and the named workload configurations.

This module only lays down input arrays.  It holds none of the ray-tracing
arithmetic: the profiles use flat-space spherical coordinates of each cell
centre (R = |x|, cos(theta) = z/R), so nothing here depends on the metric,
the camera, the integrator or the radiation physics.  Both the HIP library's
tests and the CPU reference consume these arrays unchanged.

Recipe (per cell centre, code units):
  rho   = (R/6)^-1.5 exp(-cos^2(theta)/0.1) exp(0.3 Z - 0.045),  Z ~ N(0,1)
          from a counter-based generator keyed by (seed, level, i, j, k);
          rho = 0 for R < r_floor;
  Theta = 10 (R/6)^-1 (target electron temperature);
  p     = rho Theta (m_e/m_p) (n_e/n_i + R_t)/(mu (n_e/n_i + 1)), with
          R_t = (R_high + beta^-2 R_low)/(1 + beta^-2) at beta = beta_target;
  u~    = gamma v phi_hat with v = Omega R_cyl, Omega = 1/(R^1.5 + a) for
          R >= r_isco(a) (0 inside), v capped at 0.95, gamma = (1-v^2)^-1/2;
  B     = |B| (phi_hat + s_h c_pol r_hat)/|...|, |B| = (2 p / beta_target)^1/2,
          s_h = +-1 per hemisphere drawn from seed + 1 (c_pol = 0 toroidal only).
The counter-based generator is SplitMix64 (Steele, Lea & Flood 2014) with a
Box-Muller transform, so uniform grids and mesh-refinement leaves draw their
noise independently of block layout.
"""
import math

import numpy as np

M_E_OVER_M_P = 9.1093837015e-28 / 1.67262192369e-24

_MASK = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x):
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _uniform01(bits):
    # 53 random bits -> (0, 1]
    return ((bits >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def normal_field(seed, level, ii, jj, kk):
    """Standard normal deviates keyed by (seed, level, i, j, k)."""
    key = _splitmix64(np.uint64(seed) * np.uint64(16) + np.uint64(level))
    ctr = ((kk.astype(np.uint64) << np.uint64(21)) | jj.astype(np.uint64)) << np.uint64(21)
    ctr = ctr | ii.astype(np.uint64)
    with np.errstate(over="ignore"):
        base = (ctr << np.uint64(1)) ^ key
        u1 = _uniform01(_splitmix64(base))
        u2 = _uniform01(_splitmix64(base + np.uint64(1)))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def r_isco(a):
    z1 = 1.0 + (1.0 - a * a) ** (1.0 / 3.0) * ((1.0 + a) ** (1.0 / 3.0) + (1.0 - a) ** (1.0 / 3.0))
    z2 = math.sqrt(3.0 * a * a + z1 * z1)
    return 3.0 + z2 - math.sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2))


def _fields(x, y, z, ii, jj, kk, level, a, seed, poloidal, hemi_sign,
            r_high=20.0, r_low=1.0, beta_target=10.0, mu=0.5, ne_ni=1.0):
    R = np.sqrt(x * x + y * y + z * z)
    Rc = np.sqrt(x * x + y * y)
    cth = np.where(R > 0, z / np.where(R > 0, R, 1.0), 1.0)
    Z = normal_field(seed, level, ii, jj, kk)
    r_floor = 1.0 + math.sqrt(max(0.0, 1.0 - a * a))
    Rs = np.maximum(R, 1e-3)
    rho = (Rs / 6.0) ** -1.5 * np.exp(-cth * cth / 0.1) * np.exp(0.3 * Z - 0.045)
    rho = np.where(R < r_floor, 0.0, rho)
    theta_e = 10.0 * (Rs / 6.0) ** -1.0
    binv2 = (1.0 / beta_target) ** 2
    rt = (r_high + binv2 * r_low) / (1.0 + binv2)
    p = rho * theta_e * M_E_OVER_M_P * (ne_ni + rt) / (mu * (ne_ni + 1.0))
    omega = 1.0 / (Rs ** 1.5 + a)
    v = np.minimum(omega * Rc, 0.95)
    v = np.where(R >= r_isco(a), v, 0.0)
    gam = 1.0 / np.sqrt(1.0 - v * v)
    Rcs = np.where(Rc > 0, Rc, 1.0)
    phx, phy = np.where(Rc > 0, -y / Rcs, 0.0), np.where(Rc > 0, x / Rcs, 0.0)
    ux, uy, uz = gam * v * phx, gam * v * phy, np.zeros_like(x)
    sh = np.where(z >= 0, hemi_sign[0], hemi_sign[1])
    bx = phx + poloidal * sh * x / Rs
    by = phy + poloidal * sh * y / Rs
    bz = poloidal * sh * z / Rs
    bn = np.sqrt(bx * bx + by * by + bz * bz)
    bmag = np.sqrt(2.0 * p / beta_target)
    scale = np.where(bn > 0, bmag / np.where(bn > 0, bn, 1.0), 0.0)
    out = np.stack([rho, p, ux, uy, uz, bx * scale, by * scale, bz * scale], axis=-1)
    return out


def _hemi_signs(seed):
    bits = _splitmix64(np.array([seed + 1, seed + 2], dtype=np.uint64))
    return np.where((bits & np.uint64(1)) == 1, 1.0, -1.0)


def uniform_grid(n, half_width, a, seed=0, poloidal=0.0, rho_unit=1e-17, dtype=np.float64):
    """One block of n^3 cells over [-half_width, half_width]^3."""
    return smr_grid(root=1, cells=n, half_width=half_width, a=a, seed=seed, poloidal=poloidal,
                    refine_radius=None, rho_unit=rho_unit, dtype=dtype)


def smr_grid(root, cells, half_width, a, seed=0, poloidal=0.0, refine_radius=20.0,
             rho_unit=1e-17, dtype=np.float64):
    """Two-level static mesh refinement: root^3 blocks of cells^3 cells; a
    root block whose closest point to the origin lies within refine_radius is
    replaced by its 8 children (same cells^3 each).  Returns a dict with
    bounds [nb,6], level [nb], prims [nb,cells,cells,cells,8], rho_unit."""
    L = 2.0 * half_width / root
    hemi = _hemi_signs(seed)
    blocks = []
    for bz in range(root):
        for by in range(root):
            for bx in range(root):
                lo = np.array([-half_width + L * bx, -half_width + L * by, -half_width + L * bz])
                hi = lo + L
                closest = np.clip(0.0, lo, hi)
                refine = refine_radius is not None and float(np.sqrt((closest ** 2).sum())) < refine_radius
                if not refine:
                    blocks.append((0, lo, hi, (bx, by, bz)))
                else:
                    for cz in range(2):
                        for cy in range(2):
                            for cx in range(2):
                                clo = lo + 0.5 * L * np.array([cx, cy, cz])
                                blocks.append((1, clo, clo + 0.5 * L, (2 * bx + cx, 2 * by + cy, 2 * bz + cz)))
    nb = len(blocks)
    bounds = np.zeros((nb, 6))
    level = np.zeros(nb, dtype=np.int32)
    prims = np.zeros((nb, cells, cells, cells, 8), dtype=dtype)
    idx = np.arange(cells)
    for b, (lev, lo, hi, (gx, gy, gz)) in enumerate(blocks):
        bounds[b] = [lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]]
        level[b] = lev
        dx = (hi - lo) / cells
        kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
        x = lo[0] + (ii + 0.5) * dx[0]
        y = lo[1] + (jj + 0.5) * dx[1]
        z = lo[2] + (kk + 0.5) * dx[2]
        prims[b] = _fields(x, y, z, ii + gx * cells, jj + gy * cells, kk + gz * cells, lev, a,
                           seed, poloidal, hemi)
    return {"bounds": bounds, "level": level, "prims": prims, "rho_unit": rho_unit}


def r_horizon(a):
    return 1.0 + math.sqrt(1.0 - a * a)


# ------------------------------------------------------------------ workloads
def workload(name, n=None):
    """Parameter sets of the named workloads.  Returns dict(camera, spacetime,
    integrator, plasma, grid_args).  `n` overrides the image size."""
    deg = math.pi / 180.0
    if name == "c1_64_unpol":
        a, N, th, half, cells, pol, polz = 0.9, 64, 17.0, 40.0, 64, 0.0, 0
        grid_args = dict(kind="uniform", n=64, half_width=40.0, a=a, seed=0, poloidal=0.0)
        ds_max = 0.625
    elif name == "c2_256_pol":
        a, N, th, pol, polz = 0.94, 256, 17.0, 0.5, 1
        grid_args = dict(kind="uniform", n=128, half_width=50.0, a=a, seed=0, poloidal=0.5)
        ds_max = 0.390625
    elif name == "c3_1024_smr":
        a, N, th, pol, polz = 0.5, 1024, 60.0, 0.5, 1
        grid_args = dict(kind="smr", root=8, cells=16, half_width=50.0, a=a, seed=0,
                         poloidal=0.5, refine_radius=20.0)
        ds_max = 0.1953125
    else:
        raise ValueError(name)
    if n is not None:
        N = n
    cam = dict(r=100.0, theta=th * deg, phi=0.0, u_normal=(0.0, 0.0, 0.0), k_cov=(1.0, 0.0, 0.0),
               width=30.0, n=N, freq_mode=0, psi=0.0, nu_hz=230e9)
    st = dict(a=a, mass_msun=4.152e6, r_in=1.01 * r_horizon(a), flat=0)
    integ = dict(f_abs=1e-8, f_rel=1e-8, ds_max=ds_max, h0_frac=0.1, max_steps=100000)
    pl = dict(mu=0.5, ne_ni=1.0, r_high=20.0, r_low=1.0, sigma_max=1.0, polarized=polz, interp=1)
    return dict(camera=cam, spacetime=st, integrator=integ, plasma=pl, grid_args=grid_args)


def batch_workload(n_images=64, n_min=64, n_max=512, seed=2, polarized=1):
    """Batched workload: n_images images over the shared 128^3 uniform grid
    of the 256^2 polarized workload.  Sizes N = round(exp(U[ln n_min,
    ln n_max])); (frequency, inclination, spin) drawn without replacement from
    the 128 combinations of 8 frequencies 86 (690/86)^(j/7) GHz, inclinations
    17, 45, 75, 90 degrees and spins 0, 0.5, 0.9, 0.98.  Returns
    dict(images=[(camera, spacetime)], integrator, plasma, grid_args)."""
    deg = math.pi / 180.0
    rng = np.random.default_rng(seed)
    freqs = [86e9 * (690.0 / 86.0) ** (j / 7.0) for j in range(8)]
    incs = [17.0, 45.0, 75.0, 90.0]
    spins = [0.0, 0.5, 0.9, 0.98]
    combos = [(f, i, a) for f in freqs for i in incs for a in spins]
    pick = rng.choice(len(combos), size=n_images, replace=n_images > len(combos))
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_images))).astype(int)
    images = []
    for k in range(n_images):
        f, inc, a = combos[pick[k]]
        cam = dict(r=100.0, theta=inc * deg, phi=0.0, u_normal=(0.0, 0.0, 0.0), k_cov=(1.0, 0.0, 0.0),
                   width=30.0, n=int(sizes[k]), freq_mode=0, psi=0.0, nu_hz=f)
        st = dict(a=a, mass_msun=4.152e6, r_in=1.01 * r_horizon(a), flat=0)
        images.append((cam, st))
    base = workload("c2_256_pol")
    pl = dict(base["plasma"], polarized=polarized)
    return dict(images=images, integrator=base["integrator"], plasma=pl, grid_args=base["grid_args"])


def steplog_workload(n_images=128, n=32, seed=3):
    """Cameras for logging the plain integrator's steps: spins a ~ U[0, 0.98],
    cos(inclination) ~ U[0, 1], camera at r = 100 M, n x n pixels over
    +-15 M each (a square pixel lattice standing in for uniformly drawn
    pixels).  Returns dict(images=[(camera, spacetime)], integrator)."""
    rng = np.random.default_rng(seed)
    images = []
    for _ in range(n_images):
        a = float(rng.uniform(0.0, 0.98))
        th = math.acos(float(rng.uniform(0.0, 1.0)))
        cam = dict(r=100.0, theta=th, phi=0.0, u_normal=(0.0, 0.0, 0.0), k_cov=(1.0, 0.0, 0.0), width=30.0,
                   n=n, freq_mode=0, psi=0.0, nu_hz=230e9)
        st = dict(a=a, mass_msun=4.152e6, r_in=1.01 * r_horizon(a), flat=0)
        images.append((cam, st))
    integ = dict(f_abs=1e-8, f_rel=1e-8, ds_max=0.0, h0_frac=0.1, max_steps=100000)
    return dict(images=images, integrator=integ)


def make_grid(grid_args, dtype=np.float64):
    g = dict(grid_args)
    kind = g.pop("kind")
    if kind == "uniform":
        return uniform_grid(dtype=dtype, **g)
    return smr_grid(dtype=dtype, **g)
