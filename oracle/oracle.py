"""ctypes front end of the plain FP64 CPU oracle (oracle/*.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  Parameter sets are
plain dicts (see ``camera``, ``spacetime``, ``integrator``, ``plasma`` below)
so that this module shares nothing with the HIP path's binding.
"""
import ctypes as C
import os

import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

NAUX = 10
NAVG = 21
AUX_NAMES = ["dt", "s", "lambda", "tau", "I_j", "n_acc", "n_rej", "status", "n_samp", "n_rec"]
ESCAPED, CAPTURED, MAXSTEPS, UNDERFLOW, NONFINITE = 1, 2, 3, 4, 5


class Camera(C.Structure):
    _fields_ = [("r", C.c_double), ("theta", C.c_double), ("phi", C.c_double),
                ("u_normal", C.c_double * 3), ("k_cov", C.c_double * 3),
                ("width", C.c_double), ("n", C.c_int32), ("freq_mode", C.c_int32),
                ("psi", C.c_double), ("nu_hz", C.c_double)]


class Spacetime(C.Structure):
    _fields_ = [("a", C.c_double), ("mass_msun", C.c_double), ("r_in", C.c_double),
                ("flat", C.c_int32), ("pad", C.c_int32)]


class Integrator(C.Structure):
    _fields_ = [("f_abs", C.c_double), ("f_rel", C.c_double), ("ds_max", C.c_double),
                ("h0_frac", C.c_double), ("max_steps", C.c_int64)]


class Grid(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("bnx", C.c_int32), ("bny", C.c_int32),
                ("bnz", C.c_int32), ("bounds", C.POINTER(C.c_double)),
                ("prims", C.POINTER(C.c_double)), ("rho_unit", C.c_double)]


CUT_KEYS = ("rho", "ne", "p", "theta_e", "b", "sigma", "beta_inv", "r")


class Plasma(C.Structure):
    _fields_ = [("mu", C.c_double), ("ne_ni", C.c_double), ("r_high", C.c_double),
                ("r_low", C.c_double), ("sigma_max", C.c_double),
                ("polarized", C.c_int32), ("interp", C.c_int32),
                ("use_cuts", C.c_int32), ("plane", C.c_int32),
                ("cut_lo", C.c_double * 8), ("cut_hi", C.c_double * 8),
                ("plane_x0", C.c_double * 3), ("plane_n", C.c_double * 3),
                ("frac", C.c_double * 3), ("pl_p", C.c_double), ("pl_gmin", C.c_double),
                ("pl_gmax", C.c_double), ("kappa", C.c_double), ("kappa_w", C.c_double),
                ("pl_norm", C.c_double), ("kap_norm", C.c_double), ("kap_m23", C.c_double),
                ("kap_m53", C.c_double)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            import importlib.util
            spec = importlib.util.spec_from_file_location("oracle_build", os.path.join(_HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        L = C.CDLL(path)
        d, i, i64 = C.c_double, C.c_int, C.c_int64
        P = C.POINTER(C.c_double)
        L.or_ks_radius.restype = d
        L.or_ks_radius.argtypes = [d, d, d, d]
        L.or_metric.argtypes = [d, i, P, P, P]
        L.or_metric_deriv.argtypes = [d, i, P, P, P]
        L.or_christoffel.argtypes = [d, i, P, P]
        L.or_geodesic_rhs.argtypes = [d, i, P, P]
        L.or_dp_tableau.argtypes = [P, P, P, P, P]
        L.or_camera_basis.argtypes = [C.POINTER(Camera), C.POINTER(Spacetime), P]
        L.or_camera_ray.argtypes = [C.POINTER(Camera), C.POINTER(Spacetime), i, i, P, P]
        L.or_trace_pixel.restype = i64
        L.or_trace_pixel.argtypes = [C.POINTER(Camera), C.POINTER(Spacetime), C.POINTER(Integrator),
                                     i, i, P, i64, P, P]
        L.or_trace_trials.restype = i64
        L.or_trace_trials.argtypes = [C.POINTER(Camera), C.POINTER(Spacetime), C.POINTER(Integrator),
                                      i, i, P, i64, P]
        L.or_grid_sample.restype = i
        L.or_grid_sample.argtypes = [C.POINTER(Grid), i, P, P]
        L.or_bessel_k_scaled.restype = d
        L.or_bessel_k_scaled.argtypes = [i, d]
        L.or_thermal_coeffs.argtypes = [d, d, d, d, d, i, P]
        L.or_nonthermal_prepare.argtypes = [C.POINTER(Plasma)]
        L.or_kappa_integral.restype = d
        L.or_kappa_integral.argtypes = [d, d, d]
        L.or_nonthermal_coeffs.argtypes = [i, C.POINTER(Plasma), d, d, d, d, i, P]
        L.or_sample_point.argtypes = [C.POINTER(Spacetime), C.POINTER(Grid), C.POINTER(Plasma), P, d, P]
        L.or_unpol_segment.restype = d
        L.or_unpol_segment.argtypes = [d, d, d, d]
        L.or_stokes_exact.argtypes = [P, P, P, d, P]
        L.or_transport_rhs.argtypes = [d, i, P, P, P, P, P]
        L.or_ds_dlambda.restype = d
        L.or_ds_dlambda.argtypes = [d, i, P]
        L.or_render_pixels.argtypes = [C.POINTER(Camera), C.POINTER(Spacetime), C.POINTER(Integrator),
                                       C.POINTER(Grid), C.POINTER(Plasma), i64,
                                       C.POINTER(C.c_int64), P, P, P, i]
        L.or_dense_quartic.argtypes = [P, P, P, P, P, d, d, P]
        _LIB = L
    return _LIB


# ---------------------------------------------------------------- parameters
def camera(d):
    c = Camera()
    c.r, c.theta, c.phi = d["r"], d["theta"], d.get("phi", 0.0)
    for k in range(3):
        c.u_normal[k] = d.get("u_normal", (0.0, 0.0, 0.0))[k]
        c.k_cov[k] = d.get("k_cov", (1.0, 0.0, 0.0))[k]
    c.width, c.n = d["width"], int(d["n"])
    c.freq_mode = int(d.get("freq_mode", 0))
    c.psi = d.get("psi", 0.0)
    c.nu_hz = d.get("nu_hz", 230e9)
    return c


def spacetime(d):
    s = Spacetime()
    s.a, s.mass_msun, s.r_in = d["a"], d.get("mass_msun", 4.152e6), d["r_in"]
    s.flat = int(d.get("flat", 0))
    return s


def integrator(d):
    g = Integrator()
    g.f_abs, g.f_rel = d.get("f_abs", 1e-8), d.get("f_rel", 1e-8)
    g.ds_max, g.h0_frac = d.get("ds_max", 0.0), d.get("h0_frac", 0.1)
    g.max_steps = int(d.get("max_steps", 100000))
    return g


def plasma(d):
    p = Plasma()
    p.mu, p.ne_ni = d.get("mu", 0.5), d.get("ne_ni", 1.0)
    p.r_high, p.r_low = d.get("r_high", 20.0), d.get("r_low", 1.0)
    p.sigma_max = d.get("sigma_max", 1.0)
    p.polarized, p.interp = int(d.get("polarized", 0)), int(d.get("interp", 1))
    cuts = d.get("cuts")
    for k in range(8):
        p.cut_lo[k], p.cut_hi[k] = -math.inf, math.inf
    if cuts:
        # {"rho": (lo, hi), ..., "plane": {"side": +1 or -1, "origin": x0, "normal": n}}
        p.use_cuts = 1
        for k, name in enumerate(CUT_KEYS):
            if name in cuts:
                p.cut_lo[k], p.cut_hi[k] = float(cuts[name][0]), float(cuts[name][1])
        if "plane" in cuts:
            pl = cuts["plane"]
            p.plane = int(pl["side"])
            for i in range(3):
                p.plane_x0[i], p.plane_n[i] = float(pl["origin"][i]), float(pl["normal"][i])
    # electron populations: fractions (thermal, power law, kappa) and parameters
    # (defaults: the paper's p = 3, gamma 4..1000, kappa = 4, w = 1/2)
    fr = d.get("fractions", (1.0, 0.0, 0.0))
    for k in range(3):
        p.frac[k] = float(fr[k])
    p.pl_p, p.pl_gmin, p.pl_gmax = d.get("pl_p", 3.0), d.get("pl_gamma_min", 4.0), d.get("pl_gamma_max", 1000.0)
    p.kappa, p.kappa_w = d.get("kappa", 4.0), d.get("kappa_w", 0.5)
    if p.frac[1] > 0 or p.frac[2] > 0:
        lib().or_nonthermal_prepare(C.byref(p))
    return p


class GridHandle:
    """Keeps the numpy buffers alive for as long as the C struct is used."""

    def __init__(self, bounds, prims, rho_unit):
        self.bounds = np.ascontiguousarray(bounds, dtype=np.float64)
        self.prims = np.ascontiguousarray(prims, dtype=np.float64)
        nb, bnz, bny, bnx, nv = self.prims.shape
        assert nv == 8 and self.bounds.shape == (nb, 6)
        self.s = Grid()
        self.s.n_blocks, self.s.bnx, self.s.bny, self.s.bnz = nb, bnx, bny, bnz
        self.s.bounds = _dp(self.bounds)
        self.s.prims = _dp(self.prims)
        self.s.rho_unit = rho_unit


def grid(g):
    if isinstance(g, GridHandle):
        return g
    return GridHandle(g["bounds"], g["prims"], g["rho_unit"])


# ---------------------------------------------------------------- wrappers
def ks_radius(a, x, y, z):
    return lib().or_ks_radius(a, x, y, z)


def metric(a, x, flat=0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    g, gi = np.zeros(16), np.zeros(16)
    lib().or_metric(a, flat, _dp(x), _dp(g), _dp(gi))
    return g.reshape(4, 4), gi.reshape(4, 4)


def metric_deriv(a, x, flat=0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    dg, dgi = np.zeros(48), np.zeros(48)
    lib().or_metric_deriv(a, flat, _dp(x), _dp(dg), _dp(dgi))
    return dg.reshape(3, 4, 4), dgi.reshape(3, 4, 4)


def christoffel(a, x, flat=0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    gam = np.zeros(64)
    lib().or_christoffel(a, flat, _dp(x), _dp(gam))
    return gam.reshape(4, 4, 4)


def geodesic_rhs(a, y, flat=0):
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.zeros(8)
    lib().or_geodesic_rhs(a, flat, _dp(y), _dp(dy))
    return dy


def ds_dlambda(a, y, flat=0):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().or_ds_dlambda(a, flat, _dp(y))


def dp_tableau():
    c, A, b5, b4, bm = np.zeros(7), np.zeros(49), np.zeros(7), np.zeros(7), np.zeros(7)
    lib().or_dp_tableau(_dp(c), _dp(A), _dp(b5), _dp(b4), _dp(bm))
    return c, A.reshape(7, 7), b5, b4, bm


def camera_basis(cam, st):
    out = np.zeros(20)
    c, s = camera(cam), spacetime(st)
    lib().or_camera_basis(C.byref(c), C.byref(s), _dp(out))
    return {"xc": out[0:4], "u": out[4:8], "K": out[8:12], "H": out[12:16], "V": out[16:20]}


def camera_ray(cam, st, i, j):
    y, n = np.zeros(8), np.zeros(1)
    c, s = camera(cam), spacetime(st)
    lib().or_camera_ray(C.byref(c), C.byref(s), int(i), int(j), _dp(y), _dp(n))
    return y, float(n[0])


def trace_pixel(cam, st, integ, i, j, max_records=200000):
    c, s, g = camera(cam), spacetime(st), integrator(integ)
    steps = np.zeros((max_records, 25))
    info, yend = np.zeros(8), np.zeros(8)
    n = lib().or_trace_pixel(C.byref(c), C.byref(s), C.byref(g), int(i), int(j),
                             _dp(steps), max_records, _dp(info), _dp(yend))
    return {"steps": steps[:n].copy(), "n_acc": int(info[0]), "n_rej": int(info[1]),
            "status": int(info[2]), "lambda": info[3], "s": info[4], "dt": info[5],
            "r_end": info[6], "n_norm": info[7], "y_end": yend}


def trace_trials(cam, st, integ, i, j, max_trials=200000):
    """Every trial step of pixel (i, j): rows of the state at the trial's
    start y[8], the trial step h, its error norm eps and accepted (1) or
    rejected (0)."""
    c, s, g = camera(cam), spacetime(st), integrator(integ)
    log = np.zeros((max_trials, 11))
    info = np.zeros(8)
    n = lib().or_trace_trials(C.byref(c), C.byref(s), C.byref(g), int(i), int(j), _dp(log), max_trials,
                              _dp(info))
    return {"trials": log[:min(n, max_trials)].copy(), "n_acc": int(info[0]), "n_rej": int(info[1]),
            "status": int(info[2])}


def grid_sample(gr, x, interp=1):
    gh = grid(gr)
    x = np.ascontiguousarray(x, dtype=np.float64)
    prim = np.zeros(8)
    b = lib().or_grid_sample(C.byref(gh.s), int(interp), _dp(x), _dp(prim))
    return b, prim


def bessel_k_scaled(n, x):
    return lib().or_bessel_k_scaled(int(n), float(x))


def thermal_coeffs(ne, thetae, B, nu, cos_theta, polarized=1):
    out = np.zeros(8)
    lib().or_thermal_coeffs(ne, thetae, B, nu, cos_theta, int(polarized), _dp(out))
    return out


def nonthermal_coeffs(kind, pl, ne, B, nu, cos_theta, polarized=1):
    """Fluid-frame coefficients of n_e electrons in population kind (1: power
    law, 2: kappa) with the parameters of plasma dict pl."""
    out = np.zeros(8)
    p = plasma(dict(pl, fractions=(0.0, 1.0, 0.0) if kind == 1 else (0.0, 0.0, 1.0)))
    lib().or_nonthermal_coeffs(int(kind), C.byref(p), ne, B, nu, cos_theta, int(polarized), _dp(out))
    return out


def kappa_integral(kappa, w, s):
    return lib().or_kappa_integral(kappa, w, s)


def sample_point(st, gr, pl, y, n_norm):
    gh, s, p = grid(gr), spacetime(st), plasma(pl)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(33)
    lib().or_sample_point(C.byref(s), C.byref(gh.s), C.byref(p), _dp(y), float(n_norm), _dp(out))
    return out


def unpol_segment(I, j, alpha, dl):
    return lib().or_unpol_segment(I, j, alpha, dl)


def stokes_exact(S0, J, M, s):
    S0 = np.ascontiguousarray(S0, dtype=np.float64)
    J = np.ascontiguousarray(J, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(16)
    out = np.zeros(4)
    lib().or_stokes_exact(_dp(S0), _dp(J), _dp(M), float(s), _dp(out))
    return out


def transport_rhs(a, y, Nre, Nim, flat=0):
    y = np.ascontiguousarray(y, dtype=np.float64)
    Nre = np.ascontiguousarray(Nre, dtype=np.float64).reshape(16)
    Nim = np.ascontiguousarray(Nim, dtype=np.float64).reshape(16)
    dR, dI = np.zeros(16), np.zeros(16)
    lib().or_transport_rhs(a, flat, _dp(y), _dp(Nre), _dp(Nim), _dp(dR), _dp(dI))
    return dR.reshape(4, 4), dI.reshape(4, 4)


def render_pixels(cam, st, integ, gr, pl, pixels, n_threads=None, averages=False):
    """Render pixel indices (i + N j).  Returns image [n,4] and aux [n,NAUX],
    and with averages=True also the averaged quantities [n,NAVG]."""
    c, s, g, p = camera(cam), spacetime(st), integrator(integ), plasma(pl)
    gh = grid(gr)
    pix = np.ascontiguousarray(pixels, dtype=np.int64)
    img = np.zeros((len(pix), 4))
    aux = np.zeros((len(pix), NAUX))
    avg = np.zeros((len(pix), NAVG)) if averages else None
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    lib().or_render_pixels(C.byref(c), C.byref(s), C.byref(g), C.byref(gh.s), C.byref(p),
                           len(pix), pix.ctypes.data_as(C.POINTER(C.c_int64)),
                           _dp(img), _dp(aux), _dp(avg) if averages else None, int(n_threads))
    return (img, aux, avg) if averages else (img, aux)


def render(cam, st, integ, gr, pl, n_threads=None, averages=False):
    """Whole image: returns image [4, N, N] and aux [NAUX, N, N] (row j, column
    i), and with averages=True the averaged quantities [NAVG, N, N] (<q>_lambda,
    <q>_Ij, <q>_tau for q in rho, n_e, p, Theta_e, B, sigma, beta^-1)."""
    n = int(cam["n"])
    out = render_pixels(cam, st, integ, gr, pl, np.arange(n * n), n_threads, averages)
    res = (out[0].T.reshape(4, n, n), out[1].T.reshape(NAUX, n, n))
    return res + (out[2].T.reshape(NAVG, n, n),) if averages else res


def dense_quartic(y0, y1, f0, f1, ym, h, theta):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (y0, y1, f0, f1, ym)]
    out = np.zeros(8)
    lib().or_dense_quartic(*[_dp(v) for v in arrs], float(h), float(theta), _dp(out))
    return out
