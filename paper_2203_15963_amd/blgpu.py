"""ctypes binding of libblgpu (include/blgpu.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch tensors on the context's GPU; the library
enqueues on the torch stream given at context creation.  The binding refuses
to work without the built library (there is no fallback path).
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblgpu.so")
ABI_VERSION = 2
NAUX = 10
NAVG = 21
NKERNEL = 4
KERNEL_NAMES = ["setup", "geodesic", "transfer", "overflow"]
NSAMPLE_OUT = 64
AUX_NAMES = ["dt", "s", "lambda", "tau", "I_j", "n_acc", "n_rej", "status", "n_samp", "n_rec"]
STATUS = {"OK": 0, "E_INVALID_ARG": -1, "E_DEVICE": -2, "E_OOM": -3, "E_UNSUPPORTED": -4, "E_STATE": -5}
_STATUS_NAME = {v: k for k, v in STATUS.items()}


class bl_camera(C.Structure):
    _fields_ = [("r", C.c_double), ("theta", C.c_double), ("phi", C.c_double),
                ("u_normal", C.c_double * 3), ("k_cov", C.c_double * 3),
                ("width", C.c_double), ("n", C.c_int32), ("freq_mode", C.c_int32),
                ("kind", C.c_int32), ("pad", C.c_int32), ("psi", C.c_double), ("nu_hz", C.c_double)]


class bl_spacetime(C.Structure):
    _fields_ = [("a", C.c_double), ("mass_msun", C.c_double), ("r_in", C.c_double),
                ("flat", C.c_int32), ("pad", C.c_int32)]


class bl_integrator(C.Structure):
    _fields_ = [("f_abs", C.c_double), ("f_rel", C.c_double), ("ds_max", C.c_double),
                ("h0_frac", C.c_double), ("max_steps", C.c_int64), ("record_cap", C.c_int32),
                ("pad", C.c_int32)]


class bl_grid_desc(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("bnx", C.c_int32), ("bny", C.c_int32), ("bnz", C.c_int32),
                ("bounds", C.POINTER(C.c_double)), ("prims", C.c_void_p), ("dtype", C.c_int32),
                ("pad", C.c_int32), ("rho_unit", C.c_double)]


class bl_plasma(C.Structure):
    _fields_ = [("mu", C.c_double), ("ne_ni", C.c_double), ("r_high", C.c_double),
                ("r_low", C.c_double), ("sigma_max", C.c_double), ("polarized", C.c_int32),
                ("interp", C.c_int32), ("fractions", C.c_double * 3), ("pl_p", C.c_double),
                ("pl_gamma_min", C.c_double), ("pl_gamma_max", C.c_double), ("kappa", C.c_double),
                ("kappa_w", C.c_double)]


class bl_mode(C.Structure):
    _fields_ = [("precision", C.c_int32), ("step_model", C.c_int32)]


class bl_tuning(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("transfer_waves_per_cu", C.c_int32),
                ("refill_min", C.c_int32), ("chunk_rays", C.c_int64), ("order", C.c_int32),
                ("reserved", C.c_int32)]


class bl_cuts(C.Structure):
    _fields_ = [("rho", C.c_double * 2), ("ne", C.c_double * 2), ("p", C.c_double * 2),
                ("theta_e", C.c_double * 2), ("b", C.c_double * 2), ("sigma", C.c_double * 2),
                ("beta_inv", C.c_double * 2), ("r", C.c_double * 2), ("plane", C.c_int32), ("pad", C.c_int32),
                ("plane_origin", C.c_double * 3), ("plane_normal", C.c_double * 3)]


ADAPT_MAX_REGIONS = 8
ADAPT_CRITERIA = ("value", "grad_abs", "grad_rel", "lap_abs", "lap_rel")


class bl_adaptive(C.Structure):
    _fields_ = [("block_n", C.c_int32), ("max_level", C.c_int32), ("use", C.c_int32 * 5), ("n_regions", C.c_int32),
                ("thr", C.c_double * 5), ("frac", C.c_double), ("region", (C.c_double * 5) * ADAPT_MAX_REGIONS)]


def adaptive(d):
    """bl_adaptive from {"block": B, "max_level": L, "frac": f, "thr": [5
    thresholds, None = off] (or criterion name -> threshold), "regions":
    [(x0, x1, y0, y1, min_level), ...]}."""
    a = bl_adaptive()
    a.block_n, a.max_level, a.frac = int(d["block"]), int(d["max_level"]), float(d.get("frac", 1.0))
    thr = d.get("thr", [None] * 5)
    if isinstance(thr, dict):
        thr = [thr.get(k) for k in ADAPT_CRITERIA]
    for c, v in enumerate(thr):
        a.use[c], a.thr[c] = (0, 0.0) if v is None else (1, float(v))
    regs = d.get("regions", [])
    a.n_regions = len(regs)
    for r, g in enumerate(regs[:ADAPT_MAX_REGIONS]):
        for q in range(5):
            a.region[r][q] = float(g[q])
    return a


CUT_KEYS = ("rho", "ne", "p", "theta_e", "b", "sigma", "beta_inv", "r")


def cuts(d):
    """bl_cuts from {"rho": (lo, hi), ..., "plane": {"side": +1 or -1,
    "origin": x0, "normal": n}}; absent quantities are left uncut."""
    c = bl_cuts()
    for k in CUT_KEYS:
        lo, hi = d.get(k, (-math.inf, math.inf))
        getattr(c, k)[0], getattr(c, k)[1] = float(lo), float(hi)
    if "plane" in d:
        pl = d["plane"]
        c.plane = int(pl["side"])
        for i in range(3):
            c.plane_origin[i], c.plane_normal[i] = float(pl["origin"][i]), float(pl["normal"][i])
    return c


class bl_image_desc(C.Structure):
    _fields_ = [("cam", bl_camera), ("st", bl_spacetime), ("image_out", C.c_void_p), ("aux_out", C.c_void_p)]


MLP_NIN, MLP_NHID, MLP_NPARAM, MLP_NMODEL, STEPLOG_REC = 11, 64, 9153, 9175, 12


class bl_mlp_hparams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_int64), ("n_val", C.c_int64)]


TUNING_FIELDS = ["tile_w", "tile_h", "transfer_waves_per_cu", "refill_min", "chunk_rays", "order"]


def tuning(d):
    t = bl_tuning()
    for k in TUNING_FIELDS:
        setattr(t, k, int(d.get(k, {"refill_min": 1}.get(k, 0))))
    t.reserved = 0
    return t


def tuning_dict(t):
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


_lib = None


def load():
    """Load libblgpu.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2203_15963_amd/build.py "
                           "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.bl_abi_version.restype = C.c_int
    L.bl_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.bl_create.restype = C.c_int
    L.bl_destroy.argtypes = [vp]
    L.bl_last_error.argtypes = [vp]
    L.bl_last_error.restype = C.c_char_p
    L.bl_grid_create.argtypes = [vp, C.POINTER(bl_grid_desc), C.POINTER(vp)]
    L.bl_grid_create.restype = C.c_int
    L.bl_grid_destroy.argtypes = [vp]
    L.bl_camera_rays.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), vp, vp]
    L.bl_camera_rays.restype = C.c_int
    L.bl_trace_geodesics.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime),
                                     C.POINTER(bl_integrator), vp, vp]
    L.bl_trace_geodesics.restype = C.c_int
    L.bl_render.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                            vp, C.POINTER(bl_plasma), C.POINTER(bl_mode), vp, vp]
    L.bl_render.restype = C.c_int
    L.bl_render_noalloc.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                                    vp, C.POINTER(bl_plasma), C.POINTER(bl_mode), vp, vp]
    L.bl_render_noalloc.restype = C.c_int
    L.bl_render_batch.argtypes = [vp, i32, C.POINTER(bl_image_desc), C.POINTER(bl_integrator), vp,
                                  C.POINTER(bl_plasma), C.POINTER(bl_mode), C.POINTER(bl_tuning)]
    L.bl_render_batch.restype = C.c_int
    L.bl_render_multifreq.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                                      vp, C.POINTER(bl_plasma), C.POINTER(bl_mode), i32, C.POINTER(C.c_double),
                                      C.POINTER(vp), C.POINTER(vp)]
    L.bl_render_multifreq.restype = C.c_int
    L.bl_render_models.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                                   vp, i32, C.POINTER(C.c_double), C.POINTER(bl_plasma), C.POINTER(bl_mode),
                                   C.POINTER(vp), C.POINTER(vp)]
    L.bl_render_models.restype = C.c_int
    L.bl_render_averages.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                                     vp, C.POINTER(bl_plasma), C.POINTER(bl_mode), vp, vp, vp]
    L.bl_render_averages.restype = C.c_int
    L.bl_render_adaptive.argtypes = [vp, C.POINTER(bl_camera), C.POINTER(bl_spacetime), C.POINTER(bl_integrator),
                                     vp, C.POINTER(bl_plasma), C.POINTER(bl_mode), C.POINTER(bl_adaptive), C.c_int32,
                                     vp, vp, vp, C.POINTER(C.c_int32)]
    L.bl_render_adaptive.restype = C.c_int
    L.bl_set_cuts.argtypes = [vp, C.POINTER(bl_cuts)]
    L.bl_set_cuts.restype = C.c_int
    L.bl_set_tuning.argtypes = [vp, C.POINTER(bl_tuning)]
    L.bl_set_tuning.restype = C.c_int
    L.bl_get_tuning.argtypes = [vp, C.POINTER(bl_tuning)]
    L.bl_get_tuning.restype = C.c_int
    L.bl_autotune.argtypes = [vp, i32, C.POINTER(bl_image_desc), C.POINTER(bl_integrator), vp,
                              C.POINTER(bl_plasma), C.POINTER(bl_mode), i32, C.POINTER(bl_tuning),
                              C.POINTER(C.c_double)]
    L.bl_autotune.restype = C.c_int
    L.bl_steplog.argtypes = [vp, i32, C.POINTER(bl_image_desc), C.POINTER(bl_integrator), vp, i64,
                             C.POINTER(C.c_int64)]
    L.bl_steplog.restype = C.c_int
    L.bl_mlp_init.argtypes = [vp, vp, i64, i64, vp]
    L.bl_mlp_init.restype = C.c_int
    L.bl_mlp_train.argtypes = [vp, vp, i64, C.POINTER(bl_mlp_hparams), vp, vp]
    L.bl_mlp_train.restype = C.c_int
    L.bl_mlp_forward_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.bl_mlp_forward_backward.restype = C.c_int
    L.bl_set_step_model.argtypes = [vp, vp]
    L.bl_set_step_model.restype = C.c_int
    L.bl_eval_samples.argtypes = [vp, C.POINTER(bl_spacetime), vp, C.POINTER(bl_plasma), i64, vp, vp, vp]
    L.bl_eval_samples.restype = C.c_int
    L.bl_eval_coeffs.argtypes = [vp, C.c_int32, C.POINTER(bl_plasma), i64, vp, vp]
    L.bl_eval_coeffs.restype = C.c_int
    L.bl_eval_stokes.argtypes = [vp, C.c_int32, C.c_int32, i64, vp, vp, vp]
    L.bl_eval_stokes.restype = C.c_int
    L.bl_profile_enable.argtypes = [vp, C.c_int]
    L.bl_profile_enable.restype = C.c_int
    L.bl_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.bl_profile_read.restype = C.c_int
    if L.bl_abi_version() != ABI_VERSION:
        raise RuntimeError(f"libblgpu ABI {L.bl_abi_version()} != binding ABI {ABI_VERSION}")
    _lib = L
    return L


# ------------------------------------------------------------ parameters
def camera(d):
    c = bl_camera()
    c.r, c.theta, c.phi = d["r"], d["theta"], d.get("phi", 0.0)
    for k in range(3):
        c.u_normal[k] = d.get("u_normal", (0.0, 0.0, 0.0))[k]
        c.k_cov[k] = d.get("k_cov", (1.0, 0.0, 0.0))[k]
    c.width, c.n = d["width"], int(d["n"])
    c.freq_mode = int(d.get("freq_mode", 0))
    c.kind = int(d.get("kind", 0))
    c.psi, c.nu_hz = d.get("psi", 0.0), d.get("nu_hz", 230e9)
    return c


def spacetime(d):
    s = bl_spacetime()
    s.a, s.mass_msun, s.r_in = d["a"], d.get("mass_msun", 4.152e6), d["r_in"]
    s.flat = int(d.get("flat", 0))
    return s


def integrator(d):
    g = bl_integrator()
    g.f_abs, g.f_rel = d.get("f_abs", 1e-8), d.get("f_rel", 1e-8)
    g.ds_max, g.h0_frac = d.get("ds_max", 0.0), d.get("h0_frac", 0.1)
    g.max_steps = int(d.get("max_steps", 100000))
    g.record_cap = int(d.get("record_cap", 0))
    return g


def plasma(d):
    p = bl_plasma()
    p.mu, p.ne_ni = d.get("mu", 0.5), d.get("ne_ni", 1.0)
    p.r_high, p.r_low = d.get("r_high", 20.0), d.get("r_low", 1.0)
    p.sigma_max = d.get("sigma_max", 1.0)
    p.polarized, p.interp = int(d.get("polarized", 0)), int(d.get("interp", 1))
    # electron populations: fractions (thermal, power law, kappa) and parameters
    # (defaults: the paper's p = 3, gamma 4..1000, kappa = 4, w = 1/2)
    fr = d.get("fractions", (1.0, 0.0, 0.0))
    for k in range(3):
        p.fractions[k] = float(fr[k])
    p.pl_p, p.pl_gamma_min = d.get("pl_p", 3.0), d.get("pl_gamma_min", 4.0)
    p.pl_gamma_max = d.get("pl_gamma_max", 1000.0)
    p.kappa, p.kappa_w = d.get("kappa", 4.0), d.get("kappa_w", 0.5)
    return p


def mode(precision=0, step_model=0):
    m = bl_mode()
    m.precision, m.step_model = int(precision), int(step_model)
    return m


class BlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAME.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Grid:
    """Device-resident fluid data; keeps the primitive tensor alive."""

    def __init__(self, ctx, bounds, prims, rho_unit):
        import torch
        self.ctx = ctx
        self.bounds = np.ascontiguousarray(bounds, dtype=np.float64)
        if not isinstance(prims, torch.Tensor):
            prims = torch.from_numpy(np.ascontiguousarray(prims))
        self.prims = prims.to(ctx.device).contiguous()
        nb, bnz, bny, bnx, nv = self.prims.shape
        if nv != 8 or self.bounds.shape != (nb, 6):
            raise ValueError("prims must be [nb, bnz, bny, bnx, 8] and bounds [nb, 6]")
        d = bl_grid_desc()
        d.n_blocks, d.bnx, d.bny, d.bnz = nb, bnx, bny, bnz
        d.bounds = self.bounds.ctypes.data_as(C.POINTER(C.c_double))
        d.prims = C.c_void_p(self.prims.data_ptr())
        d.dtype = 0 if self.prims.dtype == torch.float64 else 1
        d.rho_unit = rho_unit
        h = C.c_void_p()
        ctx._check(load().bl_grid_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            load().bl_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A library context on one GPU, enqueuing on a torch stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        st = load().bl_create(int(device), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != 0:
            raise BlError(st, "bl_create failed")
        self.handle = h

    def _check(self, st):
        if st != 0:
            raise BlError(st, load().bl_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            load().bl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid(self, g):
        """Grid from a dict(bounds, prims, rho_unit) (numpy or torch prims)."""
        return Grid(self, g["bounds"], g["prims"], g["rho_unit"])

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def camera_rays(self, cam, st, out=None):
        n = int(cam["n"])
        state = self._empty(n * n, 8) if out is None else out[0]
        norm = self._empty(n * n) if out is None else out[1]
        c, s = camera(cam), spacetime(st)
        self._check(load().bl_camera_rays(self.handle, C.byref(c), C.byref(s), _ptr(state), _ptr(norm)))
        return state, norm

    def trace_geodesics(self, cam, st, integ):
        n = int(cam["n"])
        state, aux = self._empty(n * n, 8), self._empty(NAUX, n, n)
        c, s, g = camera(cam), spacetime(st), integrator(integ)
        self._check(load().bl_trace_geodesics(self.handle, C.byref(c), C.byref(s), C.byref(g),
                                              _ptr(state), _ptr(aux)))
        return state, aux

    def render(self, cam, st, integ, grid, pl, precision=0, image=None, aux=None, step_model=0):
        n = int(cam["n"])
        image = self._empty(4, n, n) if image is None else image
        aux = self._empty(NAUX, n, n) if aux is None else aux
        c, s, g, p, m = camera(cam), spacetime(st), integrator(integ), plasma(pl), mode(precision, step_model)
        self._check(load().bl_render(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle,
                                     C.byref(p), C.byref(m), _ptr(image), _ptr(aux)))
        return image, aux

    def render_noalloc(self, cam, st, integ, grid, pl, image, aux, precision=0, step_model=0):
        """bl_render_noalloc: the render into caller-given outputs with every
        workspace buffer taken from the library's static scratch array."""
        c, s, g, p, m = camera(cam), spacetime(st), integrator(integ), plasma(pl), mode(precision, step_model)
        self._check(load().bl_render_noalloc(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle,
                                             C.byref(p), C.byref(m), _ptr(image), _ptr(aux)))
        return image, aux

    def render_averages(self, cam, st, integ, grid, pl, precision=0, step_model=0):
        """Render one image and its averaged quantities; returns (image, aux,
        avg [NAVG, N, N])."""
        n = int(cam["n"])
        image, aux, avg = self._empty(4, n, n), self._empty(NAUX, n, n), self._empty(NAVG, n, n)
        c, s, g, p, m = camera(cam), spacetime(st), integrator(integ), plasma(pl), mode(precision, step_model)
        self._check(load().bl_render_averages(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle,
                                              C.byref(p), C.byref(m), _ptr(image), _ptr(aux), _ptr(avg)))
        return image, aux, avg

    def render_adaptive(self, cam, st, integ, grid, pl, ad, max_blocks=None, precision=0, step_model=0):
        """Adaptive render; returns a list over the levels reached of (blocks
        [n][3] int32 (level, bx, by), image [n][4][B][B], aux [n][NAUX][B][B]),
        device tensors viewing one allocation of max_blocks blocks (default:
        every block of every level)."""
        import torch
        b, lmax = int(ad["block"]), int(ad["max_level"])
        if max_blocks is None:
            max_blocks = sum((int(cam["n"]) // b) ** 2 * 4 ** l for l in range(lmax + 1))
        blocks = torch.empty(max_blocks, 3, dtype=torch.int32, device=self.device)
        image, aux = self._empty(max_blocks, 4, b, b), self._empty(max_blocks, NAUX, b, b)
        counts = (C.c_int32 * (lmax + 1))()
        c, s, g, p, m = camera(cam), spacetime(st), integrator(integ), plasma(pl), mode(precision, step_model)
        a = adaptive(ad)
        self._check(load().bl_render_adaptive(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle,
                                              C.byref(p), C.byref(m), C.byref(a), int(max_blocks), _ptr(blocks),
                                              _ptr(image), _ptr(aux), counts))
        out, off = [], 0
        for l in range(lmax + 1):
            n = counts[l]
            if n == 0:
                break
            out.append((blocks[off:off + n], image[off:off + n], aux[off:off + n]))
            off += n
        return out

    def render_multifreq(self, cam, st, integ, grid, pl, nu_hz, precision=0, step_model=0, outputs=None):
        """One camera at several frequencies from one geodesic pass; returns a
        list of (image, aux) tensors, one per frequency (cam["nu_hz"] is
        ignored)."""
        n, k = int(cam["n"]), len(nu_hz)
        outs = outputs if outputs is not None else [(self._empty(4, n, n), self._empty(NAUX, n, n)) for _ in range(k)]
        c, s, g, p, m = camera(cam), spacetime(st), integrator(integ), plasma(pl), mode(precision, step_model)
        nus = (C.c_double * k)(*[float(v) for v in nu_hz])
        ims = (C.c_void_p * k)(*[im.data_ptr() for im, _ in outs])
        axs = (C.c_void_p * k)(*[ax.data_ptr() for _, ax in outs])
        self._check(load().bl_render_multifreq(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle,
                                               C.byref(p), C.byref(m), k, nus, ims, axs))
        return outs

    def render_models(self, cam, st, integ, grid, plasmas, nu_hz=None, precision=0, step_model=0, outputs=None):
        """One camera, one geodesic pass, one output per plasma model (list of
        plasma dicts) at nu_hz[k] (or cam["nu_hz"] for all when None);
        returns a list of (image, aux) tensors."""
        n, k = int(cam["n"]), len(plasmas)
        if nu_hz is not None and len(nu_hz) != k:
            raise ValueError("one frequency per plasma model")
        outs = outputs if outputs is not None else [(self._empty(4, n, n), self._empty(NAUX, n, n)) for _ in range(k)]
        c, s, g, m = camera(cam), spacetime(st), integrator(integ), mode(precision, step_model)
        pls = (bl_plasma * k)(*[plasma(p) for p in plasmas])
        nus = None if nu_hz is None else (C.c_double * k)(*[float(v) for v in nu_hz])
        ims = (C.c_void_p * k)(*[im.data_ptr() for im, _ in outs])
        axs = (C.c_void_p * k)(*[ax.data_ptr() for _, ax in outs])
        self._check(load().bl_render_models(self.handle, C.byref(c), C.byref(s), C.byref(g), grid.handle, k, nus,
                                            pls, C.byref(m), ims, axs))
        return outs

    def _batch_descs(self, images, outputs):
        """images: list of (camera dict, spacetime dict); outputs: list of
        (image, aux) tensors or None to allocate."""
        n = len(images)
        descs = (bl_image_desc * n)()
        outs = []
        for k, (cam, st) in enumerate(images):
            nn = int(cam["n"])
            if outputs is None:
                im, ax = self._empty(4, nn, nn), self._empty(NAUX, nn, nn)
            else:
                im, ax = outputs[k]
            descs[k].cam = camera(cam)
            descs[k].st = spacetime(st)
            descs[k].image_out = C.c_void_p(im.data_ptr())
            descs[k].aux_out = C.c_void_p(ax.data_ptr())
            outs.append((im, ax))
        return descs, outs

    def render_batch(self, images, integ, grid, pl, precision=0, tuning_=None, outputs=None, step_model=0):
        """Render many images in one batched launch sequence; returns a list
        of (image, aux) tensors in the order given."""
        descs, outs = self._batch_descs(images, outputs)
        g, p, m = integrator(integ), plasma(pl), mode(precision, step_model)
        t = C.byref(tuning(tuning_)) if tuning_ is not None else None
        self._check(load().bl_render_batch(self.handle, len(images), descs, C.byref(g), grid.handle, C.byref(p),
                                           C.byref(m), t))
        return outs

    def set_cuts(self, d):
        """Install data cuts (see cuts()) for the following renders; None
        removes them."""
        self._check(load().bl_set_cuts(self.handle, C.byref(cuts(d)) if d is not None else None))

    def set_tuning(self, d):
        t = tuning(d)
        self._check(load().bl_set_tuning(self.handle, C.byref(t)))

    def get_tuning(self):
        t = bl_tuning()
        self._check(load().bl_get_tuning(self.handle, C.byref(t)))
        return tuning_dict(t)

    def autotune(self, images, integ, grid, pl, precision=0, max_trials=16, outputs=None):
        """Run the library's autotuner on this batch; returns (tuning dict,
        ms per batch) and installs the tuning on the context."""
        descs, outs = self._batch_descs(images, outputs)
        g, p, m = integrator(integ), plasma(pl), mode(precision)
        best, ms = bl_tuning(), C.c_double()
        self._check(load().bl_autotune(self.handle, len(images), descs, C.byref(g), grid.handle, C.byref(p),
                                       C.byref(m), int(max_trials), C.byref(best), C.byref(ms)))
        return tuning_dict(best), ms.value

    # ------------------------------------------------ learned step proposals
    def steplog(self, images, integ, capacity):
        """Step log of the plain integrator over the rays of the images;
        returns (records [min(n, capacity)][12] float32 tensor, n)."""
        import torch
        descs, outs = self._batch_descs(images, None)
        rec = torch.empty(int(capacity), STEPLOG_REC, dtype=torch.float32, device=self.device)
        n = C.c_int64()
        g = integrator(integ)
        self._check(load().bl_steplog(self.handle, len(images), descs, C.byref(g), _ptr(rec), int(capacity),
                                      C.byref(n)))
        return rec[:min(n.value, int(capacity))], n.value

    def mlp_init(self, records, seed=0):
        import torch
        model = torch.empty(MLP_NMODEL, dtype=torch.float32, device=self.device)
        self._check(load().bl_mlp_init(self.handle, _ptr(records), records.shape[0], int(seed), _ptr(model)))
        return model

    def mlp_train(self, records, model, epochs=4, batch=8192, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
                  n_val=0):
        """Train model (in place); returns losses [epochs][2] (train, held out)."""
        import torch
        hp = bl_mlp_hparams()
        hp.epochs, hp.batch, hp.lr, hp.beta1, hp.beta2, hp.eps = int(epochs), int(batch), lr, beta1, beta2, eps
        hp.seed, hp.n_val = int(seed), int(n_val)
        losses = torch.empty(int(epochs), 2, dtype=torch.float32, device=self.device)
        self._check(load().bl_mlp_train(self.handle, _ptr(records), records.shape[0], C.byref(hp), _ptr(model),
                                        _ptr(losses)))
        return losses

    def mlp_forward_backward(self, model, records):
        """(outputs [n], mean squared error [1], gradient [NPARAM])."""
        import torch
        n = records.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=self.device)
        self._check(load().bl_mlp_forward_backward(self.handle, _ptr(model), _ptr(records), n, _ptr(y), _ptr(loss),
                                                   _ptr(grad)))
        return y, loss, grad

    def set_step_model(self, model):
        self._check(load().bl_set_step_model(self.handle, _ptr(model)))

    def profile_enable(self, on=True):
        self._check(load().bl_profile_enable(self.handle, int(bool(on))))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read."""
        ms = (C.c_double * NKERNEL)()
        nl = (C.c_int64 * NKERNEL)()
        self._check(load().bl_profile_read(self.handle, ms, nl))
        return {KERNEL_NAMES[k]: (ms[k], nl[k]) for k in range(NKERNEL)}

    def eval_coeffs(self, pl, rows, precision=0):
        """bl_eval_coeffs: fluid-frame coefficients for rows [n][5] = n_e,
        Theta_e, B, nu, cos theta_B; returns [n][8]."""
        import torch
        rows = torch.as_tensor(rows, dtype=torch.float64, device=self.device).contiguous()
        n = rows.shape[0]
        out = self._empty(n, 8)
        p = plasma(pl)
        self._check(load().bl_eval_coeffs(self.handle, int(precision), C.byref(p), n, _ptr(rows), _ptr(out)))
        return out

    def eval_stokes(self, coeffs, s0, precision=0, general=0):
        """bl_eval_stokes: one plasma substep per row of coeffs [n][8] from
        s0 [n][4]; returns S1 [n][4]."""
        import torch
        coeffs = torch.as_tensor(coeffs, dtype=torch.float64, device=self.device).contiguous()
        s0 = torch.as_tensor(s0, dtype=torch.float64, device=self.device).contiguous()
        n = coeffs.shape[0]
        out = self._empty(n, 4)
        self._check(load().bl_eval_stokes(self.handle, int(precision), int(general), n, _ptr(coeffs), _ptr(s0),
                                          _ptr(out)))
        return out

    def eval_samples(self, st, grid, pl, states, norms):
        import torch
        states = torch.as_tensor(states, dtype=torch.float64, device=self.device).contiguous()
        norms = torch.as_tensor(norms, dtype=torch.float64, device=self.device).contiguous()
        n = states.shape[0]
        out = self._empty(n, NSAMPLE_OUT)
        s, p = spacetime(st), plasma(pl)
        self._check(load().bl_eval_samples(self.handle, C.byref(s), grid.handle, C.byref(p), n,
                                           _ptr(states), _ptr(norms), _ptr(out)))
        return out
