"""The polarized plasma substep of the image kernels alone (paper section 2.4:
the constant-coefficient solution of the polarized transfer equation over one
segment), through bl_eval_stokes, against the oracle's exact solution (the
exponential of the augmented matrix, or_stokes_exact) over coefficient sets
far wider than the images reach: optical depths 1e-9 to 40, polarized
fractions of the absorption up to 1, Faraday rotation and conversion depths
up to 1e3 rad per segment, the optical-depth cap (M^-1 J at aI >= 100), and
input states up to 1e6 times the emission.

Both substeps in both precisions: the thermal closed form (Kirchhoff's law:
J = (jI/aI) M e_I) and the general one of the nonthermal kernels (any source
vector).  Error measure: |S_gpu - S_exact| (largest Stokes component) over
|I_exact| + 8 |I_0| u, u the unit roundoff of the arithmetic (2^-53 in FP64,
2^-24 in FP32): the result to a relative tolerance plus a few units in the
last place of the input state, which the propagation of an input much larger
than the result cannot do better than.  FP64 <= 1e-10; FP32 <= 5e-5 for
rotation depths up to 30 rad per segment (measured 1.2e-6 for the thermal
form; 1.9e-5 for the general one, at the optical-depth cap with almost fully
polarized absorption, where a - L1 << a is formed from two nearly equal FP32
numbers) and <= 2e-4 up to 1e3 rad (FP32 resolves a phase of 1e3 rad to
6e-5 rad; measured 7.4e-5)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2203_15963_amd import blgpu
    blgpu.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = blgpu.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _sets(n, thermal, seed):
    rng = np.random.default_rng(seed)
    C = np.zeros((n, 8))
    S0 = np.zeros((n, 4))
    rot = np.zeros(n)
    for i in range(n):
        tau = 10 ** rng.uniform(-9, 1.6)
        if rng.uniform() < 0.03:
            tau = rng.uniform(100, 300)            # the optical-depth cap
        pol = rng.uniform(0, 1) if rng.uniform() > 0.2 else 0.0
        ang = rng.uniform(0, 2 * math.pi)
        aQ, aV = tau * pol * math.cos(ang), tau * pol * math.sin(ang)
        r = 10 ** rng.uniform(-9, 3) if rng.uniform() > 0.25 else 0.0
        ra = rng.uniform(0, 2 * math.pi)
        rQ, rV = r * math.cos(ra), r * math.sin(ra)
        jI = 10 ** rng.uniform(-3, 3)
        if thermal:
            B = jI / tau
            jQ, jV = B * aQ, B * aV                # Kirchhoff: J = B M e_I
        else:
            jp, ja = rng.uniform(0, 1), rng.uniform(0, 2 * math.pi)
            jQ, jV = jI * jp * math.cos(ja), jI * jp * math.sin(ja)
        C[i] = [jI, jQ, jV, tau, aQ, aV, rQ, rV]
        I0 = 10 ** rng.uniform(-3, 3) * jI / max(tau, 1e-3) * rng.choice([0.0, 1.0])
        p0 = rng.uniform(0, 1)
        a0, b0 = rng.uniform(0, 2 * math.pi, 2)
        S0[i] = [I0, I0 * p0 * math.cos(a0) * math.cos(b0), I0 * p0 * math.sin(a0) * math.cos(b0),
                 I0 * p0 * math.sin(b0)]
        rot[i] = r
    return C, S0, rot


def _exact(oracle, C, S0):
    out = np.zeros_like(S0)
    for i in range(len(C)):
        jI, jQ, jV, aI, aQ, aV, rQ, rV = C[i]
        M = np.array([[aI, aQ, 0, aV], [aQ, aI, rV, 0], [0, -rV, aI, rQ], [aV, 0, -rQ, aI]], dtype=np.float64)
        J = np.array([jI, jQ, 0.0, jV])
        if aI >= 100.0:
            out[i] = np.linalg.solve(M, J)
        else:
            out[i] = oracle.stokes_exact(S0[i], J, M, 1.0)
    return out


@pytest.mark.parametrize("general", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_substep_matches_exact_solution(ctx, oracle, precision, general):
    C, S0, rot = _sets(6000, thermal=(general == 0), seed=5 + 2 * precision + general)
    ref = _exact(oracle, C, S0)
    got = ctx.eval_stokes(C, S0, precision=precision, general=general)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    u = 2.0 ** -53 if precision == 0 else 2.0 ** -24
    err = np.abs(got - ref).max(axis=1) / (np.abs(ref[:, 0]) + 8 * u * np.abs(S0[:, 0]) + 1e-300)
    assert np.isfinite(got).all()
    slow = rot <= 30.0
    ws = int(np.flatnonzero(slow)[np.argmax(err[slow])])
    print(f"[gpu-stokes] worst with rotation <= 30 rad: c {C[ws].tolist()} S0 {S0[ws].tolist()} "
          f"exact {ref[ws].tolist()} got {got[ws].tolist()}", flush=True)
    w = int(np.argmax(err))
    print(f"[gpu-stokes] precision {precision} general {general}: worst {err.max():.3e}, "
          f"rotation <= 30 rad {err[slow].max():.3e}, median {np.median(err):.3e}; worst case c {C[w].tolist()} "
          f"S0 {S0[w].tolist()} exact {ref[w].tolist()} got {got[w].tolist()}", flush=True)
    if precision == 0:
        assert err.max() <= 1e-10
    else:
        assert err[slow].max() <= 5e-5
        assert err.max() <= 2e-4


def test_substep_rejects_bad_arguments(ctx):
    from paper_2203_15963_amd import blgpu
    C, S0, _ = _sets(4, thermal=True, seed=1)
    with pytest.raises(blgpu.BlError):
        ctx.eval_stokes(C, S0, precision=2)
    with pytest.raises(blgpu.BlError):
        ctx.eval_stokes(C, S0, general=3)
    torch.cuda.synchronize()
