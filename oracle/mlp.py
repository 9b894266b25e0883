"""Plain FP64 reference of the step-proposal network (forward, loss,
backward) and of the step-log features.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library.  Written from the definitions, with numpy matrix products as the
only library primitive:

  x_n  = (x - mean) / std                       (11 features)
  z1   = W1 x_n + b1,  h1 = silu(z1)             (64)
  z2   = W2 h1 + b2,   h2 = silu(z2)             (64)
  z3   = W3 h2 + b3,   h3 = silu(z3)             (64)
  y    = w4 . h3 + b4,  silu(z) = z / (1 + e^-z)
  L    = mean over rows of (y - target)^2

and the gradient of L by the chain rule, silu'(z) = s (1 + z (1 - s)),
s = 1 / (1 + e^-z).  With bf16=True the operands that the GPU feeds to its
BF16 matrix cores are rounded the same way (to FP32, then to BF16 with
round-to-nearest-even): normalised inputs, W1, W2, W3, h1, h2 and the
pre-activation gradients dz1, dz2, dz3 where they enter a matrix product;
everything else stays FP64.

Model vector layout: W1[64][11], b1[64], W2[64][64], b2[64], W3[64][64],
b3[64], w4[64], b4, mean[11], std[11].
"""
import numpy as np

NIN, NH = 11, 64
W1, B1 = 0, NH * NIN
W2 = B1 + NH
B2 = W2 + NH * NH
W3 = B2 + NH
B3 = W3 + NH * NH
W4 = B3 + NH
B4 = W4 + NH
NPARAM = B4 + 1
MU = NPARAM
SIG = MU + NIN
NMODEL = SIG + NIN


def bf16_round(x):
    """Round to FP32 and then to BF16 (round to nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def unpack(model):
    m = np.asarray(model, dtype=np.float64)
    return dict(W1=m[W1:B1].reshape(NH, NIN), b1=m[B1:W2], W2=m[W2:B2].reshape(NH, NH), b2=m[B2:W3],
                W3=m[W3:B3].reshape(NH, NH), b3=m[B3:W4], w4=m[W4:B4], b4=m[B4], mu=m[MU:SIG], sig=m[SIG:NMODEL])


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def forward(model, X, bf16=False):
    """X [n][11] raw features -> (y [n], cache)."""
    p = unpack(model)
    r = bf16_round if bf16 else (lambda a: a)
    xn = r((np.asarray(X, np.float64) - p["mu"]) / p["sig"])
    z1 = xn @ r(p["W1"]).T + p["b1"]
    h1 = silu(z1)
    z2 = r(h1) @ r(p["W2"]).T + p["b2"]
    h2 = silu(z2)
    z3 = r(h2) @ r(p["W3"]).T + p["b3"]
    h3 = silu(z3)
    y = h3 @ p["w4"] + p["b4"]
    return y, dict(p=p, xn=xn, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, r=r)


def loss_and_grad(model, X, target, bf16=False):
    """Mean squared error of y against target and its gradient with respect
    to the first NPARAM model entries."""
    y, c = forward(model, X, bf16)
    p, r = c["p"], c["r"]
    n = len(y)
    d = y - np.asarray(target, np.float64)
    loss = float(np.mean(d * d))
    dy = 2.0 * d / n
    g = np.zeros(NPARAM)
    g[W4:B4] = c["h3"].T @ dy
    g[B4] = dy.sum()
    dz3 = np.outer(dy, p["w4"]) * dsilu(c["z3"])
    g[W3:B3] = (r(dz3).T @ r(c["h2"])).ravel()
    g[B3:W4] = dz3.sum(0)
    dz2 = (r(dz3) @ r(p["W3"])) * dsilu(c["z2"])
    g[W2:B2] = (r(dz2).T @ r(c["h1"])).ravel()
    g[B2:W3] = dz2.sum(0)
    dz1 = (r(dz2) @ r(p["W2"])) * dsilu(c["z1"])
    g[W1:B1] = (r(dz1).T @ c["xn"]).ravel()
    g[B1:W2] = dz1.sum(0)
    return y, loss, g


def features(y7, kt, a, h_last, eps_last):
    """Step-log features of a state: x^mu, k_mu (k_t held fixed), spin,
    log|h| and log eps (eps floored at 1e-10) of the last accepted step."""
    y7 = np.asarray(y7, np.float64)
    return np.array([y7[0], y7[1], y7[2], y7[3], kt, y7[4], y7[5], y7[6], a, np.log(abs(h_last)),
                     np.log(max(eps_last, 1e-10))])
