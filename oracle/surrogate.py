"""Oracle of the learned collide: training pairs, the MLP (FP64, optionally
rounding to BF16 where the GPU kernels do), its gradient, Adam, the
conserved-moment projection, the residual test and the surrogate collide.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definitions (the paper gives the plain collide; this learned replacement and
all its choices are readings stated here):
* Pair: (rho, u, T) drawn as in philox.pair_draws; f = f_eq(rho, u, T) + 1e-3
  w_p n_p; pre = f - w (shifted populations); post = collide(f) - w.
* Conserved part of shifted populations g: the orthogonal projection, in the
  inner product <a, b> = sum a b / w, onto w * {1, xi_x, xi_y, xi^2 - 2}:
      P(g)_p = w_p [ m0 + mx xi_px + my xi_py + mE (xi_p^2 - 2) / 4 ]
  with m0 = sum g, mx = sum g xi_x, my = sum g xi_y, mE = sum g (xi^2 - 2); the
  Gram matrix of these four functions under w is diag(1, 1, 1, 4).
* Network input z = g / w standardised per feature; target
  y = (g_eq - P(g)) / w standardised per feature, where g_eq = pre + tau (post - pre)
  is the equilibrium the pair encodes. The network learns the part of the
  equilibrium that the conserved moments do not fix.
* MLP 37 -> 128 -> 128 -> 37, GELU in its tanh form
  gelu(a) = a / (1 + exp(-2 c (a + 0.044715 a^3))), c = sqrt(2 / pi).
* Surrogate equilibrium: g_hat = P(g) + d - P(d), d = w (mu_y + sd_y o); the
  projection makes mass, momentum and energy of g_hat those of g exactly.
* Residual: largest deviation of g_hat's stress (sum xi_x xi_y, sum (xi_x^2 -
  xi_y^2)) and heat flux (sum xi xi^2) from the equilibrium values rho u_x
  u_y, rho (u_x^2 - u_y^2), rho u (|u|^2 + 4 T). A site falls back to the
  plain equilibrium if the residual exceeds the threshold or if (rho, |u|, T)
  leaves the training box [0.9, 1.1] x [0, 0.1] x [0.9, 1.1].
* BF16 emulation mirrors the GPU's training: inputs and weights rounded to
  BF16, hidden activations rounded to BF16 after GELU, sums in high
  precision; in the backward pass the output gradient and the
  pre-activation gradients are rounded to BF16 before the products, bias
  gradients use the unrounded ones.
* Inference form (binary16 hidden layer, the GPU's default for the learned
  collide): the inputs and W1 in BF16 as above; each pre-activation, taken
  as the FP32 value the GPU accumulates, rounded to binary16 (IEEE half,
  nearest even) and put through the GELU's tanh form evaluated in binary16
  arithmetic, one rounding per operation (gelu_f16); W2 and W3 rounded to
  binary16; sums in high precision.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm
from .lattice import Q, constants
from .philox import MASK, pair_draws, philox4x32_10, uniform_from_u32

HIDDEN = 128
PERTURBATION = 1e-3
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715
BOX = {"rho": (0.9, 1.1), "u": 0.1, "T": (0.9, 1.1)}
SHAPES = [("W1", (HIDDEN, Q)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (Q, HIDDEN)), ("b3", (Q,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
ADAM = {"beta1": 0.9, "beta2": 0.999, "eps": 1e-8}


# ---- pairs ------------------------------------------------------------------

def make_pairs(n: int, seed: int, tau: float, start: int = 0):
    """(pre, post), each (n, 37) FP64 shifted populations."""
    w = constants()["w"]
    rho, ux, uy, T, nrm = pair_draws(np.arange(start, start + n), seed)
    f = lbm.init(rho[:, None], ux[:, None], uy[:, None], T[:, None])[:, :, 0].T  # (n, 37)
    f = f + PERTURBATION * w * nrm
    post = lbm.collide(f.T[:, :, None], tau)[:, :, 0].T
    return np.ascontiguousarray(f - w), np.ascontiguousarray(post - w)


# ---- conserved projection and residual ----------------------------------------

def _basis():
    xi = constants()["xi"]
    return np.stack([np.ones(Q), xi[:, 0], xi[:, 1], (xi ** 2).sum(1) - 2.0])  # (4, 37)


def gram():
    """Gram matrix sum_p w_p phi_a(p) phi_b(p) of the four conserved functions."""
    phi = _basis()
    return (phi * constants()["w"]) @ phi.T


def conserved_part(g: np.ndarray) -> np.ndarray:
    phi = _basis()
    coef = g @ phi.T / np.diag(gram())
    return constants()["w"] * (coef @ phi)


def macro(g: np.ndarray):
    """rho, ux, uy, T of shifted populations (FP64)."""
    xi = constants()["xi"]
    drho = g.sum(-1)
    rho = 1.0 + drho
    ux = (g @ xi[:, 0]) / rho
    uy = (g @ xi[:, 1]) / rho
    e2 = g @ ((xi ** 2).sum(1) - 2.0)
    u2 = ux * ux + uy * uy
    T = 1.0 + (e2 - rho * u2) / (2.0 * rho)
    return rho, ux, uy, T


def residual(g_hat: np.ndarray, rho, ux, uy, T) -> np.ndarray:
    xi = constants()["xi"]
    x, y = xi[:, 0], xi[:, 1]
    x2 = x * x + y * y
    u2 = ux * ux + uy * uy
    r = np.stack([
        np.abs(g_hat @ (x * y) - rho * ux * uy),
        np.abs(g_hat @ (x * x - y * y) - rho * (ux * ux - uy * uy)),
        np.abs(g_hat @ (x * x2) - rho * ux * (u2 + 4.0 * T)),
        np.abs(g_hat @ (y * x2) - rho * uy * (u2 + 4.0 * T)),
    ])
    return r.max(0)


def in_box(rho, ux, uy, T):
    return ((rho >= BOX["rho"][0]) & (rho <= BOX["rho"][1]) & (np.sqrt(ux * ux + uy * uy) <= BOX["u"])
            & (T >= BOX["T"][0]) & (T <= BOX["T"][1]))


# ---- MLP ------------------------------------------------------------------------

def bf16(x: np.ndarray) -> np.ndarray:
    """Round to BF16 (nearest even), via the FP32 value as the GPU does."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3(x) -> np.ndarray:
    """Round to FP8 e4m3 (the OCP "fn" variant: 1 sign, 4 exponent bits with
    bias 7, 3 mantissa bits, no infinities, largest finite value 448),
    nearest with ties to an even mantissa; magnitudes that round beyond 448
    become NaN (there is no saturation). Subnormals step by 2^-9."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, e = np.frexp(np.where(a > 0, a, 1.0))       # a = f 2^e, f in [0.5, 1)
    quantum = np.ldexp(1.0, np.maximum(e - 1, -6) - 3)
    r = np.rint(a / quantum) * quantum              # rint: ties to even
    r = np.where(a > 0, r, 0.0)
    out = np.copysign(r, x)
    return np.where(r > 448.0, np.nan, out)


# FP8 form of the hidden layer: its inputs h1 (first-layer activations) and
# weights W2 are rounded to e4m3 after scaling by powers of two, h1 by
# FP8_ACT_SCALE and W2 by 2^fp8_weight_exponent(W2), so that the largest
# weight lands in [128, 256); products are summed in high precision and
# divided by the scales again.
FP8_ACT_SCALE = 16.0


def fp8_weight_exponent(W2) -> int:
    m = float(np.max(np.abs(np.asarray(W2, dtype=np.float64))))
    _, e = np.frexp(m if m > 0 else 1.0)
    return int(8 - e)


def gelu(a):
    return a / (1.0 + np.exp(-2.0 * GELU_C * (a + GELU_A * a ** 3)))


def f16(x) -> np.ndarray:
    """Round to IEEE binary16 (11 significant bits, nearest with ties to
    even, subnormals below 2^-14, beyond the largest finite value 65504:
    infinity), returned as float64."""
    with np.errstate(over="ignore"):
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


# The tanh form written as a / (1 + 2^(a (K1 a^2 + K2))): K1 = -2 log2(e) c A,
# K2 = -2 log2(e) c, rounded to binary16 for the binary16 evaluation.
LOG2E = 1.0 / math.log(2.0)
GELU_K1_F16 = float(f16(-2.0 * LOG2E * GELU_C * GELU_A))
GELU_K2_F16 = float(f16(-2.0 * LOG2E * GELU_C))


def gelu_f16(a):
    """GELU evaluated in binary16 arithmetic, every operation rounded to
    nearest even: x = h(a); s = h(x^2); t = h(K1 s + K2) (one rounding for
    the product and sum); y = h(x t); e = h(2^y); r = h(1 / h(e + 1));
    result h(x r). The products and the sum of binary16 values are exact in
    float64 before their one rounding, and 2^y and 1 / d are rounded
    correctly from float64 (float64 error far below the binary16 spacing)."""
    x = f16(a)
    with np.errstate(over="ignore", invalid="ignore"):
        s = f16(x * x)
        t = f16(GELU_K1_F16 * s + GELU_K2_F16)
        y = f16(x * t)
        e = f16(np.exp2(y))
        r = f16(1.0 / f16(e + 1.0))
        return f16(x * r)


def gelu_grad(a):
    s = 1.0 / (1.0 + np.exp(-2.0 * GELU_C * (a + GELU_A * a ** 3)))
    return s + a * s * (1.0 - s) * 2.0 * GELU_C * (1.0 + 3.0 * GELU_A * a * a)


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shape)
        k += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """Xavier-uniform weights, zero biases. Weight element i (index in the
    packed vector) draws U from Philox counter (i, 0, 0xFFFFFFFF, 0) with key
    (seed mod 2^32, seed div 2^32), first word; value a (2U - 1), a =
    sqrt(6 / (fan_in + fan_out))."""
    theta = np.zeros(NPARAM)
    k = 0
    key = (seed & MASK, (seed >> 32) & MASK)
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W"):
            idx = np.arange(k, k + n, dtype=np.uint64)
            z = np.zeros_like(idx)
            u = uniform_from_u32(philox4x32_10((idx, z, z + np.uint64(0xFFFFFFFF), z), key)[0])
            a = math.sqrt(6.0 / (shape[0] + shape[1]))
            theta[k:k + n] = (a * (2.0 * u - 1.0)).astype(np.float32)
        k += n
    return theta


def f32(v) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def forward(theta, x_std, emulate=True, fp8=False, infer=False):
    """Network outputs (standardised) and the intermediates. emulate: the
    training form's BF16 roundings; with infer, the inference form's
    binary16 hidden layer instead (see the module notes); fp8: the hidden
    layer's inputs and weights in e4m3 (FP8 form above), the rest in BF16
    (emulate must be set)."""
    p = unpack(theta)
    q = bf16 if emulate else (lambda v: v)
    x = q(x_std)
    a1 = x @ q(p["W1"]).T + p["b1"]
    if emulate and infer and not fp8:
        h1 = gelu_f16(f32(a1))
        a2 = h1 @ f16(p["W2"]).T + p["b2"]
        h2 = gelu_f16(f32(a2))
        o = h2 @ f16(p["W3"]).T + p["b3"]
        return o, (x, a1, h1, a2, h2)
    if fp8:
        sw = 2.0 ** fp8_weight_exponent(p["W2"])
        h1 = e4m3(gelu(a1) * FP8_ACT_SCALE) / FP8_ACT_SCALE
        a2 = h1 @ (e4m3(p["W2"] * sw) / sw).T + p["b2"]
    else:
        h1 = q(gelu(a1))
        a2 = h1 @ q(p["W2"]).T + p["b2"]
    h2 = q(gelu(a2))
    o = h2 @ q(p["W3"]).T + p["b3"]
    return o, (x, a1, h1, a2, h2)


def loss_and_grad(theta, x_std, y_std, emulate=True):
    """Mean squared error over samples and the 37 outputs, and its gradient."""
    p = unpack(theta)
    q = bf16 if emulate else (lambda v: v)
    o, (x, a1, h1, a2, h2) = forward(theta, x_std, emulate)
    n = x_std.shape[0]
    diff = o - y_std
    loss = float((diff ** 2).sum() / (n * Q))
    dO = 2.0 * diff / (n * Q)
    dOq = q(dO)
    g = {"W3": dOq.T @ h2, "b3": dO.sum(0)}
    dA2 = (dOq @ q(p["W3"])) * gelu_grad(a2)
    dA2q = q(dA2)
    g["W2"], g["b2"] = dA2q.T @ h1, dA2.sum(0)
    dA1 = (dA2q @ q(p["W2"])) * gelu_grad(a1)
    dA1q = q(dA1)
    g["W1"], g["b1"] = dA1q.T @ x, dA1.sum(0)
    return loss, pack(g)


# ---- normalisation, targets -------------------------------------------------------

def features(pre, post, tau):
    """z = pre / w and y = (g_eq - P(pre)) / w of pairs."""
    w = constants()["w"]
    geq = pre + tau * (post - pre)
    return pre / w, (geq - conserved_part(pre)) / w


def fit_normalization(pre, post, tau) -> np.ndarray:
    """(4, 37): mean and standard deviation of z, then of y (deviations below
    1e-12 are replaced by 1)."""
    z, y = features(pre, post, tau)
    sz, sy = z.std(0), y.std(0)
    sz[sz < 1e-12] = 1.0
    sy[sy < 1e-12] = 1.0
    return np.stack([z.mean(0), sz, y.mean(0), sy])


# ---- training -----------------------------------------------------------------------

def epoch_order(n: int, seed: int, epoch: int):
    """Sample order of an epoch: i -> (a i + c) mod n, with (a, c) from Philox
    counter (epoch, 0, 0xFFFFFFFE, 0), key (seed mod 2^32, seed div 2^32): a is
    the first word reduced mod n, moved up to the next value coprime with n
    (at least 1); c is the second word mod n."""
    key = (seed & MASK, (seed >> 32) & MASK)
    r = philox4x32_10((epoch, 0, 0xFFFFFFFE, 0), key)
    a = int(r[0]) % n
    if a == 0:
        a = 1
    while math.gcd(a, n) != 1:
        a = a + 1 if a + 1 < n else 1
    c = int(r[1]) % n
    return a, c


def adam_step(theta, m, v, grad, t, lr):
    b1, b2, eps = ADAM["beta1"], ADAM["beta2"], ADAM["eps"]
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def cosine_lr(lr0, step, total):
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * step / total))


def train(pre, post, tau, theta0, norm, batch, epochs, lr0, seed, emulate=True, max_steps=None):
    """Minibatch Adam with a cosine learning-rate schedule. Steps per epoch:
    n // batch (the tail of each epoch's order is dropped). Returns
    (theta, per-step losses)."""
    n = pre.shape[0]
    z, y = features(pre, post, tau)
    zs = (z - norm[0]) / norm[1]
    ys = (y - norm[2]) / norm[3]
    theta = np.array(theta0, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    spe = n // batch
    total = spe * epochs
    losses = []
    step = 0
    for e in range(epochs):
        a, c = epoch_order(n, seed, e)
        for b in range(spe):
            idx = (a * (np.arange(b * batch, (b + 1) * batch, dtype=np.int64)) + c) % n
            loss, g = loss_and_grad(theta, zs[idx], ys[idx], emulate)
            theta, m, v = adam_step(theta, m, v, g, step + 1, cosine_lr(lr0, step, total))
            losses.append(loss)
            step += 1
            if max_steps is not None and step >= max_steps:
                return theta, losses
    return theta, losses


# ---- the learned collide --------------------------------------------------------------

def surrogate_equilibrium(g, theta, norm, emulate=True, fp8=False):
    """Learned equilibrium of the sites g; with emulate, in the GPU's
    inference form (binary16 hidden layer, or the FP8 form)."""
    w = constants()["w"]
    zs = (g / w - norm[0]) / norm[1]
    o, _ = forward(theta, zs, emulate, fp8, infer=True)
    d = w * (norm[2] + norm[3] * o)
    return conserved_part(g) + d - conserved_part(d)


def surrogate_collide(g, tau, theta, norm, threshold, emulate=True, fp8=False):
    """Post-collision shifted populations, fallback flags and residuals of the
    sites g (n, 37). A residual that is not a number (an FP8 activation out
    of range) counts as above the threshold."""
    w = constants()["w"]
    rho, ux, uy, T = macro(g)
    ghat = surrogate_equilibrium(g, theta, norm, emulate, fp8)
    res = residual(ghat, rho, ux, uy, T)
    fb = (~in_box(rho, ux, uy, T)) | ~(res <= threshold)
    if fb.any():
        idx = np.where(fb)[0]
        exact = lbm.init(rho[idx, None], ux[idx, None], uy[idx, None], T[idx, None])[:, :, 0].T - w
        ghat[idx] = exact
    return g + (ghat - g) / tau, fb, res


# ---- tolerance of the learned collide's parity ------------------------------------------

def bf16_ulp(v: np.ndarray) -> np.ndarray:
    """Unit in the last place of BF16 at |v| (8 significant bits): 2^(e - 7)
    for 2^e <= |v| < 2^(e + 1); 0 at v = 0."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def gelu_grad_max() -> float:
    """max over a of |gelu'(a)| (about 1.129, near a = 2.4), on a grid fine
    enough that the next grid point cannot exceed it by 1e-6."""
    a = np.linspace(-8.0, 8.0, 160001)
    return float(np.abs(gelu_grad(a)).max()) + 1e-6


def flip_bound(theta, norm, g, fp8=False, infer=True) -> np.ndarray:
    """B2 per site: the largest |change of g_hat_p| / w_p over populations
    that one BF16 rounding flip of one second-layer activation can cause at
    each of the sites g (n, 37): h2_j rounded to the neighbouring BF16 value,
    one unit in the last place at its own magnitude. Returns (n,). infer:
    h2 and W3 of the inference form (binary16, or the FP8 form's); else of
    the BF16 training form. In the binary16 form a hidden activation's flip
    is 2^-3 of this unit; the unit stays the BF16 one because the network's
    inputs are BF16 in every form and their flips reach the output too.

    Why flips set the tolerance: the GPU kernels and the emulating forward
    pass round the same quantities to BF16 at the same points; the values
    before rounding differ only by FP32 accumulation, the folded FP32
    standardisation and the hardware exponential (relative 1e-7 to 1e-6).
    So the two sides disagree by more than that only where a value lies
    that close to a BF16 rounding boundary, and then by one BF16 unit.

    Propagation of a second-layer flip of unit j: the output o
    (standardised) moves by |do_p| = |W3_pj| ulp(h2_j); d_p = w_p (mu_y +
    sd_y o_p) and g_hat = P(g) + d - P(d), so
      |dg_hat_p| / w_p <= sd_y,p |do_p|
                          + sum_a |phi_a(p)| sum_q w_q sd_y,q |do_q| |phi_a(q)| / G_aa
    (P: the projection onto the conserved functions phi, Gram diagonal
    G_aa), maximised over p and j with W3 at its BF16 values (fp8: the
    second-layer activations of the FP8 form). A flip of an
    input or of a first-layer activation reaches the output through the
    next layers and through the roundings it changes there; planted on this
    forward pass (over every unit, at sampled sites) it moves g_hat by at
    most 4 B2 of its site."""
    w = constants()["w"]
    p = unpack(theta)
    W3 = np.abs(f16(p["W3"]) if infer and not fp8 else bf16(p["W3"]))
    zs = (np.asarray(g, dtype=np.float64) / w - norm[0]) / norm[1]
    _, (_, _, _, _, h2) = forward(theta, zs, emulate=True, fp8=fp8, infer=infer)
    v = np.asarray(norm[3], dtype=np.float64)[:, None] * W3          # (37 outputs, 128 units)
    phi = np.abs(_basis())
    proj = phi.T @ ((phi * w) @ v / np.diag(gram())[:, None])
    col = (v + proj).max(axis=0)                                        # per unit j, per unit ulp
    return (bf16_ulp(h2) * col).max(axis=1)


def e4m3_ulp(v: np.ndarray) -> np.ndarray:
    """Spacing of e4m3 values at |v|: 2^(e - 3) for 2^e <= |v| < 2^(e + 1),
    e >= -6; 2^-9 below 2^-6."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a >= 2.0 ** -6, 2.0 ** (e - 3), 2.0 ** -9)


def fp8_flip_bound(theta, norm, g) -> np.ndarray:
    """B1 per site for the FP8 form: the largest |change of g_hat_p| / w_p
    that one e4m3 rounding flip of one hidden-layer input h1_j can cause,
    to first order: a2 moves by W2q[:, j] ulp(h1_j), h2 by at most
    max|gelu'| times that, and h2 reaches g_hat as in flip_bound. Returns
    (n,). (A flip also changes which way some h2 round to BF16; those are
    second-layer flips, bounded by flip_bound.)"""
    w = constants()["w"]
    p = unpack(theta)
    sw = 2.0 ** fp8_weight_exponent(p["W2"])
    W2q = np.abs(e4m3(p["W2"] * sw) / sw)                               # (128 out, 128 in)
    W3 = np.abs(bf16(p["W3"]))
    zs = (np.asarray(g, dtype=np.float64) / w - norm[0]) / norm[1]
    _, (_, _, h1, _, _) = forward(theta, zs, emulate=True, fp8=True)
    v = np.asarray(norm[3], dtype=np.float64)[:, None] * W3
    phi = np.abs(_basis())
    proj = phi.T @ ((phi * w) @ v / np.diag(gram())[:, None])
    col = (v + proj).max(axis=0)                                        # per second-layer unit
    per_input = gelu_grad_max() * (col @ W2q)                           # per first-layer unit j
    ulp = e4m3_ulp(h1 * FP8_ACT_SCALE) / FP8_ACT_SCALE
    return (ulp * per_input).max(axis=1)
