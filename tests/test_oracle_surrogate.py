"""Pins of the learned-collide oracle: the counter-based generator against
its published known-answer vectors, the pair law, the conserved-moment
projection, the residual closed forms, the MLP gradient against finite
differences, BF16 rounding, Adam and a short training run."""
import math

import numpy as np
import pytest

from oracle import lbm, surrogate as S
from oracle.philox import pair_draws, philox4x32_10, uniform_from_u32

# Known-answer vectors of Philox4x32-10 published with the Random123 library
# (Salmon et al., SC11): counter, key -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = philox4x32_10(ctr, key)
    assert tuple(int(v) for v in got) == want


def test_uniform_open_interval_and_fp32_exact():
    u = uniform_from_u32(np.array([0, 1, 511, 512, 0xFFFFFFFF], dtype=np.uint64))
    assert np.all((u > 0) & (u < 1))
    assert np.array_equal(u, u.astype(np.float32).astype(np.float64))
    assert u[0] == 2.0 ** -24 and u[-1] == 1 - 2.0 ** -24


def test_pair_law():
    rho, ux, uy, T, n = pair_draws(np.arange(20000), seed=3)
    assert rho.min() >= 0.9 and rho.max() <= 1.1 and T.min() >= 0.9 and T.max() <= 1.1
    r = np.sqrt(ux ** 2 + uy ** 2)
    assert r.max() <= 0.1
    # uniform in the disk: P(r < 0.05) = 1/4
    assert abs((r < 0.05).mean() - 0.25) < 0.015
    assert abs(n.mean()) < 0.01 and abs(n.var() - 1) < 0.01
    assert abs(np.mean(n[:, 0] * n[:, 1])) < 0.02


def test_pairs_are_bgk_collisions(consts):
    tau = 0.8
    pre, post = S.make_pairs(256, seed=1, tau=tau)
    xi = consts["xi"]
    for phi in (np.ones(37), xi[:, 0], xi[:, 1], (xi ** 2).sum(1)):
        assert np.max(np.abs(pre @ phi - post @ phi)) < 1e-14
    w = consts["w"]
    rho, ux, uy, T = S.macro(pre)
    feq = lbm.init(rho[:, None], ux[:, None], uy[:, None], T[:, None])[:, :, 0].T - w
    assert np.max(np.abs((pre + tau * (post - pre)) - feq) / w) < 1e-13
    # the perturbation is 1e-3 w N(0,1) around the drawn equilibrium
    assert 3e-4 < np.std((pre - feq) / w) < 3e-3


def test_gram_is_diagonal():
    G = S.gram()
    assert np.allclose(G, np.diag([1.0, 1.0, 1.0, 4.0]), rtol=0, atol=1e-14)


def test_projection_properties(consts):
    rng = np.random.default_rng(0)
    g = rng.standard_normal((50, 37)) * consts["w"]
    P = S.conserved_part(g)
    assert np.allclose(S.conserved_part(P), P, atol=1e-16)
    for phi in S._basis():
        assert np.allclose(P @ phi, g @ phi, atol=1e-15)


def test_surrogate_equilibrium_conserves_for_any_network(consts):
    theta = S.init_params(11)
    norm = np.stack([np.zeros(37), np.ones(37), np.zeros(37), np.full(37, 0.3)])
    pre, _ = S.make_pairs(64, seed=2, tau=0.8)
    ghat = S.surrogate_equilibrium(pre, theta, norm)
    for phi in S._basis():
        assert np.max(np.abs(ghat @ phi - pre @ phi)) < 1e-14


def test_residual_of_exact_equilibrium_is_zero(consts):
    rho, ux, uy, T, _ = pair_draws(np.arange(200), seed=4)
    w = consts["w"]
    g = lbm.init(rho[:, None], ux[:, None], uy[:, None], T[:, None])[:, :, 0].T - w
    r = S.residual(g, rho, ux, uy, T)
    assert r.max() < 1e-14
    # and it sees a perturbed stress
    g2 = g + 1e-3 * w * (consts["xi"][:, 0] * consts["xi"][:, 1])
    assert np.all(S.residual(g2, rho, ux, uy, T) > 5e-4)


def test_gelu_forms_and_derivative():
    a = np.linspace(-6, 6, 1001)
    assert np.allclose(S.gelu(a), 0.5 * a * (1 + np.tanh(S.GELU_C * (a + S.GELU_A * a ** 3))), atol=1e-15)
    h = 1e-6
    fd = (S.gelu(a + h) - S.gelu(a - h)) / (2 * h)
    assert np.max(np.abs(fd - S.gelu_grad(a))) < 1e-8


def test_bf16_rounding_examples():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7, -2.5, 3.0e-3, 65504.0])
    got = S.bf16(x)
    want = np.array([1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -7, -2.5, 0.0030059814453125, 65536.0])
    assert np.array_equal(got, want)


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    theta = S.init_params(7) + 0.01 * rng.standard_normal(S.NPARAM)
    x = rng.standard_normal((6, 37))
    y = rng.standard_normal((6, 37))
    _, g = S.loss_and_grad(theta, x, y, emulate=False)
    idx = rng.choice(S.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [0, 4736, 4736 + 127, S.NPARAM - 1, S.NPARAM - 38]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (S.loss_and_grad(tp, x, y, False)[0] - S.loss_and_grad(tm, x, y, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_and_convergence():
    theta = np.array([0.0, 10.0])
    m = v = np.zeros(2)
    g = 2 * (theta - 3.0)
    t1, m, v = S.adam_step(theta, m, v, g, 1, 0.1)
    assert np.allclose(t1 - theta, [0.1, -0.1], atol=1e-7)
    th = t1
    for t in range(2, 3000):
        th, m, v = S.adam_step(th, m, v, 2 * (th - 3.0), t, 0.05)
    assert np.allclose(th, 3.0, atol=1e-3)


def test_epoch_order_is_a_permutation():
    for n in (1, 7, 64, 1000, 4096):
        a, c = S.epoch_order(n, 123, 2)
        assert math.gcd(a, n) == 1
        idx = (a * np.arange(n) + c) % n
        assert len(set(idx.tolist())) == n


def test_short_training_reduces_loss():
    tau = 0.8
    pre, post = S.make_pairs(4096, seed=9, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta, losses = S.train(pre, post, tau, S.init_params(1), norm, batch=256, epochs=6, lr0=3e-3, seed=2)
    assert losses[-1] < 0.1 * losses[0]


def test_bf16_ulp():
    v = np.array([1.0, 1.5, -2.0, 3.0e-3, 0.0, 2.0 ** -130])
    u = S.bf16_ulp(v)
    assert np.array_equal(u[:5], [2.0 ** -7, 2.0 ** -7, 2.0 ** -6, 2.0 ** -16, 0.0])
    # neighbouring BF16 values differ by exactly one ulp
    for a in (1.0, 1.7, 0.0123, 77.0):
        b = S.bf16(a)
        nxt = np.array([b], dtype=np.float32).view(np.uint32) + np.uint32(1 << 16)
        assert nxt.view(np.float32)[0] - b == S.bf16_ulp(b)


def test_gelu_grad_max():
    G = S.gelu_grad_max()
    assert 1.12 < G < 1.14
    a = np.random.default_rng(0).uniform(-20, 20, 100000)
    assert np.abs(S.gelu_grad(a)).max() <= G


@pytest.mark.parametrize("trained", [False, True])
def test_flip_bound_covers_single_flips_anywhere(consts, trained):
    """Plant one BF16 flip (one unit in the last place, either direction) in
    one network input, one first-layer or one second-layer activation of
    the emulating forward pass, then round everything downstream again: at
    sampled sites and over every unit, g_hat moves by at most 4 B2 of the
    site, and at the median site the worst second-layer flip comes within a
    factor 3 of B2 (the bound is not loose)."""
    w = consts["w"]
    tau = 0.8
    pre, post = S.make_pairs(2048, seed=21, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta = S.init_params(4)
    if trained:
        theta, _ = S.train(pre, post, tau, theta, norm, batch=256, epochs=2, lr0=3e-3, seed=8)
    sites = pre[::97]
    B2s = S.flip_bound(theta, norm, sites, infer=False)
    p = S.unpack(theta)
    W1, W2, W3 = (S.bf16(p[k]) for k in ("W1", "W2", "W3"))

    def ghat(g, x=None, h1=None, h2=None):
        if h1 is None:
            h1 = S.bf16(S.gelu(x @ W1.T + p["b1"]))
        if h2 is None:
            h2 = S.bf16(S.gelu(h1 @ W2.T + p["b2"]))
        d = w * (norm[2] + norm[3] * (h2 @ W3.T + p["b3"]))
        return S.conserved_part(g) + d - S.conserved_part(d), h1, h2

    rng = np.random.default_rng(0)
    ratio = {"x": 0.0, "h1": 0.0, "h2": 0.0}
    h2_ratio = []
    for g, B2 in zip(sites, B2s):
        worst = {"x": 0.0, "h1": 0.0, "h2": 0.0}
        g = g[None, :]
        x = S.bf16((g / w - norm[0]) / norm[1])
        base, h1, h2 = ghat(g, x=x)
        for kind, n in (("x", 37), ("h1", 128), ("h2", 128)):
            for k in range(n):
                v = {"x": x, "h1": h1, "h2": h2}[kind].copy()
                v[0, k] += rng.choice([-1.0, 1.0]) * S.bf16_ulp(v[0, k])
                args = {"x": dict(x=v), "h1": dict(h1=v), "h2": dict(h1=h1, h2=v)}[kind]
                moved, _, _ = ghat(g, **args)
                worst[kind] = max(worst[kind], float(np.max(np.abs(moved - base) / w)))
        for kind in ratio:
            ratio[kind] = max(ratio[kind], worst[kind] / B2)
        h2_ratio.append(worst["h2"] / B2)
    assert max(ratio.values()) <= 4.0, ratio
    assert np.median(h2_ratio) >= 1 / 3, h2_ratio


# ---- FP8 (e4m3) form of the hidden layer -------------------------------------------

def _e4m3_codes():
    """Every e4m3 code decoded by the format's definition (OCP FP8 "E4M3",
    the variant without infinities): sign bit, exponent field E (bias 7),
    mantissa field M (3 bits); E = 0 subnormal M 2^-9; E = 15, M = 7 is NaN.
    Returns {code: value} for the finite codes."""
    out = {}
    for code in range(256):
        sgn = -1.0 if code & 0x80 else 1.0
        E, M = (code >> 3) & 0xF, code & 0x7
        if E == 15 and M == 7:
            continue
        out[code] = sgn * (M * 2.0 ** -9 if E == 0 else (1 + M / 8) * 2.0 ** (E - 7))
    return out


def test_e4m3_rounding_against_the_format_definition():
    """Finite codes are fixed points; any value goes to the nearest finite
    code (a tie to the code with an even mantissa field); values beyond the
    midpoint of 448 and the next (would-be) step 480 are NaN."""
    codes = _e4m3_codes()
    assert max(codes.values()) == 448.0 and min(v for v in codes.values() if v > 0) == 2.0 ** -9
    vals = np.array(list(codes.values()))
    assert np.array_equal(S.e4m3(vals), vals)
    pos = sorted(set(abs(v) for v in codes.values()))
    even = {abs(v): (c & 1) == 0 for c, v in codes.items()}
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-470, 470, 4000), rng.normal(0, 1, 4000), rng.normal(0, 0.01, 2000),
                        [(a + b) / 2 for a, b in zip(pos, pos[1:])], [463.99, 464.0, 464.01, 479.0, 1e6]])
    got = S.e4m3(x)
    for xi, gi in zip(x, got):
        a = abs(xi)
        if a > 464.0:
            assert np.isnan(gi), xi
            continue
        d = [abs(a - v) for v in pos]
        best = min(d)
        near = [v for v, dv in zip(pos, d) if dv == best]
        want = near[0] if len(near) == 1 else [v for v in near if even[v]][0]
        assert abs(gi) == want and (gi == 0 or np.sign(gi) == np.sign(xi)), (xi, gi, want)


def test_e4m3_worked_values():
    """Values worked out by hand from the format: 0.3 -> 1.25 x 2^-2; 449 and
    464 -> 448 (464 is a tie, 448's mantissa field 6 is even); 470 -> NaN;
    1.5 x 2^-9 and 2.5 x 2^-9 -> 2^-8 (ties to the even subnormal 2); 1e-5
    -> 0."""
    x = np.array([0.3, 449.0, 464.0, 470.0, 1.5 * 2 ** -9, 2.5 * 2 ** -9, 1e-5, -1.75, 240.0])
    want = np.array([0.3125, 448.0, 448.0, np.nan, 2 ** -8, 2 ** -8, 0.0, -1.75, 240.0])
    assert np.array_equal(S.e4m3(x), want, equal_nan=True)


def test_fp8_weight_exponent_puts_the_largest_weight_in_128_256():
    rng = np.random.default_rng(1)
    for scale in (1e-3, 0.09, 0.2, 0.5, 3.0):
        W = scale * rng.standard_normal((128, 128))
        m = np.abs(W).max() * 2.0 ** S.fp8_weight_exponent(W)
        assert 128.0 <= m < 256.0


def test_fp8_forward_rounds_only_the_hidden_layer():
    """The FP8 form keeps the first layer and its inputs (BF16), puts the
    hidden layer's inputs on the e4m3 grid (scaled by 16) and differs from
    the BF16 form by about the e4m3 rounding (3 mantissa bits)."""
    tau = 0.8
    pre, post = S.make_pairs(512, seed=3, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta = S.init_params(2)
    zs = (pre / S.constants()["w"] - norm[0]) / norm[1]
    o8, (x8, a18, h18, _, _) = S.forward(theta, zs, emulate=True, fp8=True)
    o16, (x16, a116, h116, _, _) = S.forward(theta, zs, emulate=True)
    assert np.array_equal(x8, x16) and np.array_equal(a18, a116)
    assert np.array_equal(S.e4m3(h18 * S.FP8_ACT_SCALE) / S.FP8_ACT_SCALE, h18)
    rel = np.abs(o8 - o16).max() / np.abs(o16).max()
    assert 1e-4 < rel < 0.2, rel


def test_fp8_flip_bound_covers_planted_flips(consts):
    """One e4m3 flip (one step of the grid, either direction) of one
    hidden-layer input, everything downstream rounded again: g_hat moves by
    at most B1 + 8 B2 of the site (B2: the BF16 re-roundings it triggers)."""
    w = consts["w"]
    tau = 0.8
    pre, post = S.make_pairs(1024, seed=22, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta = S.init_params(6)
    sites = pre[::67]
    B1 = S.fp8_flip_bound(theta, norm, sites)
    B2 = S.flip_bound(theta, norm, sites, fp8=True)
    p = S.unpack(theta)
    sw = 2.0 ** S.fp8_weight_exponent(p["W2"])
    W2q = S.e4m3(p["W2"] * sw) / sw
    W3 = S.bf16(p["W3"])
    zs = (sites / w - norm[0]) / norm[1]
    _, (_, _, h1, _, _) = S.forward(theta, zs, emulate=True, fp8=True)
    rng = np.random.default_rng(2)

    def ghat(g, h1row):
        h2 = S.bf16(S.gelu(h1row @ W2q.T + p["b2"]))
        d = w * (norm[2] + norm[3] * (h2 @ W3.T + p["b3"]))
        return S.conserved_part(g) + d - S.conserved_part(d)

    worst = 0.0
    for i, g in enumerate(sites):
        base = ghat(g[None, :], h1[i:i + 1])
        for j in range(128):
            v = h1[i:i + 1].copy()
            v[0, j] += rng.choice([-1.0, 1.0]) * S.e4m3_ulp(v[0, j] * S.FP8_ACT_SCALE) / S.FP8_ACT_SCALE
            moved = ghat(g[None, :], v)
            worst = max(worst, float(np.max(np.abs(moved - base) / w) / (B1[i] + 8 * B2[i])))
    assert worst <= 1.0, worst


# ---- the inference form's binary16 hidden layer ---------------------------------------

def test_f16_rounding_examples():
    """Binary16 rounding: 11 significant bits, ties to even, subnormals down
    to 2^-24 (ties to even there too), overflow at 65520 and beyond."""
    cases = [(1.0 + 2.0 ** -11, 1.0), (1.0 + 3 * 2.0 ** -11, 1.0 + 2.0 ** -9), (1.0 + 2.0 ** -11 + 2.0 ** -30, 1.0 + 2.0 ** -10),
             (65504.0, 65504.0), (65519.99, 65504.0), (2.0 ** -25, 0.0), (1.5 * 2.0 ** -24, 2.0 ** -23),
             (-2.302734375, -2.302734375), (0.1, 0.0999755859375)]
    for v, want in cases:
        assert S.f16(v) == want, (v, S.f16(v), want)
    assert np.isinf(S.f16(65520.0)) and np.isinf(S.f16(-1e6))


def test_gelu_f16_constants_and_special_values():
    """K1 = -2 log2(e) c A and K2 = -2 log2(e) c (c = sqrt(2/pi), A = 0.044715)
    on the binary16 grid; gelu(0) = 0, large positive inputs come back
    unchanged, large negative ones give -0, and 1 and -1 are worked by hand."""
    l2e = 1.0 / math.log(2.0)
    assert S.GELU_K1_F16 == -0.10296630859375 == S.f16(-2 * l2e * math.sqrt(2 / math.pi) * 0.044715)
    assert S.GELU_K2_F16 == -2.302734375 == S.f16(-2 * l2e * math.sqrt(2 / math.pi))
    v = S.gelu_f16(np.array([0.0, 300.0, 60000.0, -300.0, 20.0]))
    assert v[0] == 0.0 and v[1] == 300.0 and v[2] == 60000.0 and v[3] == 0.0 and np.signbit(v[3]) and v[4] == 20.0
    # a = 1: s = 1, t = h(K1 + K2) = -2.40625, y = -2.40625, e = h(2^-2.40625)
    e = S.f16(2.0 ** -2.40625)
    assert S.f16(S.GELU_K1_F16 + S.GELU_K2_F16) == -2.40625
    r = S.f16(1.0 / S.f16(e + 1.0))
    assert S.gelu_f16(np.array([1.0]))[0] == r
    assert abs(r - S.gelu(1.0)) < 2 ** -10
    # a = -1: y = h(-1 * h(K1 + K2)) = 2.40625, result -h(1 / h(2^2.40625 + 1))
    assert S.gelu_f16(np.array([-1.0]))[0] == -S.f16(1.0 / S.f16(S.f16(2.0 ** 2.40625) + 1.0))


def test_gelu_f16_follows_gelu_on_every_binary16_input():
    """Over every binary16 value in [-12, 12] the binary16 evaluation stays
    within 1 % + 2^-13 of the tanh form in FP64 (seven roundings, and the
    exponential's amplification of the rounded exponent); a halved K1 or
    K2, a dropped cubic or the natural exponential instead of 2^y each
    break that by more than 0.01."""
    x = np.arange(65536, dtype=np.uint16).view(np.float16).astype(np.float64)
    x = x[np.isfinite(x) & (np.abs(x) <= 12)]
    exact = S.gelu(x)
    assert np.max(np.abs(S.gelu_f16(x) - exact) - 0.01 * np.abs(exact)) <= 2.0 ** -13
    # the mutants, evaluated with the same roundings
    xx = S.f16(x)
    for k1f, k2f, base in ((0.5, 1.0, 2.0), (1.0, 0.5, 2.0), (0.0, 1.0, 2.0), (1.0, 1.0, math.e)):
        t = S.f16(S.GELU_K1_F16 * k1f * S.f16(xx * xx) + S.GELU_K2_F16 * k2f)
        m = S.f16(xx * S.f16(1.0 / S.f16(S.f16(base ** S.f16(xx * t)) + 1.0)))
        assert np.max(np.abs(m - exact) - 0.01 * np.abs(exact)) > 0.01


def test_f16_forward_rounds_only_the_hidden_layer():
    """The inference form keeps the first layer and its BF16 inputs, puts
    both hidden layers' activations on the binary16 grid, and differs from
    the BF16 training form by about the BF16 rounding it no longer does."""
    tau = 0.8
    pre, post = S.make_pairs(512, seed=3, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta = S.init_params(2)
    zs = (pre / S.constants()["w"] - norm[0]) / norm[1]
    oh, (xh, a1h, h1h, _, h2h) = S.forward(theta, zs, emulate=True, infer=True)
    ob, (xb, a1b, _, _, _) = S.forward(theta, zs, emulate=True)
    assert np.array_equal(xh, xb) and np.array_equal(a1h, a1b)
    assert np.array_equal(S.f16(h1h), h1h) and np.array_equal(S.f16(h2h), h2h)
    rel = np.abs(oh - ob).max() / np.abs(ob).max()
    assert 1e-5 < rel < 0.05, rel
    # and the FP8 form is untouched by infer
    o8a, _ = S.forward(theta, zs, emulate=True, fp8=True)
    o8b, _ = S.forward(theta, zs, emulate=True, fp8=True, infer=True)
    assert np.array_equal(o8a, o8b)


def test_flip_bound_covers_planted_flips_in_the_f16_form(consts):
    """In the binary16 inference form: one BF16 flip of one input, or one
    binary16 flip (one unit in the last place, either direction) of one
    first- or second-layer activation, everything downstream rounded again
    as the form does: g_hat moves by at most 4 B2 of the site."""
    w = consts["w"]
    tau = 0.8
    pre, post = S.make_pairs(2048, seed=21, tau=tau)
    norm = S.fit_normalization(pre, post, tau)
    theta, _ = S.train(pre, post, tau, S.init_params(4), norm, batch=256, epochs=2, lr0=3e-3, seed=8)
    sites = pre[::131]
    B2s = S.flip_bound(theta, norm, sites)
    p = S.unpack(theta)
    W1, W2, W3 = S.bf16(p["W1"]), S.f16(p["W2"]), S.f16(p["W3"])

    def f16_ulp(v):
        a = abs(v)
        return 2.0 ** (max(math.floor(math.log2(a)), -14) - 10) if a > 0 else 2.0 ** -24

    def ghat(g, x=None, h1=None, h2=None):
        if h1 is None:
            h1 = S.gelu_f16(S.f32(x @ W1.T + p["b1"]))
        if h2 is None:
            h2 = S.gelu_f16(S.f32(h1 @ W2.T + p["b2"]))
        d = w * (norm[2] + norm[3] * (h2 @ W3.T + p["b3"]))
        return S.conserved_part(g) + d - S.conserved_part(d), h1, h2

    rng = np.random.default_rng(5)
    worst = 0.0
    for g, B2 in zip(sites, B2s):
        g = g[None, :]
        x = S.bf16((g / w - norm[0]) / norm[1])
        base, h1, h2 = ghat(g, x=x)
        for kind, n in (("x", 37), ("h1", 128), ("h2", 128)):
            for k in range(n):
                v = {"x": x, "h1": h1, "h2": h2}[kind].copy()
                step = S.bf16_ulp(v[0, k]) if kind == "x" else f16_ulp(v[0, k])
                v[0, k] += rng.choice([-1.0, 1.0]) * step
                args = {"x": dict(x=v), "h1": dict(h1=v), "h2": dict(h1=h1, h2=v)}[kind]
                moved, _, _ = ghat(g, **args)
                worst = max(worst, float(np.max(np.abs(moved - base) / w) / B2))
    assert worst <= 4.0, worst
