"""GPU parity of the learned collide against its oracle (oracle/surrogate.py).

Every network used here is created by the oracle (its own Philox init, its
own training) and handed to the GPU; GPU-trained networks are judged only by
the plain collide (fallback statistics, error against the FP64 run).

Tolerances:
* pairs: FP32 evaluation of the equilibrium and of the Box-Muller draws,
  |pre_gpu - pre_oracle| / w_p <= 4e-6;
* network parameters after init: bit-exact;
* gradient: per parameter block relative L2 <= 2e-3 and cosine >= 0.9999;
  the kernels and the BF16-emulating oracle round at the same points, so the
  residue is FP32 versus FP64 accumulation plus rare BF16 ties that round the
  other way;
* learned equilibrium g_hat (the binary16 inference form, emulated by the
  oracle operation by operation), per site, in units of w_p (a step relaxes
  by 1/tau, so the step bars are these divided by tau):
  - every site: <= 8 B2, B2 = surrogate.flip_bound of that site, the move
    of g_hat that one BF16 rounding flip of a second-layer activation
    causes there. Both sides round the same values at the same points
    (inputs to BF16, pre-activations to binary16, then the GELU's binary16
    arithmetic, which the device reproduces bit for bit: test_gelu16_*),
    and differ before rounding only by FP32 accumulation and the folded
    standardisation, so they disagree only where a value sits that close
    to a rounding boundary, and then by one unit (BF16 for an input,
    binary16, 2^-3 of that, for an activation); one flip anywhere in the
    network, with the roundings it changes downstream, moves g_hat by at
    most 4 B2 (pinned on the oracle by planting flips), and 8 B2 allows two
    at one site;
  - the median site: <= 1e-6 (FLOOR): at a site without a flip only the
    FP32 arithmetic differs (measured about 2e-8), so an error common to
    all sites (a permuted weight column, a dropped bias, a wrong
    standardisation constant) fails here even where it stays under 5 B2;
  - conserved moments of g_hat equal those of the input to FP32 rounding.
"""
import numpy as np
import pytest

from oracle import lbm, surrogate as S
from oracle.lattice import constants
from paper_1804_01918_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1804_01918_amd import lb  # noqa: E402

TAU = 0.8
FLOOR = 1e-6  # per-site agreement without a rounding flip (FP32 arithmetic only)


def _bar(theta, nf, g):
    """Largest |g_hat_gpu - g_hat_oracle| / w_p allowed at each of the sites
    g: two flips of 4 B2 each (see the module docstring)."""
    return 8.0 * S.flip_bound(theta, nf, g)


def _check_sites(err, bar, floor=FLOOR, what=""):
    """err: per-site max over populations; bar: per-site bars (or one).
    Every site within its bar, the median site within floor. Prints the
    distribution."""
    err = np.asarray(err, dtype=np.float64)
    bar = np.broadcast_to(np.asarray(bar, dtype=np.float64), err.shape)
    frac = float(np.mean(err > floor))
    worst = int(np.argmax(err / bar))
    print(f"{what} sites={err.size} max={err.max():.3e} worst/bar={err[worst] / bar[worst]:.3f} "
          f"bar range=[{bar.min():.2e}, {bar.max():.2e}] median={np.median(err):.3e} floor={floor:.1e} "
          f"above_floor={frac:.4f}")
    assert np.all(err <= bar), (err[worst], bar[worst])
    assert np.median(err) <= floor, (np.median(err), floor)
    return frac


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32).astype(np.float64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def oracle_net():
    """A network trained by the oracle on its own pairs (FP32-rounded)."""
    pre, post = S.make_pairs(4096, seed=21, tau=TAU)
    pre, post = _f32(pre), _f32(post)
    norm = S.fit_normalization(pre, post, TAU)
    theta, losses = S.train(pre, post, TAU, S.init_params(4), norm, batch=256, epochs=6, lr0=3e-3, seed=8)
    return _f32(theta), _f32(norm), losses


def _gpu_net(theta, norm, max_batch=8192):
    m = lb.Mlp(max_batch)
    m.set_params(theta)
    m.set_normalization(norm)
    return m


def test_pairgen_matches_oracle(consts):
    pre, post = lb.pairgen(4096, 7, TAU)
    opre, opost = S.make_pairs(4096, 7, TAU)
    w = consts["w"]
    assert np.max(np.abs(pre.cpu().numpy() - opre) / w) <= 4e-6
    assert np.max(np.abs(post.cpu().numpy() - opost) / w) <= 4e-6


def test_pairgen_offsets_are_counter_based(consts):
    a, _ = lb.pairgen(300, 5, TAU)
    b, _ = S.make_pairs(100, 5, TAU, start=200)
    assert np.max(np.abs(a[200:].cpu().numpy() - b) / consts["w"]) <= 4e-6


def test_init_bitwise():
    m = lb.Mlp(256)
    m.init(1)
    assert np.array_equal(m.get_params(), S.init_params(1).astype(np.float32))
    m.init(2 ** 40 + 3)
    assert np.array_equal(m.get_params(), S.init_params(2 ** 40 + 3).astype(np.float32))


def test_params_and_normalization_roundtrip(oracle_net):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    assert np.array_equal(m.get_params(), theta.astype(np.float32))
    assert np.allclose(m.get_normalization(), norm, rtol=1e-6, atol=0)


def test_fit_normalization_matches_oracle():
    pre, post = S.make_pairs(2048, seed=3, tau=TAU)
    pre, post = _f32(pre), _f32(post)
    m = lb.Mlp(256)
    m.fit_normalization(_dev(pre), _dev(post), TAU)
    got = m.get_normalization()
    want = S.fit_normalization(pre, post, TAU)
    scale = np.stack([want[1], want[1], want[3], want[3]])
    assert np.max(np.abs(got - want) / scale) < 1e-4


@pytest.mark.parametrize("n", [32, 256])
def test_gradient_matches_oracle(n):
    rng = np.random.default_rng(n)
    pre, post = S.make_pairs(n, seed=3, tau=TAU)
    pre, post = _f32(pre), _f32(post)
    norm = _f32(S.fit_normalization(pre, post, TAU))
    theta = _f32(S.init_params(1) + 0.02 * rng.standard_normal(S.NPARAM))
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    g_gpu, loss_gpu = m.gradient(_dev(pre), _dev(post), TAU)
    z, y = S.features(pre, post, TAU)
    loss, g = S.loss_and_grad(theta, (z - nf[0]) / nf[1], (y - nf[2]) / nf[3], emulate=True)
    assert abs(loss_gpu / loss - 1) < 1e-5
    k = 0
    for name, shape in S.SHAPES:
        cnt = int(np.prod(shape))
        a, b = g_gpu[k:k + cnt].astype(np.float64), g[k:k + cnt]
        k += cnt
        assert np.linalg.norm(a - b) <= 2e-3 * np.linalg.norm(b), name
        assert a @ b >= 0.9999 * np.linalg.norm(a) * np.linalg.norm(b), name


def test_training_steps_match_oracle(oracle_net):
    """Two Adam steps (batch 128 of 256 pairs, the epoch order of the seed):
    the loss of the steps and the parameters agree with the oracle's."""
    pre, post = S.make_pairs(256, seed=12, tau=TAU)
    pre, post = _f32(pre), _f32(post)
    norm = _f32(S.fit_normalization(pre, post, TAU))
    theta0 = _f32(S.init_params(9))
    m = _gpu_net(theta0, norm, max_batch=256)
    nf = m.get_normalization().astype(np.float64)
    lr = 1e-3
    losses = m.train(_dev(pre), _dev(post), TAU, batch=128, epochs=1, lr=lr, seed=77)
    theta_gpu = m.get_params().astype(np.float64)
    theta_orc, ol = S.train(pre, post, TAU, theta0, nf, batch=128, epochs=1, lr0=lr, seed=77)
    assert abs(losses[0] / np.mean(ol) - 1) < 1e-4
    # Adam moves each parameter by about lr per step; gradients that differ in
    # sign between the two sides (entries near zero) move it the other way.
    d = np.abs(theta_gpu - theta_orc)
    assert np.quantile(d, 0.99) <= 0.05 * lr
    assert d.max() <= 4 * lr


def test_training_is_reproducible():
    """Pair generation, standardisation and training use no floating-point
    atomics: two runs from the same seeds give bit-identical parameters,
    standardisation and loss history."""
    out = []
    for _ in range(2):
        pre, post = lb.pairgen(1 << 16, 5, TAU)
        m = lb.Mlp(2048)
        m.fit_normalization(pre, post, TAU)
        m.init(2)
        losses = m.train(pre, post, TAU, 2048, 3, 2e-3, 9)
        out.append((m.get_params(), m.get_normalization(), losses))
        m.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


def test_learned_equilibrium_matches_oracle(consts, oracle_net):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    pre, _ = S.make_pairs(2048, seed=31, tau=TAU)
    pre = _f32(pre)
    gh, res, fb = m.equilibrium(_dev(pre), 1e9)
    gh = gh.cpu().numpy()
    want = S.surrogate_equilibrium(pre, theta, nf, emulate=True)
    w = consts["w"]
    rho, ux, uy, T = S.macro(pre)
    # perturbed pairs slightly outside the training box take the plain
    # equilibrium (compare those where the box test is not a rounding tie)
    box = S.in_box(rho, ux, uy, T)
    assert np.array_equal(fb.cpu().numpy().astype(bool), ~box)
    exact = lbm.init(rho[:, None], ux[:, None], uy[:, None], T[:, None])[:, :, 0].T - w
    want = np.where(box[:, None], want, exact)
    _check_sites(np.max(np.abs(gh - want) / w, axis=1), _bar(theta, nf, pre), what="equilibrium")
    # projection: conserved moments of g_hat are those of the input
    for phi in S._basis():
        scale = np.abs(pre * phi).sum(1) + 1e-3
        assert np.max(np.abs(gh @ phi - pre @ phi) / scale) < 1e-5
    # residual and verdict agree with the oracle away from the threshold
    r_orc = S.residual(S.surrogate_equilibrium(pre, theta, nf, emulate=True), rho, ux, uy, T)
    assert np.max(np.abs(res.cpu().numpy() - r_orc)) < 1e-5 + 1e-2 * r_orc.max()
    thr = float(np.median(r_orc))
    _, _, fb2 = m.equilibrium(_dev(pre), thr)
    fb2 = fb2.cpu().numpy().astype(bool)
    away = np.abs(r_orc - thr) > 0.05 * thr
    assert np.array_equal(fb2[away], ((r_orc > thr) | ~box)[away])


def test_out_of_box_sites_fall_back(oracle_net):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    w = constants()["w"]
    hot = lbm.init(np.full((8, 1), 1.0), np.zeros((8, 1)), np.zeros((8, 1)), np.full((8, 1), 1.3))[:, :, 0].T - w
    gh, _, fb = m.equilibrium(_dev(hot), 1e9)
    assert fb.cpu().numpy().all()
    # the fallback is the plain equilibrium
    assert np.max(np.abs(gh.cpu().numpy() - hot) / w) < 1e-5


@pytest.mark.parametrize("kind", ["shear_wave", "rayleigh_taylor"])
def test_learned_step_matches_oracle(consts, oracle_net, kind):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    lx, ly = 64, 128
    fields = inputs.make_state(kind, lx, ly, seed=2)
    sites = [(0, 0), (lx - 1, ly - 1), (5, 64), (33, 7), (17, 100), (60, 3)]
    with lb.Lattice(lx, ly, TAU, fields, precision="f32s", layout="caosoa") as lat:
        lat.set_surrogate(m, 1e9)
        lat.step(1)
        f = lat.get_populations().cpu().numpy()
        nfb, ntot = lat.surrogate_counts()
    assert ntot == lx * ly
    got = np.stack([f[:, x, y] for x, y in sites])
    w = consts["w"]

    def collide(win):
        g = _f32(win.reshape(37, -1).T - w)
        out, _, _ = S.surrogate_collide(g, TAU, theta, nf, 1e9)
        return (out + w).T.reshape(win.shape)

    ref = np.stack([_window_step(fields, s, collide) for s in sites])
    pulled = np.stack([_window_step(fields, s, lambda win: win) for s in sites]) - w
    _check_sites(np.max(np.abs(got - ref) / w, axis=1), _bar(theta, nf, pulled) / TAU, FLOOR / TAU,
                 what=f"step {kind}")


def _learned_sampled_parity(consts, oracle_net, lx, ly, layout, kind, sites, seed=2):
    """One learned step on the GPU (no fallback) against the oracle's learned
    collide on each sampled site's dependency window."""
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    fields = inputs.make_state(kind, lx, ly, seed=seed)
    with lb.Lattice(lx, ly, TAU, [torch.from_numpy(a).cuda() for a in fields], precision="f32s",
                    layout=layout) as lat:
        lat.set_surrogate(m, 1e9)
        lat.step(1)
        f = lat.get_populations()
        got = torch.stack([f[:, x, y] for x, y in sites]).cpu().numpy()
        nfb, ntot = lat.surrogate_counts()
    assert (nfb, ntot) == (0, lx * ly)
    w = consts["w"]

    def collide(win):
        g = _f32(win.reshape(37, -1).T - w)
        out, _, _ = S.surrogate_collide(g, TAU, theta, nf, 1e9)
        return (out + w).T.reshape(win.shape)

    ref = np.stack([_window_step(fields, s, collide) for s in sites])
    pulled = np.stack([_window_step(fields, s, lambda win: win) for s in sites]) - w
    return np.max(np.abs(got - ref) / w, axis=1), _bar(theta, nf, pulled) / TAU


@pytest.mark.parametrize("L,kind", [(2048, "shear_wave"), (8192, "rayleigh_taylor")])
def test_learned_step_full_size_sampled(consts, oracle_net, L, kind):
    """2048 x 2048 and 8192 x 8192, CAoSoA, the persistent launch the
    benchmark times: corners, edges (periodic wrap), tile seams and random
    sites."""
    lx = ly = L
    rng = np.random.default_rng(5)
    sites = [(0, 0), (lx - 1, ly - 1), (0, ly - 1), (lx - 1, 0), (L // 2, 511), (L // 2, 512), (7, L - 513),
             (L - 48, L // 2)] + [(int(x), int(y)) for x, y in rng.integers(0, L, size=(8, 2))]
    err, bar = _learned_sampled_parity(consts, oracle_net, lx, ly, "caosoa", kind, sites)
    _check_sites(err, bar, FLOOR / TAU, what=f"full size {L}")


@pytest.mark.parametrize("lx,ly,layout", [(1, 1, "soa"), (1, 5, "aos"), (3, 96, "aos"), (3, 96, "csoa"),
                                          (9, 608, "caosoa"), (9, 608, "soa")])
def test_learned_step_ragged_tiles(consts, oracle_net, lx, ly, layout):
    """The 1 x 1 lattice (every population its own neighbour), grids below
    one workgroup per XCD (1 or 3 rows) and rows of 608 sites (a full
    512-site tile and a ragged one), in every layout."""
    sites = [(0, 0), (lx - 1, ly - 1), (lx // 2, ly // 2), (1, ly - 3), (lx - 1, 2)]
    if ly > 512:
        sites += [(2, 511), (2, 512), (lx - 2, 600)]
    sites = sorted({(x % lx, y % ly) for x, y in sites})
    err, bar = _learned_sampled_parity(consts, oracle_net, lx, ly, layout, "rayleigh_taylor", sites)
    _check_sites(err, bar, FLOOR / TAU, what=f"ragged {lx}x{ly} {layout}")


@pytest.mark.parametrize("layout,ly", [("caosoa", 29020032), ("aos", 29020049)])
def test_learned_step_longest_accepted_row(consts, oracle_net, layout, ly):
    """Rows of the longest length the host accepts for FP32 storage in the
    interleaved layouts (ly * 37 * 4 bytes just under 4 GiB, the limit of the
    kernel's 32-bit in-row offsets; a whole number of 32-site clusters in
    CAoSoA): two rows, sampled at both row ends and at the cluster-lane
    seams, where the offsets are largest. Random equilibrium, so every
    neighbour differs."""
    assert lb.buffer_bytes(2, ly, "f32s", layout) > 0
    assert lb.buffer_bytes(2, ly + (32 if layout == "caosoa" else 1), "f32s", layout) == 0
    ys = {0, 1, 2, ly // 2, ly - 3, ly - 2, ly - 1}
    if layout == "caosoa":
        ys |= {k * (ly // 32) + d for k in (1, 16, 31) for d in (-1, 0)}
    sites = sorted((x, y) for x in range(2) for y in ys)
    err, bar = _learned_sampled_parity(consts, oracle_net, 2, ly, layout, "random_equilibrium", sites)
    _check_sites(err, bar, FLOOR / TAU, what=f"longest row {layout}")


def _window_step(fields, site, collide):
    """One step at `site` on its 7 x 7 dependency window with a given collide."""
    rho, ux, uy, T = fields
    lx, ly = rho.shape
    x0, y0 = site
    xs, ys = (x0 + np.arange(-3, 4)) % lx, (y0 + np.arange(-3, 4)) % ly
    ix = np.ix_(xs, ys)
    win = lbm.init(rho[ix], ux[ix], uy[ix], T[ix])
    w = constants()["w"][:, None, None]
    win = w + _f32(win - w)   # the lattice stores FP32 deviations
    c = constants()["c"]
    new = np.empty((37, 1, 1))
    for p, (cx, cy) in enumerate(c):
        new[p, 0, 0] = win[p, 3 - cx, 3 - cy]
    return collide(new)[:, 0, 0]


def test_threshold_zero_is_the_plain_step(oracle_net):
    """With threshold 0 every site falls back to the plain FP32 collide: the
    learned step is then bit-identical to the plain step."""
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    fields = inputs.shear_wave(32, 64, seed=3)
    outs = []
    for learned in (True, False):
        with lb.Lattice(32, 64, TAU, fields, precision="f32s", layout="soa") as lat:
            if learned:
                lat.set_surrogate(m, 0.0)
            lat.step(5)
            outs.append(lat.get_populations().cpu().numpy())
            if learned:
                assert lat.surrogate_counts() == (5 * 32 * 64, 5 * 32 * 64)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("layout", ["soa", "caosoa"])
def test_learned_fused_equals_split(oracle_net, layout):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    fields = inputs.rayleigh_taylor(24, 64, seed=1)
    outs = []
    for fused in (True, False):
        with lb.Lattice(24, 64, TAU, fields, precision="f32s", layout=layout) as lat:
            lat.set_surrogate(m, 1e-3)
            if fused:
                lat.step(4)
            else:
                for _ in range(4):
                    lat.propagate()
                    lat.collide()
            outs.append(lat.get_populations().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_learned_conserves_mass_momentum_energy(consts, oracle_net):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    lx, ly, n = 64, 128, 100
    fields = inputs.shear_wave(lx, ly, seed=2)
    f0 = lbm.init(*fields)
    g = np.abs(f0 - consts["w"][:, None, None])
    xi = consts["xi"]
    scale = np.array([g.sum(), (g * np.abs(xi[:, 0])[:, None, None]).sum(),
                      (g * np.abs(xi[:, 1])[:, None, None]).sum(),
                      (g * 0.5 * (xi ** 2).sum(1)[:, None, None]).sum()])
    with lb.Lattice(lx, ly, TAU, fields, precision="f32s", layout="soa") as lat:
        lat.set_surrogate(m, 1e-3)
        a0 = lat.audit()
        lat.step(n)
        a1 = lat.audit()
    assert np.all(np.abs(a1 - a0) <= n * 2.0 ** -24 * scale * 8), (a1 - a0)


@pytest.mark.parametrize("where", ["rows", "scattered"])
def test_learned_fused_audit_matches_standalone(oracle_net, where):
    """The FP64 audit fused into the learned step (one partial per persistent
    workgroup) equals the standalone audit of the same state up to the
    summation order: a missing or repeated partial would be off by about a
    tile's worth of mass (~1), far above the bound. Fallback sites fill whole
    rows (full batches), or are scattered (about 10 %: mixed tiles, partial
    batches carried across tiles; a fallback lane's provisional store must
    not enter the audit, its batch's result must)."""
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    lx, ly = 64, 1024
    rho, ux, uy, T = inputs.rayleigh_taylor(lx, ly, seed=4)
    T = T.copy()
    # outside the training box: these sites take the plain collide
    if where == "rows":
        T[:2, :] = 1.25
    else:
        T[np.random.default_rng(9).random((lx, ly)) < 0.1] = 1.25
    fields = (rho, ux, uy, T)
    totals = []
    for audit in (True, False):
        with lb.Lattice(lx, ly, TAU, fields, precision="f32s", layout="caosoa", audit=audit) as lat:
            lat.set_surrogate(m, 1e9)
            lat.step(3)
            totals.append(lat.audit())
            nfb, ntot = lat.surrogate_counts()
            assert ntot == 3 * lx * ly and 0 < nfb < ntot  # both branches of the kernel ran
    assert np.allclose(totals[0], totals[1], rtol=1e-13, atol=1e-9), totals


def test_set_surrogate_rejects_other_precisions(oracle_net):
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    with lb.Lattice(8, 64, TAU, inputs.random_equilibrium(8, 64), precision="f64") as lat:
        with pytest.raises(lb.LBError) as e:
            lat.set_surrogate(m, 1e-3)
        assert e.value.code == lb.LB_EUNSUPPORTED


def test_trained_network_gain(consts):
    """What training buys: the same network before and after GPU training
    (Adam on GPU-drawn pairs), judged only by the exact equilibrium and the
    plain FP64 step.
    * Held-out pairs: the trained network's equilibrium error is at least
      ten times smaller; at residual threshold 1e-3 at most 5 % of the pairs
      fall back, where the untrained network sends at least 90 % to the
      plain collide.
    * A 1024 x 1024 shear wave, 1000 steps, threshold 1e-4: the trained
      network collides at least 99 % of the site updates itself and stays
      within 3e-4 of the FP64 run in every field; the untrained network
      passes the residual test at fewer than 10 % of them."""
    w = consts["w"]
    pre, post = lb.pairgen(1 << 20, 31, TAU)
    trained, untrained = lb.Mlp(8192), lb.Mlp(8192)
    for m in (trained, untrained):
        m.fit_normalization(pre, post, TAU)
        m.init(5)
    losses = trained.train(pre, post, TAU, 8192, 32, 3e-3, 17)
    assert losses[-1] < losses[0] / 100

    vpre, vpost = lb.pairgen(1 << 16, 77, TAU)
    geq = (vpre + TAU * (vpost - vpre)).double().cpu().numpy()
    wd = np.asarray(w)
    stats = {}
    for name, m in (("trained", trained), ("untrained", untrained)):
        ghat, res, _ = m.equilibrium(vpre, 1e30)
        err = np.abs(ghat.double().cpu().numpy() - geq) / wd
        _, _, fb = m.equilibrium(vpre, 1e-3)
        stats[name] = (float(np.median(err)), float(fb.float().mean()))
    print("held-out median error / fallback fraction:", stats)
    assert stats["trained"][0] * 10 <= stats["untrained"][0]
    assert stats["untrained"][1] >= 0.9
    assert stats["trained"][1] <= 0.05

    lx, ly, nsteps = 1024, 1024, 1000
    fields = [torch.from_numpy(a).cuda() for a in inputs.shear_wave(lx, ly, seed=3)]
    ref = lb.Lattice(lx, ly, TAU, fields, precision="f64")
    ref.step(nsteps)
    rm = ref.moments()
    ref.close()
    out = {}
    for name, m in (("trained", trained), ("untrained", untrained)):
        lat = lb.Lattice(lx, ly, TAU, fields, precision="f32s")
        lat.set_surrogate(m, 1e-4)
        lat.step(nsteps)
        mm = lat.moments()
        nfb, ntot = lat.surrogate_counts()
        lat.close()
        out[name] = (nfb / ntot, max(float((b - a).abs().max()) for a, b in zip(rm, mm)))
    print("lattice fallback fraction / max field error after", nsteps, "steps:", out)
    assert out["trained"][0] <= 0.01
    assert out["trained"][1] <= 3e-4
    assert out["untrained"][0] >= 0.9
    trained.close()
    untrained.close()


@pytest.fixture(scope="module")
def mixed_state(consts, oracle_net):
    """A 256 x 1536 Rayleigh-Taylor-like lattice in which a random tenth of
    the sites (scattered, not whole rows or tiles) start at T = 1.6, outside
    the training box (after the pull a site mixes populations from 37
    neighbours, so these sites and some of their neighbours fall back). 768 row tiles of 512 sites: three per persistent
    workgroup on 256 compute units, so a wavefront's fallback queue carries
    partial batches from tile to tile, and rows of three tiles.

    The oracle side: the FP32-shifted initial state, one pull propagate,
    then for every site both branches of the learned collide (network
    equilibrium; plain equilibrium) with the residual and the box verdict."""
    theta, norm, _ = oracle_net
    w = consts["w"]
    lx, ly = 256, 1536
    rho, ux, uy, T = inputs.rayleigh_taylor(lx, ly, seed=6)
    hot = np.random.default_rng(11).random((lx, ly)) < 0.1
    T = np.where(hot, 1.6, T)
    fields = (rho, ux, uy, T)
    f0 = lbm.init(*fields)
    f0 = w[:, None, None] + _f32(f0 - w[:, None, None])
    g = (lbm.propagate(f0) - w[:, None, None]).reshape(37, -1).T.copy()   # (sites, 37), x-major
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    m.close()
    n = g.shape[0]
    learned = np.empty_like(g)
    plain = np.empty_like(g)
    res = np.empty(n)
    box = np.empty(n, dtype=bool)
    edge = np.empty(n, dtype=bool)  # within FP32 reach of a training-box edge: either verdict
    bar = np.empty(n)
    for a in range(0, n, 32768):
        b = min(n, a + 32768)
        ga = g[a:b]
        rho_, ux_, uy_, T_ = S.macro(ga)
        gh = S.surrogate_equilibrium(ga, theta, nf, emulate=True)
        res[a:b] = S.residual(gh, rho_, ux_, uy_, T_)
        box[a:b] = S.in_box(rho_, ux_, uy_, T_)
        speed = np.sqrt(ux_ * ux_ + uy_ * uy_)
        edge[a:b] = ((np.minimum(np.abs(rho_ - 0.9), np.abs(rho_ - 1.1)) < 1e-5)
                     | (np.minimum(np.abs(T_ - 0.9), np.abs(T_ - 1.1)) < 1e-5) | (np.abs(speed - 0.1) < 1e-5))
        exact = lbm.init(rho_[:, None], ux_[:, None], uy_[:, None], T_[:, None])[:, :, 0].T - w
        learned[a:b] = ga + (gh - ga) / TAU
        plain[a:b] = ga + (exact - ga) / TAU
        bar[a:b] = _bar(theta, nf, ga) / TAU
    return dict(fields=fields, lx=lx, ly=ly, g=g, learned=learned, plain=plain, res=res, box=box, edge=edge,
                nf=nf, bar=bar)


@pytest.mark.parametrize("thr_kind", ["box_only", "median_residual"])
@pytest.mark.parametrize("path", ["fused", "in_place"])
def test_learned_mixed_verdicts_every_site(consts, oracle_net, mixed_state, thr_kind, path):
    """Every site of a lattice with scattered fallback sites against the
    oracle's learned collide: the fused step into a destination filled with
    0xFF bytes (NaN, so a site never written shows), and propagate followed
    by the in-place collide. Verdicts: with threshold 1e9 only the training
    box decides (clear-cut here); with the median residual as threshold the
    residual decides too, and sites whose oracle residual lies within 5 % of
    the threshold may take either branch (the GPU's residual comes from its
    own FP32 network pass), but must then equal that branch. Fallback sites
    take the plain FP32 collide: within 2e-6 of the FP64 plain collide per
    w_p (FP32 rounding of deviations up to about 1.5 w_p). The fallback
    count equals the number of fallback verdicts."""
    theta, norm, _ = oracle_net
    st = mixed_state
    w = consts["w"]
    lx, ly = st["lx"], st["ly"]
    res, box = st["res"], st["box"]
    if thr_kind == "box_only":
        thr = 1e9
        tie = st["edge"].copy()
    else:
        thr = float(np.median(res[box]))
        tie = st["edge"] | (box & (np.abs(res - thr) <= 0.05 * thr))
    fb = ~box | (res > thr)
    m = _gpu_net(theta, norm)
    with lb.Lattice(lx, ly, TAU, [torch.from_numpy(a).cuda() for a in st["fields"]], precision="f32s",
                    layout="caosoa") as lat:
        lat.set_surrogate(m, thr)
        if path == "fused":
            lat.bufs[1 - lat.current_buffer()].fill_(0xFF)
            lat.step(1)
        else:
            lat.propagate()
            lat.collide()
        got = (lat.get_populations().cpu().numpy() - w[:, None, None]).reshape(37, -1).T
        nfb, ntot = lat.surrogate_counts()
    m.close()
    assert np.isfinite(got).all()
    err_l = np.max(np.abs(got - st["learned"]) / w, axis=1)
    err_p = np.max(np.abs(got - st["plain"]) / w, axis=1)
    print(f"{path} {thr_kind}: fallback {int(fb.sum())} of {fb.size}, ties {int(tie.sum())}, gpu count {nfb}")
    assert ntot == lx * ly
    clear_l = ~fb & ~tie
    clear_p = fb & ~tie
    _check_sites(err_l[clear_l], st["bar"][clear_l], FLOOR / TAU, what=f"{path} {thr_kind} learned sites")
    assert err_p[clear_p].max() <= 2e-6, err_p[clear_p].max()
    took_plain = err_p <= 2e-6
    assert np.all((err_l[tie] <= st["bar"][tie]) | took_plain[tie])
    assert nfb == int(clear_p.sum()) + int(took_plain[tie].sum())
    assert 0.05 * fb.size < fb.sum() < 0.95 * fb.size  # both branches well represented


def test_gelu16_matches_oracle_on_every_binary16_input():
    """The device's binary16 GELU (lb_mlp_gelu16, the instructions of the
    hidden layers) equals the oracle's operation-by-operation binary16
    evaluation bit for bit on all 63,490 non-NaN binary16 inputs (infinities
    included), and returns a NaN for each NaN input; an odd count exercises
    the unpaired last value."""
    bits = np.arange(65536, dtype=np.uint16)
    x = bits.view(np.float16).astype(np.float64)
    got = lb.gelu16(torch.from_numpy(bits.view(np.int16).copy()).cuda()).cpu().numpy().view(np.uint16)
    with np.errstate(invalid="ignore"):
        want = S.gelu_f16(x)
    nan = np.isnan(x)
    got_v = got.view(np.float16).astype(np.float64)
    assert np.all(np.isnan(got_v[nan]))
    wb = want[~nan].astype(np.float16).view(np.uint16)
    gb = got[~nan]
    wn = np.isnan(want[~nan])
    assert np.array_equal(np.isnan(got_v[~nan]), wn)
    bad = np.flatnonzero((gb != wb) & ~wn)
    assert bad.size == 0, [(float(x[~nan][i]), hex(gb[i]), hex(wb[i])) for i in bad[:8]]
    odd = lb.gelu16(torch.from_numpy(bits[:7].view(np.int16).copy()).cuda()).cpu().numpy().view(np.uint16)
    assert np.array_equal(odd, got[:7])


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 15, 17, 2051])
def test_gelu16_ragged_counts_write_only_their_outputs(n):
    """Counts that leave a lane partly filled (eight values per lane): the
    first n outputs equal those of the full evaluation, and the output
    words past n keep their poison."""
    rng = np.random.default_rng(n)
    bits = rng.integers(0, 0x7C00, size=n, dtype=np.uint16)  # finite, non-negative
    bits[::3] |= 0x8000  # and some negative
    want = lb.gelu16(torch.from_numpy(bits.view(np.int16).copy()).cuda()).cpu().numpy().view(np.uint16)
    x = torch.from_numpy(np.concatenate([bits, np.zeros(16, np.uint16)]).view(np.int16)).cuda()
    y = torch.full((n + 16,), 0x5A5A, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    assert lb.lib().lb_mlp_gelu16(x.data_ptr(), y.data_ptr(), n, None) == lb.LB_OK
    torch.cuda.synchronize()
    out = y.cpu().numpy().view(np.uint16)
    assert np.array_equal(out[:n], want)
    assert np.all(out[n:] == 0x5A5A)
    with np.errstate(invalid="ignore"):
        ref = S.gelu_f16(bits.view(np.float16).astype(np.float64)).astype(np.float16).view(np.uint16)
    assert np.array_equal(out[:n], ref)


def test_binary16_overflow_falls_back_without_leaking(consts, oracle_net):
    """Sites whose moments lie inside the training box but whose populations
    are far from equilibrium (a moment-free perturbation of 3e4 w_p) drive
    the binary16 hidden layer past its largest value: the activations become
    infinite, the outputs NaN, the residual NaN, and the verdict fallback, on
    the device as in the oracle's emulation. Such a site must come back as
    the plain equilibrium (finite), and the ordinary sites of the same call
    must not notice (bars as in test_learned_equilibrium_matches_oracle)."""
    theta, norm, _ = oracle_net
    m = _gpu_net(theta, norm)
    nf = m.get_normalization().astype(np.float64)
    w = consts["w"]
    pre, _ = S.make_pairs(1024, seed=41, tau=TAU)
    rng = np.random.default_rng(5)
    noise = rng.standard_normal(pre.shape) * w
    noise = noise - S.conserved_part(noise)           # moment-free
    wild = np.zeros(pre.shape[0], dtype=bool)
    wild[::3] = True
    pre = np.where(wild[:, None], pre + 3e4 * noise, pre)
    pre = _f32(pre)
    rho, ux, uy, T = S.macro(pre)
    box = S.in_box(rho, ux, uy, T)
    with np.errstate(all="ignore"):
        z = (pre / w - nf[0]) / nf[1]
        o, _ = S.forward(theta, z, emulate=True, infer=True)
    assert np.all(np.isnan(o[wild & box]).any(axis=1))   # the emulation overflows too
    gh, res, fb = m.equilibrium(_dev(pre), 1e9)
    gh, fb = gh.cpu().numpy(), fb.cpu().numpy().astype(bool)
    assert np.all(np.isfinite(gh))
    assert np.all(fb[wild]) and np.array_equal(fb[~wild], ~box[~wild])
    exact = lbm.init(rho[:, None], ux[:, None], uy[:, None], T[:, None])[:, :, 0].T - w
    scale = np.max(np.abs(pre[wild]) / w, axis=1) + 1.0
    assert np.max(np.max(np.abs(gh[wild] - exact[wild]) / w, axis=1) / scale) < 1e-5
    keep = ~wild & box
    with np.errstate(all="ignore"):
        want = S.surrogate_equilibrium(pre[keep], theta, nf, emulate=True)
    _check_sites(np.max(np.abs(gh[keep] - want) / w, axis=1), _bar(theta, nf, pre[keep]),
                 what="ordinary sites beside overflowing ones")
    m.close()
