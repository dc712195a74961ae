"""Physics of the body force and walls at scale on the GPU: the
Rayleigh-Taylor instability (the paper's production setting, Section 3).

A light (hot) layer under a heavy (cold) one, each isothermal and in
hydrostatic balance under gravity g along -y, between walls at the layers'
temperatures, with the interface displaced by 2 sites in a cosine of
wavelength LX. Linear theory for a sharp interface between inviscid,
incompressible layers gives growth exp(sigma t) with sigma = sqrt(A k g')
(Atwood number A, wavenumber k = 2 pi / LX, g' = g / r in sites per step^2).
Viscosity, the diffusion that widens the interface and the layers'
compressibility all slow it; on this lattice (512 x 512, tau = 0.6, g =
4e-4) the measured mean rate is about 0.6 sigma. The tests check what no
plausible error survives: the unstable stratification grows by more than
e^1.5 over 10,000 steps at a mean rate between 0.3 and 1 sigma; the same
layers inverted (heavy below) do not grow; without gravity the
perturbation only diffuses away. Measured by the first Fourier mode in x of
the temperature deviation from its row mean.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1804_01918_amd import lb  # noqa: E402

LX = LY = 512
TAU = 0.6
G = 4e-4


def _layers(t_lo, t_hi, g, eta0=2.0):
    """Hydrostatic isothermal layers (p = rho T continuous at the interface,
    d ln p / dy = -g r / T), interface at LY/2 + eta0 cos(2 pi x / LX)."""
    r = lb.model_constants()[0]
    y = np.arange(LY)[None, :] + 0.5
    yi = LY / 2 + eta0 * np.cos(2 * np.pi * np.arange(LX) / LX)[:, None]
    p_i = np.exp(-g * r / t_lo * yi)
    p = np.where(y < yi, np.exp(-g * r / t_lo * y), p_i * np.exp(-g * r / t_hi * (y - yi)))
    T = np.where(y < yi, t_lo, t_hi) * np.ones_like(p)
    rho = p / T
    rho = rho / rho.mean()
    z = np.zeros((LX, LY))
    return rho, z, z.copy(), T


def _amplitudes(t_lo, t_hi, g, chunks, per=250):
    fields = _layers(t_lo, t_hi, g)
    mode = torch.cos(2 * math.pi * torch.arange(LX, device="cuda", dtype=torch.float64) / LX)
    out = []
    with lb.Lattice(LX, LY, TAU, fields, precision="f32s", layout="caosoa", force=(0.0, -g), walls=True,
                    t_bottom=t_lo, t_top=t_hi) as lat:
        for i in range(chunks + 1):
            if i:
                lat.step(per)
            T = lat.moments()[3]
            out.append(float(((T - T.mean(0, keepdim=True)) * mode[:, None]).sum() / LX))
    return np.array(out), per


def _sigma(g):
    r = lb.model_constants()[0]
    atwood = (1 / 0.95 - 1 / 1.05) / (1 / 0.95 + 1 / 1.05)
    return math.sqrt(atwood * (2 * math.pi / LX) * g / r)


def test_rayleigh_taylor_interface_grows():
    a, per = _amplitudes(1.05, 0.95, G, 40)
    print("unstable amplitudes:", np.round(a[::4], 4), flush=True)
    assert np.all(np.isfinite(a))
    assert a[-1] / a[0] > math.exp(1.5)
    # mean growth rate over steps 2500..10000 (after the acoustic adjustment)
    rate = (math.log(abs(a[-1])) - math.log(abs(a[10]))) / (30 * per)
    ratio = rate / _sigma(G)
    print(f"growth rate {rate:.3e} per step = {ratio:.3f} of sqrt(A k g)", flush=True)
    assert 0.3 < ratio < 1.0, ratio


def test_inverted_layers_do_not_grow():
    a, _ = _amplitudes(0.95, 1.05, G, 16)
    print("stable amplitudes:", np.round(a, 4), flush=True)
    assert np.max(np.abs(a)) <= 1.05 * abs(a[0])


def test_without_gravity_the_perturbation_diffuses():
    a, _ = _amplitudes(1.05, 0.95, 0.0, 16)
    print("no-gravity amplitudes:", np.round(a, 4), flush=True)
    assert abs(a[-1]) < abs(a[0]) and np.max(np.abs(a)) <= 1.05 * abs(a[0])
