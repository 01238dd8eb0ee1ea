"""Seeded synthetic workloads (no CHR arithmetic lives here).

The paper evaluates on the temperature field of the Nyx cosmology code
(Sec. III).  That data is not available here, so these seeded synthetic fields
stand in for it, with the shapes and value structure of the five workloads the
benchmark and tests use:

* ``gaussians``   -- sum of 8 isotropic Gaussians plus small noise (64^3);
* ``taylor_green`` -- Taylor-Green vortex velocity magnitude plus noise (256^3);
* ``phantom``     -- nested blurred ellipsoid shells with Poisson-like noise,
                    values in [0, 4095] (512^3);
* ``grf``         -- Gaussian random field with a k^-5/3 energy spectrum,
                    evolving by phase drift (timesteps of uneven sizes, and
                    the 1024^3 serving field).

Every generator is a pure function of its arguments and seed.  Both the GPU
path and the CPU oracle consume the arrays produced here; nothing in this
module compresses, reconstructs or extracts anything.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 240805462


def abs_error_bound(rel: float, field: np.ndarray) -> float:
    """Relative bound -> absolute bound: rel * (max - min), in double."""
    return float(rel) * (float(np.float64(field.max())) - float(np.float64(field.min())))


# --------------------------------------------------------------------------
# 1. Gaussians
# --------------------------------------------------------------------------

def gaussians(n: int = 64, seed: int = SEED_BASE + 1, n_blobs: int = 8,
              noise: float = 1e-3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, n - 1, size=(n_blobs, 3))
    sig = rng.uniform(4, 12, size=n_blobs)
    amp = rng.uniform(0.5, 1.0, size=n_blobs)
    ax = np.arange(n, dtype=np.float64)
    f = np.zeros((n, n, n), np.float64)
    for j in range(n_blobs):
        gz = np.exp(-((ax - c[j, 0]) ** 2) / (2 * sig[j] ** 2))
        gy = np.exp(-((ax - c[j, 1]) ** 2) / (2 * sig[j] ** 2))
        gx = np.exp(-((ax - c[j, 2]) ** 2) / (2 * sig[j] ** 2))
        f += amp[j] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    f += rng.normal(0.0, noise, size=f.shape)
    return f.astype(np.float32)


# --------------------------------------------------------------------------
# 2. Taylor-Green vortex velocity magnitude
# --------------------------------------------------------------------------

def taylor_green(n: int = 256, seed: int = SEED_BASE + 2, nu: float = 0.1,
                 noise: float = 1e-4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0)
    F = np.exp(-3.0 * nu * t)
    a = 2 * np.pi * np.arange(n, dtype=np.float64) / n
    sx, cx = np.sin(a), np.cos(a)
    out = np.empty((n, n, n), np.float32)
    for z in range(n):  # slab by slab to bound memory
        cz = np.cos(a[z])
        u = F * sx[None, :] * cx[:, None] * cz       # [y][x]: sin x cos y cos z
        v = -F * cx[None, :] * sx[:, None] * cz      # -cos x sin y cos z
        mag = np.sqrt(u * u + v * v)
        out[z] = (mag + rng.normal(0.0, noise, size=mag.shape)).astype(np.float32)
    return out


# --------------------------------------------------------------------------
# 3. Medical-like phantom
# --------------------------------------------------------------------------

def phantom(n: int = 512, seed: int = SEED_BASE + 3):
    """Returns (field, intensities) -- intensities[j] is the value inside
    ellipsoid j (0 = outermost) before blurring and noise."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    scales = np.array([1.0, 0.8, 0.6, 0.4, 0.2])
    semi = 0.45 * n * scales[:, None] * rng.uniform(0.8, 1.0, size=(5, 3))
    centre = (n - 1) / 2.0 + rng.uniform(-0.02, 0.02, size=(5, 3)) * n
    inten = rng.choice(np.arange(200, 4001), size=5, replace=False).astype(np.float64)
    ax = np.arange(n, dtype=np.float64)
    vol = np.zeros((n, n, n), np.float32)
    for z in range(n):
        sl = np.zeros((n, n), np.float32)
        for j in range(5):  # nested: inner ellipsoids overwrite outer ones
            dz = ((ax[z] - centre[j, 0]) / semi[j, 0]) ** 2
            dy = ((ax[:, None] - centre[j, 1]) / semi[j, 1]) ** 2
            dx = ((ax[None, :] - centre[j, 2]) / semi[j, 2]) ** 2
            sl[(dz + dy + dx) <= 1.0] = inten[j]
        vol[z] = sl
    vol = gaussian_filter(vol, sigma=1.5, mode="nearest", output=np.float32)
    for z in range(n):
        sd = np.sqrt(np.maximum(vol[z].astype(np.float64), 1.0))
        vol[z] = np.clip(vol[z] + rng.normal(0.0, 1.0, size=sd.shape) * sd, 0, 4095).astype(np.float32)
    return vol, inten


# --------------------------------------------------------------------------
# 4/5. Gaussian random field with a k^-5/3 spectrum
# --------------------------------------------------------------------------

def grf(n: int, t: float = 0.0, seed: int = SEED_BASE + 4) -> np.ndarray:
    """Real field on an n^3 periodic grid whose Fourier amplitudes fall as
    |k|^(-11/6) (energy spectrum k^(-5/3)), with the phase of every mode
    drifting as 0.1*|k|^(2/3)*t.  Normalised to mean 0, standard deviation 1."""
    rng = np.random.default_rng((seed, n))
    kz = np.fft.fftfreq(n) * n
    kx = np.fft.rfftfreq(n) * n
    kk = np.sqrt(kz[:, None, None] ** 2 + kz[None, :, None] ** 2 + kx[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (-11.0 / 6.0)
    coef = rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)
    phase = np.exp(1j * 0.1 * np.power(kk, 2.0 / 3.0) * t)
    spec = amp * coef * phase
    spec[0, 0, 0] = 0
    f = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
    f = (f - f.mean()) / f.std()
    return f.astype(np.float32)


def grf_torch(n: int, t: float = 0.0, seed: int = SEED_BASE + 4, device="cuda"):
    """The recipe of ``grf`` drawn with torch's generator on `device` (for
    fields too large to synthesise quickly on the host): same spectrum,
    phase drift and normalisation; different random draws."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 4099 + int(n))
    kz = torch.fft.fftfreq(n, device=device, dtype=torch.float32) * n
    kx = torch.fft.rfftfreq(n, device=device, dtype=torch.float32) * n
    kk = torch.sqrt(kz[:, None, None] ** 2 + kz[None, :, None] ** 2 + kx[None, None, :] ** 2)
    amp = torch.where(kk > 0, kk.clamp_min(1e-30) ** (-11.0 / 6.0), torch.zeros_like(kk))
    re = torch.randn(kk.shape, generator=g, device=device)
    im = torch.randn(kk.shape, generator=g, device=device)
    ph = 0.1 * kk ** (2.0 / 3.0) * float(t)
    spec = torch.complex(amp * (re * torch.cos(ph) - im * torch.sin(ph)), amp * (re * torch.sin(ph) + im * torch.cos(ph)))
    del re, im, ph, amp, kk
    spec[0, 0, 0] = 0
    f = torch.fft.irfftn(spec, s=(n, n, n), dim=(0, 1, 2))
    del spec
    f = (f - f.mean()) / f.std()
    return f.float().contiguous()


def sample_quantiles(values, count: int = 8, max_samples: int = 1 << 20):
    """Isovalues at the (2j+1)/(2 count) quantiles of an evenly strided sample
    (numpy array or torch tensor), as float32 values."""
    flat = values.reshape(-1)
    step = max(1, flat.shape[0] // max_samples)
    sample = flat[::step]
    sample = sample.cpu().numpy() if hasattr(sample, "cpu") else np.asarray(sample)
    qs = [(2 * j + 1) / (2 * count) for j in range(count)]
    return [float(np.float32(v)) for v in np.quantile(sample.astype(np.float64), qs)]


def batch_sizes(count: int = 64, seed: int = SEED_BASE + 4):
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice([96, 128, 192, 256, 384], size=count)]


def quantile_isovalues(field: np.ndarray, count: int = 8):
    qs = [(2 * j + 1) / (2 * count) for j in range(count)]
    return [float(np.float32(v)) for v in np.quantile(field, qs)]


# --------------------------------------------------------------------------
# Named workloads: field + compression parameters
# --------------------------------------------------------------------------

def workload(name: str, n: int | None = None):
    """Returns dict(field, levels, error_bound, isovalues, block, name)."""
    if name == "gaussians64":
        f = gaussians(n or 64)
        return dict(name=name, field=f, levels=3, block=64, error_bound=abs_error_bound(1e-3, f),
                    isovalues=[0.3])
    if name == "taylor_green256":
        f = taylor_green(n or 256)
        isos = [float(np.float32(v)) for v in np.percentile(f, [25, 50, 75])]
        return dict(name=name, field=f, levels=5, block=64, error_bound=abs_error_bound(1e-4, f),
                    isovalues=isos)
    if name == "phantom512":
        f, inten = phantom(n or 512)
        k = float(np.float32(0.5 * (inten[1] + inten[2])))
        return dict(name=name, field=f, levels=6, block=64, error_bound=abs_error_bound(1e-3, f),
                    isovalues=[k])
    raise KeyError(name)
