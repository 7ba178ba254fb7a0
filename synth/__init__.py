"""Seeded synthetic inputs for the expanded-encoding reconstruction.

This module draws the data that stand in for the paper's scanner inputs
(Methods 2.2: the in-vivo k-space, the measured spiral trajectories, the
field-probe spherical-harmonic coefficients, the GRE image and B0 map, and
the ESPIRiT coil maps), none of which are available.  It holds no step of
the reconstruction method itself: no encoding operator, no basis
evaluation, no wavelet, no solver.  It is imported by the oracle's tests,
by the GPU tests and by the benchmark alike; both the oracle and the HIP
path consume its arrays as plain inputs.

Conventions shared with the operator definitions:

* image grid ``N x N``, row-major ``[y][x]`` (x fastest), pixel centres at
  ``(i - N/2) * dx`` with ``dx = fov / N`` (metres);
* trajectory/field series ``coef[T][L]`` in rad per basis unit
  (rad/m^degree), ``time[T]`` in seconds from the first sample;
* ``dw0[R]`` is the off-resonance in rad/s (``2*pi*dB0[Hz]``);
* coil maps ``smaps[C][R]`` complex, scaled so that max_r sum_c |S_c|^2 = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Degree of each real solid-harmonic term, in the basis order used by the
# operator (0th order; x, y, z; five 2nd-order terms; seven 3rd-order terms).
SH_DEGREE = (0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3)
# Crude upper bound of max|b_l| on the box |x|,|y|,|z| <= h, divided by h^deg
# (sum of absolute polynomial coefficients).  Used only to scale the random
# perturbation amplitudes of the synthetic field series.
_SH_COEF_ABS = (1, 1, 1, 1, 1, 1, 4, 1, 2, 4, 1, 6, 8, 6, 2, 4)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One reconstruction problem's shape and recipe."""
    name: str
    n: int                 # image side N
    fov: float             # metres
    ncoils: int            # C
    nsamples: int          # T
    dwell: float           # seconds
    accel: float           # R (acceleration factor of the spiral)
    nbasis: int            # L (9: up to 2nd order, 16: up to 3rd order)
    db0_hz: float          # peak |dB0|
    snr: float
    n_iter: int            # FISTA iterations
    wavelet: str           # "haar" | "db4"
    levels: int            # J
    seed: int
    alpha: float = 1.0     # spiral density exponent (1 = uniform Archimedean)
    z0: float = 0.0        # slice position (metres)
    dwi: bool = False      # apply b=1000-like signal attenuation to the phantom

    @property
    def npix(self) -> int:
        return self.n * self.n

    @property
    def n_pad(self) -> int:
        """Wavelet grid side: N rounded up to a multiple of 2^levels."""
        m = 1 << self.levels
        return -(-self.n // m) * m


# The five workloads the reconstruction is exercised on.
TINY = Workload("tiny-32px-8coil-2048", 32, 0.222, 8, 2048, 2e-6, 1.5, 9, 50.0, 30.0,
                20, "haar", 2, 0, alpha=1.5)
MM15 = Workload("1.5mm-148px-32coil-16384", 148, 0.222, 32, 16384, 1e-6, 4.0, 16, 150.0, 15.0,
                50, "db4", 3, 1)
MM11 = Workload("1.1mm-200px-32coil-40000", 200, 0.220, 32, 40000, 1e-6, 3.0, 16, 200.0, 8.0,
                100, "db4", 4, 2, dwi=True)
DIFF = Workload("diff-128px-16coil-12000", 128, 0.192, 16, 12000, 1e-6, 4.0, 16, 150.0, 15.0,
                10, "db4", 3, 4)
WORKLOADS = {w.name: w for w in (TINY, MM15, MM11, DIFF)}


def batch_workloads(n_slices: int = 5, n_vol: int = 36, seed: int = 3):
    """The batched workload: n_slices x n_vol mixed-size problems.

    Volume v (0-based, 6 b=0 then 30 diffusion directions) takes the size
    class ``v % 3``: 148 px / R=4 / T=16384, 170 px / R=5 / T=17340,
    200 px / R=6 / T=20000; slices sit at z in {-6,-3,0,3,6} mm.  Each
    problem gets its own seed ``1000 + index`` for field perturbations and
    dB0.
    """
    sizes = ((148, 4.0, 16384), (170, 5.0, 17340), (200, 6.0, 20000))
    zs = (-0.006, -0.003, 0.0, 0.003, 0.006)
    out = []
    for s in range(n_slices):
        for v in range(n_vol):
            n, accel, t = sizes[v % 3]
            idx = s * n_vol + v
            out.append(Workload(f"batch-{idx}", n, 0.222, 32, t, 1e-6, accel, 16, 150.0,
                                15.0 if v < 6 else 8.0, 100, "db4", 3, 1000 + idx,
                                z0=zs[s % len(zs)], dwi=v >= 6))
    return out


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


def pixel_coords(n: int, fov: float):
    """Pixel-centre coordinates (metres), each of shape [N][N] (x fastest)."""
    dx = fov / n
    c = (np.arange(n) - n / 2) * dx
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return xx, yy


def phantom(w: Workload) -> np.ndarray:
    """Complex head-like phantom [N*N]: a head ellipse plus 10 random interior
    ellipses with intensities in [0.1, 1], times a smooth background phase
    (degree-2 polynomial, range about +-pi/2).  With ``dwi`` each ellipse is
    attenuated by exp(-1000 s/mm^2 * D), D in [0.5, 3.0]e-3 mm^2/s."""
    rng = _rng(w.seed, 1)
    n = w.n
    u = (np.arange(n) - n / 2 + 0.5) / (n / 2)
    yy, xx = np.meshgrid(u, u, indexing="ij")
    img = np.zeros((n, n))
    head = (xx / 0.72) ** 2 + (yy / 0.9) ** 2 <= 1.0
    img[head] = 0.8 if not w.dwi else 0.8 * math.exp(-1000 * 0.8e-3)
    for _ in range(10):
        cx, cy = rng.uniform(-0.4, 0.4, 2)
        ax, ay = rng.uniform(0.05, 0.3, 2)
        th = rng.uniform(0, np.pi)
        val = rng.uniform(0.1, 1.0)
        if w.dwi:
            val *= math.exp(-1000 * rng.uniform(0.5e-3, 3.0e-3))
        xr = (xx - cx) * np.cos(th) + (yy - cy) * np.sin(th)
        yr = -(xx - cx) * np.sin(th) + (yy - cy) * np.cos(th)
        m = ((xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0) & head
        img[m] = val
    p = rng.uniform(-1, 1, 6)
    ph = p[0] + p[1] * xx + p[2] * yy + p[3] * xx * yy + p[4] * xx ** 2 + p[5] * yy ** 2
    ph = ph / max(np.max(np.abs(ph)), 1e-12) * (np.pi / 2)
    return (img * np.exp(1j * ph)).reshape(-1)


def coil_maps(w: Workload, ncoils: Optional[int] = None) -> np.ndarray:
    """Smooth Gaussian coil sensitivities [C][N*N] on a circle of radius
    0.6*FOV, width 0.35*FOV, phase 2*pi*c/C, normalised so that
    max_r sum_c |S_c(r)|^2 = 1."""
    c_n = w.ncoils if ncoils is None else ncoils
    xx, yy = pixel_coords(w.n, w.fov)
    s = np.empty((c_n, w.npix), dtype=np.complex128)
    for c in range(c_n):
        a = 2 * np.pi * c / c_n
        px, py = 0.6 * w.fov * np.cos(a), 0.6 * w.fov * np.sin(a)
        g = np.exp(-((xx - px) ** 2 + (yy - py) ** 2) / (2 * (0.35 * w.fov) ** 2))
        s[c] = (g * np.exp(1j * a)).reshape(-1)
    s /= np.sqrt(np.max(np.sum(np.abs(s) ** 2, axis=0)))
    return s


def sample_times(w: Workload) -> np.ndarray:
    """Sample times t = n*dwell (seconds), first sample at k-space centre."""
    return np.arange(w.nsamples) * w.dwell


def field_series(w: Workload) -> np.ndarray:
    """Synthetic monitored-field coefficients coef[T][L] (rad / m^degree).

    Terms 1 and 2 (x, y) carry a single-shot spiral-out
    k(t) = k_max u^alpha exp(i 2 pi n_turns u), u = sqrt(t/T_read),
    k_max = pi/dx, n_turns = N/(2R); every other term (including the 0th
    order and z) gets a smooth random series sum_{m=1..4} a_m sin(2 pi m
    t/T_read + psi_m) whose peak phase over the FOV is at most 5% of the
    first-order phase range; the x and y terms get the same kind of
    perturbation at 1% amplitude."""
    rng = _rng(w.seed, 2)
    t_n = w.nsamples
    tt = np.arange(t_n) / t_n
    u = np.sqrt(tt)
    dx = w.fov / w.n
    kmax = np.pi / dx
    n_turns = w.n / (2 * w.accel)
    k = kmax * u ** w.alpha * np.exp(1j * 2 * np.pi * n_turns * u)
    coef = np.zeros((t_n, w.nbasis))
    coef[:, 1] = k.real
    coef[:, 2] = k.imag
    h = w.fov / 2
    phase_range = kmax * h          # rad, peak first-order phase at the FOV edge

    def smooth(amp):
        a = rng.uniform(-1, 1, 4)
        psi = rng.uniform(0, 2 * np.pi, 4)
        s = sum(a[m] * np.sin(2 * np.pi * (m + 1) * tt + psi[m]) for m in range(4))
        return amp * s / max(np.max(np.abs(s)), 1e-12)

    for l in range(w.nbasis):
        deg = SH_DEGREE[l]
        bound = _SH_COEF_ABS[l] * h ** deg
        frac = 0.01 if l in (1, 2) else 0.05
        coef[:, l] += smooth(frac * phase_range / bound)
    return coef


def db0_map(w: Workload) -> np.ndarray:
    """Off-resonance dw0[R] in rad/s: a random cubic polynomial in (x, y)
    scaled to a peak of db0_hz, times 2*pi."""
    rng = _rng(w.seed, 3)
    u = (np.arange(w.n) - w.n / 2 + 0.5) / (w.n / 2)
    yy, xx = np.meshgrid(u, u, indexing="ij")
    terms = [np.ones_like(xx), xx, yy, xx * yy, xx ** 2, yy ** 2,
             xx ** 3, xx ** 2 * yy, xx * yy ** 2, yy ** 3]
    p = rng.normal(size=len(terms))
    f = sum(pi * ti for pi, ti in zip(p, terms))
    f = f / np.max(np.abs(f)) * w.db0_hz
    return (2 * np.pi * f).reshape(-1)


def image_noise(w: Workload, x_clean: np.ndarray) -> np.ndarray:
    """Complex white noise added to the image before encoding: re and im
    each N(0, sigma^2), sigma = mean|x| over the object support / SNR."""
    rng = _rng(w.seed, 4)
    supp = np.abs(x_clean) > 0
    sigma = np.mean(np.abs(x_clean[supp])) / w.snr
    return sigma * (rng.normal(size=x_clean.shape) + 1j * rng.normal(size=x_clean.shape))


def power_start(n_pix: int, seed: int = 7) -> np.ndarray:
    """Seeded complex Gaussian start vector for a power iteration."""
    rng = _rng(seed, 5)
    v = rng.normal(size=n_pix) + 1j * rng.normal(size=n_pix)
    return v / np.linalg.norm(v)


def random_complex(shape, seed: int) -> np.ndarray:
    rng = _rng(seed, 6)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def random_real(shape, seed: int) -> np.ndarray:
    return _rng(seed, 8).normal(size=shape)


@dataclasses.dataclass
class Problem:
    """All raw inputs of one problem (FP64 / complex128 numpy arrays)."""
    w: Workload
    x_true: np.ndarray     # [R] clean object
    x_noisy: np.ndarray    # [R] object + image-domain noise (input to encoding)
    smaps: np.ndarray      # [C][R]
    coef: np.ndarray       # [T][L]
    time: np.ndarray       # [T]
    dw0: np.ndarray        # [R]


def make_problem(w: Workload) -> Problem:
    x = phantom(w)
    return Problem(w, x, x + image_noise(w, x), coil_maps(w), field_series(w),
                   sample_times(w), db0_map(w))


def cartesian_coef(n: int, fov: float, nbasis: int = 3) -> np.ndarray:
    """Fully sampled Cartesian trajectory (T = N^2) in the first-order terms:
    k = 2*pi*m/FOV, m = -N/2..N/2-1 for each axis, row-major over (ky, kx)."""
    m = np.arange(n) - n // 2
    ky, kx = np.meshgrid(m, m, indexing="ij")
    coef = np.zeros((n * n, nbasis))
    coef[:, 1] = (2 * np.pi / fov) * kx.reshape(-1)
    coef[:, 2] = (2 * np.pi / fov) * ky.reshape(-1)
    return coef
