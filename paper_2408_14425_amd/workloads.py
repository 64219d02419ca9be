"""Seeded synthetic inputs for the radiance-cascades solver.

This module is shared by the tests, the benchmark and the oracle harness. It
only draws and shapes random fields; it contains none of the method's
arithmetic (no ray marching, merging, rates or populations).

All fields are built in float64 with ``numpy.random.default_rng(seed)``
(PCG64) and rounded to float32, the precision the GPU path consumes. The
oracle receives the same float32 values widened to float64, so that parity
measures solver error and not input rounding.

Layout: row-major with x fastest, fields ``[n_wave][nz][nx]``. Cell (x, z)
occupies [x, x+1) x [z, z+1) in cell units; its centre is (x+1/2, z+1/2).

The paper's own production input (a 2.5D MHD prominence snapshot, Sec. 4.1)
is not available; these generators stand in for it with the same shape
class: uniform 2D grids with optically thick structures embedded in thin
surroundings, a line-profile-shaped opacity over wavelength, and smooth
source functions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Second radiation constant h c / k_B [m K], used only to shape a smooth,
# Planck-like source-function input for the multi-wavelength workload.
_C2_RAD = 1.4388e-2


def n_cascades_for(nx: int, nz: int) -> int:
    """Default cascade count for a grid: ceil(log4(max(nx, nz))) + 2.

    Reproduces 5 cascades at 64^2 and 7 at 1024^2 (the paper's scaling law,
    Eq. RcScalingLaw, with alpha = 2 and t_1 = 1.5 cells).
    """
    m = max(int(nx), int(nz))
    k = 0
    while 4 ** k < m:
        k += 1
    return k + 2


def grf(rng: np.random.Generator, shape: tuple[int, int], corr_len: float) -> np.ndarray:
    """Gaussian random field: white noise filtered in Fourier space by a
    Gaussian kernel of correlation length ``corr_len`` cells, standardised to
    zero mean and unit variance (periodic)."""
    nz, nx = shape
    noise = rng.standard_normal(shape)
    kz = np.fft.fftfreq(nz)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi * corr_len) ** 2 * (kx * kx + kz * kz))
    f = np.fft.ifft2(np.fft.fft2(noise) * filt).real
    f -= f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


@dataclass
class FormalSolveInput:
    """chi, eta: float32 ``[n_wave][nz][nx]``; voxel_scale: length of one cell
    in the units chi is given per."""
    chi: np.ndarray
    eta: np.ndarray
    voxel_scale: float
    n_cascades: int
    name: str

    @property
    def nx(self) -> int:
        return int(self.chi.shape[2])

    @property
    def nz(self) -> int:
        return int(self.chi.shape[1])

    @property
    def n_wave(self) -> int:
        return int(self.chi.shape[0])


def blobs_medium(n: int = 64, seed: int = 1, n_blobs: int = 3) -> FormalSolveInput:
    """Single-wavelength medium on an n x n grid: opacity log-uniform in
    [1e-3, 1e1] per cell plus ``n_blobs`` optically thick Gaussian blobs of
    peak 1e3 (centres uniform in [n/8, 7n/8]^2, widths uniform in [2, 5]
    cells); a smooth sinusoidal source function in [0.5, 2]; eta = chi * S.

    At n = 64, seed = 1 this is the 64^2, 1-wavelength, 5-cascade formal-solve
    parity workload.
    """
    rng = np.random.default_rng(seed)
    chi = 10.0 ** rng.uniform(-3.0, 1.0, size=(n, n))
    zc, xc = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    for _ in range(n_blobs):
        cx, cz = rng.uniform(n / 8.0, 7.0 * n / 8.0, size=2)
        sig = rng.uniform(2.0, 5.0)
        chi = chi + 1e3 * np.exp(-((xc - cx) ** 2 + (zc - cz) ** 2) / (2.0 * sig * sig))
    phx, phz = rng.uniform(0.0, 2.0 * math.pi, size=2)
    src = 1.25 + 0.75 * np.sin(2 * math.pi * xc / n + phx) * np.sin(2 * math.pi * zc / n + phz)
    chi32 = chi.astype(np.float32)
    eta32 = (chi32.astype(np.float64) * src).astype(np.float32)
    return FormalSolveInput(chi32[None], eta32[None], 1.0, n_cascades_for(n, n),
                            f"blobs{n}x{n}_s{seed}")


def line_medium(n: int = 1024, n_wave: int = 64, seed: int = 2, nz: int | None = None,
                wave_subset: np.ndarray | None = None) -> FormalSolveInput:
    """Multi-wavelength medium: a log-normal density rho = exp(1.5 GRF(32)),
    a Gaussian line-profile opacity over wavelength with 0.1 .. 1e4 contrast
    (kappa_w = 0.1 + 1e4 exp(-x_w^2), x_w spanning [-4, 4]), chi = 1e-2 rho
    kappa_w per cell, a temperature T = 6000 + 2000 tanh(GRF(128)) K and a
    Planck-ratio source function S = (e^{c2/(l0 T0)} - 1)/(e^{c2/(l0 T)} - 1)
    at l0 = 500 nm, T0 = 6000 K; eta = chi * S.

    At n = 1024, n_wave = 64, seed = 2 this is the 1024^2, 64-wavelength,
    7-cascade formal-solve workload. ``wave_subset`` selects wavelength
    indices out of the ``n_wave`` grid (same fields, fewer wavelengths).
    """
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    rho = np.exp(1.5 * grf(rng, (nz, n), 32.0 * n / 1024.0 if n < 1024 else 32.0))
    temp = 6000.0 + 2000.0 * np.tanh(grf(rng, (nz, n), 128.0 * n / 1024.0 if n < 1024 else 128.0))
    lam0, t0 = 500e-9, 6000.0
    src = np.expm1(_C2_RAD / (lam0 * t0)) / np.expm1(_C2_RAD / (lam0 * temp))
    waves = np.arange(n_wave) if wave_subset is None else np.asarray(wave_subset)
    half = 0.5 * (n_wave - 1)
    xw = (waves - half) / (half if half > 0 else 1.0) * 4.0
    kappa = 0.1 + 1e4 * np.exp(-xw * xw)
    chi = np.empty((len(waves), nz, n), dtype=np.float32)
    eta = np.empty_like(chi)
    for i, k in enumerate(kappa):
        c = (1e-2 * rho * k).astype(np.float32)
        chi[i] = c
        eta[i] = (c.astype(np.float64) * src).astype(np.float32)
    return FormalSolveInput(chi, eta, 1.0, n_cascades_for(n, nz), f"line{n}x{nz}_w{n_wave}_s{seed}")


def disc_in_vacuum(n: int = 256, radius: float = 4.0, chi_disc: float = 1e3,
                   src: float = 1.0) -> FormalSolveInput:
    """Opaque pixelised disc in vacuum at the grid centre: every cell whose
    centre lies within ``radius`` of the centre gets chi = ``chi_disc``,
    eta = chi * ``src``; everything else is empty (chi = eta = 0)."""
    zc, xc = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    r = np.hypot(xc - n / 2.0, zc - n / 2.0)
    inside = r <= radius
    chi = np.where(inside, chi_disc, 0.0).astype(np.float32)
    eta = np.where(inside, chi_disc * src, 0.0).astype(np.float32)
    return FormalSolveInput(chi[None], eta[None], 1.0, n_cascades_for(n, n), f"disc{n}_r{radius}")


def active_cells(nx: int, nz: int, seed: int = 7, frac: float = 0.25, corr_len: float | None = None) -> np.ndarray:
    """Flags of a sparse solve: cool structure in a hot corona. A Gaussian
    random field (correlation length ``corr_len``, default max(nx, nz) / 16)
    thresholded at its (1 - frac) quantile marks ``frac`` of the cells as
    active ([nz][nx] bool); the paper flags about 25% of its cells by a
    temperature cut."""
    rng = np.random.default_rng(seed)
    cl = max(nx, nz) / 16.0 if corr_len is None else corr_len
    f = grf(rng, (nz, nx), cl)
    return f > np.quantile(f, 1.0 - frac)


def uneven_batch(seed: int = 4, n_atm: int = 16, sizes=None, waves=None):
    """List of (side, n_wave, atmosphere seed) for a batch of independent
    line-medium atmospheres of uneven size: sides uniform on multiples of 128
    in [256, 2048], wavelength counts uniform on multiples of 32 in [32, 256].
    """
    rng = np.random.default_rng(seed)
    sizes = list(range(256, 2049, 128)) if sizes is None else list(sizes)
    waves = list(range(32, 257, 32)) if waves is None else list(waves)
    out = []
    for a in range(n_atm):
        out.append((int(rng.choice(sizes)), int(rng.choice(waves)), 4000 + a))
    return out


# ------------------------------------------------------------------ non-LTE

# Synthetic hydrogen-like model atom: 3 bound levels + continuum. Level data
# (energies [eV], statistical weights), two lines (lower, upper, rest
# wavelength [nm], oscillator strength), one bound-free continuum (lower,
# upper, edge wavelength [nm], cross-section at the edge [m^2], scaling as
# lambda^3 below the edge), atomic mass [amu], and per-transition collisional
# de-excitation coefficients q [m^3/s] (downward rate n_e q (T/1e4 K)^-1/2).
# This is input data, in the role of an atomic-model file.
SYNTH_ATOM = {
    # energies consistent with the line and edge wavelengths (E = h c / lambda)
    "E_eV": [0.0, 10.1985850483837, 12.0877817088518, 13.5977405607809],
    "g": [2.0, 8.0, 18.0, 1.0],
    "mass_amu": 1.008,
    "lines": [(0, 1, 121.57, 0.4164), (1, 2, 656.28, 0.6407)],
    "continua": [(0, 3, 91.18, 6.3e-22)],
    # transitions in order: lines, then continua
    "q_coll": [2.6e-11, 2.4e-10, 1.0e-12],
}


@dataclass
class NlteInput:
    """A non-LTE problem: atmosphere on an nx x nz grid and a wavelength grid.

    T, ne, ntot: [nz][nx] float64 (K, m^-3, m^-3; ntot = all hydrogen
    particles, neutral and ionised); vel: [2][nz][nx] float32 (vx, vz, m/s);
    lambda_nm: [n_wave] float64; trans: [n_wave] int32 index of the
    transition each wavelength belongs to (lines first, then continua), grouped
    by transition; dnu: [n_wave] float64 frequency quadrature weights [Hz]
    (trapezoid in frequency within each transition's sub-grid); voxel: cell
    size [m]."""
    T: np.ndarray
    ne: np.ndarray
    ntot: np.ndarray
    vel: np.ndarray
    lambda_nm: np.ndarray
    trans: np.ndarray
    dnu: np.ndarray
    voxel: float
    atom: dict
    name: str

    @property
    def nx(self) -> int:
        return int(self.T.shape[1])

    @property
    def nz(self) -> int:
        return int(self.T.shape[0])

    @property
    def n_wave(self) -> int:
        return int(len(self.lambda_nm))


_C_LIGHT = 2.99792458e8


def nlte_wavelength_grid(atom: dict, n_line: int = 64, n_cont: int = 32, vmax: float = 150e3,
                         stretch: float = 3.0):
    """Per line: n_line points over +-vmax in Doppler velocity, sinh-stretched
    towards the core; per continuum: n_cont points log-spaced over
    [0.5, 1] x the edge wavelength. Returns (lambda_nm, trans, dnu)."""
    lams, trans, dnus = [], [], []
    t = 0
    for (_, _, lam0, _) in atom["lines"]:
        s = np.linspace(-1.0, 1.0, n_line)
        v = vmax * np.sinh(stretch * s) / np.sinh(stretch)
        lam = lam0 * (1.0 + v / _C_LIGHT)
        lams.append(lam)
        trans.append(np.full(n_line, t))
        t += 1
    for (_, _, ledge, _) in atom["continua"]:
        lam = ledge * np.logspace(np.log10(0.5), 0.0, n_cont)
        lams.append(lam)
        trans.append(np.full(n_cont, t))
        t += 1
    for lam in lams:
        nu = _C_LIGHT / (lam * 1e-9)
        w = np.zeros_like(nu)
        d = np.abs(np.diff(nu))
        w[:-1] += 0.5 * d
        w[1:] += 0.5 * d
        dnus.append(w)
    return (np.concatenate(lams), np.concatenate(trans).astype(np.int32), np.concatenate(dnus))


def nlte_atmosphere(n: int = 64, seed: int = 3, n_line: int = 64, n_cont: int = 32,
                    n0: float = 5e16, voxel: float = 1e3, nz: int | None = None,
                    corona_frac: float = 0.0) -> NlteInput:
    """Synthetic prominence-like atmosphere: a hot (1e5 K), tenuous
    background with cool blobs, log10 T = 5 - sum_b (5 - log10 T_b)
    exp(-r^2 / 2 sigma_b^2) clipped to [log10 5e3, 5], 24 blobs per 1024^2
    (count scaled by area, at least 3), widths sigma uniform in [20, 80]
    cells from 512^2 up (the cells keep their size, so a larger grid is a
    larger patch of the same kind of atmosphere) and in [5, 20] cells on
    smaller grids (several blobs in view), blob temperatures log-uniform in
    [5e3, 3e4] K;
    hydrogen density
    ntot = n0 (1e4 K / T); a prescribed ionisation fraction
    x(T) = 1e-4 + (1 - 1e-4) / (1 + (6540 K / T)^16) (shaped like a hydrogen
    ionisation curve at these densities: about 1% at 5000 K, 75% at 7000 K),
    ne = x ntot; velocities
    uniform in +-20 km/s on a 32 x 32 coarse grid, bilinearly upsampled.
    corona_frac > 0: that fraction of the cells, the hottest (the background
    farthest from the blobs), becomes 1e6 K corona (density and ionisation
    follow T as above), so a 250 kK cut flags the rest."""
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    zc, xc = np.meshgrid(np.arange(nz) + 0.5, np.arange(n) + 0.5, indexing="ij")
    n_blobs = max(3, int(round(24 * n * nz / 1024.0 ** 2)))
    logt = np.full((nz, n), 5.0)
    for _ in range(n_blobs):
        cx, cz = rng.uniform(0, n), rng.uniform(0, nz)
        sig = rng.uniform(20.0, 80.0) * (1.0 if max(n, nz) >= 512 else 0.25)
        tb = 10 ** rng.uniform(np.log10(5e3), np.log10(3e4))
        logt -= (5.0 - np.log10(tb)) * np.exp(-((xc - cx) ** 2 + (zc - cz) ** 2) / (2 * sig * sig))
    T = 10 ** np.clip(logt, np.log10(5e3), 5.0)
    if corona_frac > 0.0:
        T = np.where(T > np.quantile(T, 1.0 - corona_frac), 1e6, T)
    ntot = n0 * (1e4 / T)
    xion = 1e-4 + (1.0 - 1e-4) / (1.0 + (6540.0 / T) ** 16)
    ne = xion * ntot
    coarse = rng.uniform(-20e3, 20e3, size=(2, 32, 32))
    vel = np.empty((2, nz, n))
    gz = (np.arange(nz) + 0.5) / nz * 32 - 0.5
    gx = (np.arange(n) + 0.5) / n * 32 - 0.5
    for d in range(2):
        rows = np.array([np.interp(gx, np.arange(32), coarse[d, j]) for j in range(32)])
        vel[d] = np.array([np.interp(gz, np.arange(32), rows[:, i]) for i in range(n)]).T
    lam, trans, dnu = nlte_wavelength_grid(SYNTH_ATOM, n_line, n_cont)
    return NlteInput(T, ne, ntot, vel.astype(np.float32), lam, trans, dnu, voxel, SYNTH_ATOM,
                     f"nlte{n}x{nz}_w{len(lam)}_s{seed}" + (f"_corona{corona_frac:g}" if corona_frac > 0 else ""))


def mlp_init_params(n_in: int = 6, width: int = 128, depth: int = 4, n_out: int = 4, seed: int = 0):
    """Seeded initial parameters of the warm-start network, flat FP32, layer
    by layer W [fan_in][fan_out] then b [fan_out], each uniform in
    +-1/sqrt(fan_in) (the common default for linear layers)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [width] * depth + [n_out]
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = 1.0 / np.sqrt(a)
        out.append(rng.uniform(-lim, lim, a * b))
        out.append(rng.uniform(-lim, lim, b))
    return np.concatenate(out).astype(np.float32)
