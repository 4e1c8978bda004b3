"""Seeded synthetic inputs (initial fields and force fields).

Shared by the tests, the benchmark and the oracle's checks. It contains no
part of the lattice Boltzmann method: only velocity/density/force fields on a
periodic grid, returned as NumPy arrays with shape (3, nz, ny, nx) for vectors
and (nz, ny, nx) for scalars (x fastest).

Seeds: initial fields 1202, forcing 6074, adjoint force parameter 42.
"""
from __future__ import annotations

import numpy as np

SEED_INIT = 1202
SEED_FORCE = 6074
SEED_PARAM = 42


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def taylor_green_3d(shape, u0=0.02, rho_mode="pressure"):
    """3D Taylor-Green vortex on a periodic box of side L = nx (k = 2 pi / L).

    u = u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0). With
    rho_mode='pressure' the density carries the standard incompressible
    pressure p = (u0^2/16)(cos 2kx + cos 2ky)(cos 2kz + 2) through rho = 1 + 3p;
    with rho_mode='uniform' rho = 1.
    """
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    k = 2 * np.pi / nx
    ky, kz = 2 * np.pi / ny, 2 * np.pi / nz
    u = np.zeros((3,) + tuple(shape))
    u[0] = u0 * np.sin(k * x) * np.cos(ky * y) * np.cos(kz * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(ky * y) * np.cos(kz * z)
    if rho_mode == "pressure":
        p = (u0 ** 2 / 16.0) * (np.cos(2 * k * x) + np.cos(2 * ky * y)) * (np.cos(2 * kz * z) + 2.0)
        rho = 1.0 + 3.0 * p
    else:
        rho = np.ones(tuple(shape))
    return rho, u


def taylor_green_2d_in_3d(shape, u0=0.01):
    """u = u0 (sin kx cos ky, -cos kx sin ky, 0), independent of z; rho = 1 + 3p,
    p = (u0^2/4)(cos 2kx + cos 2ky). Exact Navier-Stokes solution decaying as exp(-2 nu k^2 t)."""
    nz, ny, nx = shape
    x, y, _ = _grid(shape)
    k = 2 * np.pi / nx
    u = np.zeros((3,) + tuple(shape))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y)
    rho = 1.0 + 3.0 * (u0 ** 2 / 4.0) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho, u


def shear_wave(shape, amp=1e-4, axis_u=0, axis_k=1):
    """u_{axis_u} = amp sin(2 pi y / L) along axis_k; rho = 1."""
    x, y, z = _grid(shape)
    coord = (x, y, z)[axis_k]
    L = shape[2 - axis_k]
    u = np.zeros((3,) + tuple(shape))
    u[axis_u] = amp * np.sin(2 * np.pi * coord / L)
    return np.ones(tuple(shape)), u


def _wavenumbers(shape):
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    return KX, KY, KZ


def _project_solenoidal(hat, KX, KY, KZ):
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2s = np.where(k2 == 0, 1.0, k2)
    dot = (hat[0] * KX + hat[1] * KY + hat[2] * KZ) / k2s
    return np.stack([hat[0] - dot * KX, hat[1] - dot * KY, hat[2] - dot * KZ])


def turbulence_velocity(shape, k0=4.0, urms=0.03, seed=SEED_INIT):
    """Solenoidal Gaussian random velocity with E(k) ~ k^4 exp(-2 (k/k0)^2).

    k in units of 2 pi / L. White noise in physical space is filtered by
    sqrt(E(k) / k^2) (shell area), projected onto the plane normal to k, and
    scaled so that the per-component rms sqrt(<|u|^2>/3) equals ``urms``.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3,) + tuple(shape))
    hat = np.fft.rfftn(noise, axes=(1, 2, 3))
    KX, KY, KZ = _wavenumbers(shape)
    k = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    ks = np.where(k == 0, 1.0, k)
    amp = np.where(k == 0, 0.0, np.sqrt(ks ** 4 * np.exp(-2.0 * (ks / k0) ** 2) / ks ** 2))
    hat = _project_solenoidal(hat * amp, KX, KY, KZ)
    u = np.fft.irfftn(hat, s=tuple(shape), axes=(1, 2, 3))
    u *= urms / np.sqrt((u ** 2).sum(axis=0).mean() / 3.0)
    return u


def band_forcing(shape, kmin=1.0, kmax=2.0, frms=1e-4, seed=SEED_FORCE):
    """Static solenoidal force on integer wave vectors with kmin <= |k| <= kmax.

    Random complex Gaussian amplitudes, projected normal to k, Hermitian
    symmetric (real field), scaled so that the rms of |F| equals ``frms``.
    The field is sum over one representative k of each +-k pair of
    2 Re(a_k exp(2 pi i k.x / L)), evaluated by an inverse real FFT.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    kmax_i = int(np.floor(kmax))
    modes = []
    for a in range(-kmax_i, kmax_i + 1):
        for b in range(-kmax_i, kmax_i + 1):
            for c in range(-kmax_i, kmax_i + 1):
                kk = a * a + b * b + c * c
                if kmin ** 2 <= kk <= kmax ** 2 and (c, b, a) > (0, 0, 0):
                    modes.append((a, b, c))
    hat = np.zeros((3, nz, ny, nx // 2 + 1), dtype=np.complex128)
    scale = float(nx * ny * nz)
    for a, b, c in modes:
        kv = np.array([a, b, c], dtype=np.float64)
        amp = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        amp = amp - kv * (amp @ kv) / (kv @ kv)
        if a > 0:
            hat[:, c % nz, b % ny, a] += scale * amp
        elif a < 0:
            hat[:, (-c) % nz, (-b) % ny, -a] += scale * np.conj(amp)
        else:
            hat[:, c % nz, b % ny, 0] += scale * amp
            hat[:, (-c) % nz, (-b) % ny, 0] += scale * np.conj(amp)
    F = np.fft.irfftn(hat, s=tuple(shape), axes=(1, 2, 3))
    F *= frms / np.sqrt((F ** 2).sum(axis=0).mean())
    return F


def smooth_random_force(shape, sigma=4.0, frms=1e-5, seed=SEED_PARAM):
    """White noise filtered by a Gaussian of width ``sigma`` cells (spectrally),
    scaled to per-component rms ``frms``. Not projected (has a divergence)."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3,) + tuple(shape))
    hat = np.fft.rfftn(noise, axes=(1, 2, 3))
    nz, ny, nx = shape
    KX, KY, KZ = _wavenumbers(shape)
    kr2 = (2 * np.pi * KX / nx) ** 2 + (2 * np.pi * KY / ny) ** 2 + (2 * np.pi * KZ / nz) ** 2
    F = np.fft.irfftn(hat * np.exp(-0.5 * kr2 * sigma ** 2), s=tuple(shape), axes=(1, 2, 3))
    F -= F.mean(axis=(1, 2, 3), keepdims=True)
    F *= frms / np.sqrt((F ** 2).mean())
    return F


def turbulence_velocity_2d(shape, k0=8.0, urms=0.03, seed=SEED_INIT):
    """Solenoidal 2D Gaussian random velocity, shape (ny, nx) -> (2, ny, nx).

    A random stream function psi whose velocity spectrum is
    E(k) ~ k^4 exp(-2 (k/k0)^2) (k in units of 2 pi / L; the shell of radius k
    has circumference ~ k, so |u_k|^2 ~ E(k) / k and |psi_k| = |u_k| / k);
    u = d psi / dy, v = -d psi / dx spectrally, scaled to per-component rms
    ``urms``.
    """
    rng = np.random.default_rng(seed)
    ny, nx = shape
    hat = np.fft.rfft2(rng.standard_normal((ny, nx)))
    KY, KX = np.meshgrid(np.fft.fftfreq(ny) * ny, np.fft.rfftfreq(nx) * nx, indexing="ij")
    k = np.sqrt(KX ** 2 + KY ** 2)
    ks = np.where(k == 0, 1.0, k)
    amp = np.where(k == 0, 0.0, np.sqrt(ks ** 4 * np.exp(-2.0 * (ks / k0) ** 2) / ks) / ks)
    # Nyquist modes have no consistent derivative on an even grid: leave them out
    amp[(np.abs(KY) == ny / 2) | (KX == nx / 2)] = 0.0
    psi = hat * amp
    u = np.stack([np.fft.irfft2(1j * KY * psi, s=(ny, nx)), np.fft.irfft2(-1j * KX * psi, s=(ny, nx))])
    u *= urms / np.sqrt((u ** 2).sum(axis=0).mean() / 2.0)
    return u


def kolmogorov_force_2d(shape, kf=4, amp=1e-5):
    """Kolmogorov forcing F = (amp sin(2 pi kf y / ny), 0), shape (ny, nx) -> (2, ny, nx)."""
    ny, nx = shape
    F = np.zeros((2, ny, nx))
    F[0] = amp * np.sin(2 * np.pi * kf * np.arange(ny) / ny)[:, None]
    return F


def random_populations(Q, ncells, w, amp=0.05, seed=SEED_INIT):
    """Populations w_i (1 + amp * N(0,1)) for per-cell tests (positive for small amp)."""
    rng = np.random.default_rng(seed)
    return w[:, None] * (1.0 + amp * rng.standard_normal((Q, ncells)))


def shell_spectrum(u):
    """Shell-summed kinetic energy spectrum E(k), k = 0 .. kmax (integer shells)."""
    shape = u.shape[1:]
    hat = np.fft.rfftn(u, axes=(1, 2, 3)) / np.prod(shape)
    KX, KY, KZ = _wavenumbers(shape)
    weight = np.where(KX == 0, 1.0, 2.0)
    weight = np.where((KX == shape[2] // 2) & (shape[2] % 2 == 0), 1.0, weight)
    e = 0.5 * (np.abs(hat) ** 2).sum(axis=0) * weight
    k = np.rint(np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)).astype(int)
    return np.bincount(k.ravel(), weights=e.ravel())
