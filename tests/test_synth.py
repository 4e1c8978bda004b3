"""The seeded input generators (CPU only): the structure each workload relies on."""
import numpy as np

import synth


def _div_spectral_3d(u):
    nz, ny, nx = u.shape[1:]
    kx = np.fft.fftfreq(nx)[None, None, :]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kz = np.fft.fftfreq(nz)[:, None, None]
    hat = [np.fft.fftn(u[d]) for d in range(3)]
    return np.abs(kx * hat[0] + ky * hat[1] + kz * hat[2]).max() / max(np.abs(h).max() for h in hat)


def test_turbulence_velocity_is_solenoidal_with_requested_rms_and_peak():
    u = synth.turbulence_velocity((32, 32, 32), k0=4.0, urms=0.03)
    assert abs(np.sqrt((u ** 2).sum(axis=0).mean() / 3) - 0.03) < 1e-12
    assert _div_spectral_3d(u) < 1e-3   # only the Nyquist planes carry a residual
    assert np.abs(u.mean(axis=(1, 2, 3))).max() < 1e-15
    E = synth.shell_spectrum(u)
    assert 2 <= int(np.argmax(E)) <= 5   # E(k) ~ k^4 exp(-2 (k/k0)^2) peaks at k = k0


def test_band_forcing_modes_and_rms():
    F = synth.band_forcing((16, 16, 16), kmin=1.0, kmax=2.0, frms=1e-4)
    assert abs(np.sqrt((F ** 2).sum(axis=0).mean()) - 1e-4) < 1e-16
    hat = np.fft.fftn(F, axes=(1, 2, 3))
    power = (np.abs(hat) ** 2).sum(axis=0)
    k = np.fft.fftfreq(16) * 16
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    kk = KX ** 2 + KY ** 2 + KZ ** 2
    inside = (kk >= 1) & (kk <= 4)
    assert power[~inside].max() < 1e-20 * power.max()
    assert _div_spectral_3d(F) < 1e-12


def test_turbulence_velocity_2d_is_solenoidal():
    u = synth.turbulence_velocity_2d((64, 128), k0=8.0, urms=0.03)
    assert u.shape == (2, 64, 128)
    assert abs(np.sqrt((u ** 2).sum(axis=0).mean() / 2) - 0.03) < 1e-12
    kx = np.fft.fftfreq(128) * 128
    ky = np.fft.fftfreq(64) * 64
    div = np.fft.ifft2(1j * kx[None, :] * np.fft.fft2(u[0]) + 1j * ky[:, None] * np.fft.fft2(u[1])).real
    assert np.abs(div).max() < 1e-12


def test_kolmogorov_force_2d():
    F = synth.kolmogorov_force_2d((64, 32), kf=4, amp=1e-5)
    assert F.shape == (2, 64, 32) and np.all(F[1] == 0)
    assert abs(F[0].max() - 1e-5) < 1e-18 and abs(F[0].sum()) < 1e-15
    assert np.array_equal(F[0][:, 0], F[0][:, 17])


def test_generators_are_seeded():
    a = synth.turbulence_velocity((8, 8, 8))
    b = synth.turbulence_velocity((8, 8, 8))
    assert np.array_equal(a, b)
    assert np.array_equal(synth.turbulence_velocity_2d((16, 16)), synth.turbulence_velocity_2d((16, 16)))
