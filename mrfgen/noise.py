"""Measurement noise n of eq. (1): circular complex Gaussian at a stated SNR."""
import numpy as np


def noise_sigma(clean_power, snr_db):
    """Per-sample complex variance sigma_n^2 = mean|b_clean|^2 * 10^(-SNR/10)."""
    return float(clean_power) * 10.0 ** (-float(snr_db) / 10.0)


def complex_noise(shape, sigma2, seed):
    """Complex64 noise with E|n|^2 = sigma2 (variance sigma2/2 per component)."""
    rng = np.random.default_rng(seed)
    s = np.sqrt(sigma2 / 2.0)
    return (rng.standard_normal(shape) * s + 1j * rng.standard_normal(shape) * s).astype(np.complex64)
