"""Measurement noise: i.i.d. Gaussian with sigma = rel * max(y_clean)."""
import numpy as np


def add_noise(y_clean: np.ndarray, rel: float, seed) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sigma = rel * float(np.max(y_clean)) if y_clean.size else 0.0
    return y_clean + rng.normal(0.0, sigma, size=y_clean.shape)
