"""Plain FP64 oracle of the membrane force and the trapezoid weights.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The membrane applies the elastic force of eq. (elastic_force),
    f = -kappa_b X_ssss + (sigma X_s)_s,
to the fluid; arclength derivatives are spectral (Section 2.2.1): with the N
points at alpha_k = 2 pi k / N, d/ds = (1/|X_alpha|) d/dalpha, and d/dalpha
multiplies Fourier mode k by i k.  For even N the Nyquist mode N/2 has no
well-defined odd derivative on the grid; it is set to zero (the derivative of
the real, symmetric band-limited interpolant).  The trapezoid weight of point
k is w_k = |X_alpha(alpha_k)| 2 pi / N (the ds of eq. (single_layer)).
"""
import numpy as np


def spectral_derivative(v):
    """d/dalpha of periodic samples v[..., N] via the FFT."""
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[-1]
    k = np.fft.fftfreq(n, 1.0 / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return np.real(np.fft.ifft(1j * k * np.fft.fft(v, axis=-1), axis=-1))


def vesicle_force(x, sigma, kappa_b):
    """Force density and weights of one vesicle: x (2, N), sigma (N,) -> f (2, N), w (N,)."""
    n = x.shape[1]
    xa = spectral_derivative(x)
    J = np.sqrt(xa[0] ** 2 + xa[1] ** 2)
    xs = xa / J
    xss = spectral_derivative(xs) / J
    xsss = spectral_derivative(xss) / J
    xssss = spectral_derivative(xsss) / J
    tension = spectral_derivative(sigma * xs) / J
    return -kappa_b * xssss + tension, J * (2.0 * np.pi / n)


def elastic_force(X, sigma, kappa_b, offsets):
    """All vesicles of a suspension: X (2, P), sigma (P,) or None -> f (2, P), w (P,)."""
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[1]
    sigma = np.zeros(P) if sigma is None else np.asarray(sigma, dtype=np.float64)
    f = np.empty_like(X)
    w = np.empty(P)
    for v in range(len(offsets) - 1):
        a, b = int(offsets[v]), int(offsets[v + 1])
        if b > a:
            f[:, a:b], w[a:b] = vesicle_force(X[:, a:b], sigma[a:b], kappa_b)
    return f, w
