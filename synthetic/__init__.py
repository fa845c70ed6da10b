"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds random-number generation and the layout of the random
signals only; it contains none of the transform arithmetic.  Both the CPU
oracle and the GPU path receive arrays produced here.

Generator: SplitMix64 (Steele, Lea & Flood 2014) evaluated counter-style,
z_i = mix(seed_key + (i + 1) * 0x9E3779B97F4A7C15), followed by the
Box-Muller transform for standard normal deviates.

Signals follow the paper's validation protocol (Section 4.4, "Numerical
Validation"): a random band-limited signal given by its harmonic
coefficients.  Coefficients are complex Gaussian with E|f_lm|^2 = C_l,
C_l = 1/(l+1)^2 on the sphere and 1/((l+1)^2 (p+1)^2) on the ball; the
m = 0 coefficient is real N(0, C_l) and f_{l,-m} = (-1)^m conj(f_lm) so that
the pixel-space signal is real.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_key(seed: int, index: int = 0) -> int:
    """Key of the random stream for (seed k, map b): seed k, map b in a batch."""
    return ((int(seed) & 0xFFFFFFFF) << 32) | (int(index) & 0xFFFFFFFF)


def uniforms(key: int, n: int) -> np.ndarray:
    """n uniform deviates in [0, 1) from SplitMix64 at counters 1..n of `key`."""
    with np.errstate(over="ignore"):
        base = _mix(np.uint64(key & 0xFFFFFFFFFFFFFFFF) + _GOLDEN)
        ctr = np.arange(1, n + 1, dtype=np.uint64) * _GOLDEN
        z = _mix(base + ctr)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normals(key: int, n: int) -> np.ndarray:
    """n standard normal deviates (Box-Muller on pairs of uniforms)."""
    m = (n + 1) // 2
    u = uniforms(key, 2 * m)
    r = np.sqrt(-2.0 * np.log1p(-u[0::2]))
    t = 2.0 * np.pi * u[1::2]
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(t)
    z[1::2] = r * np.sin(t)
    return z[:n]


def sphere_flm(L: int, key: int, spectrum=None) -> np.ndarray:
    """Harmonic coefficients of a real band-limited Gaussian field on S^2.

    Returns a complex array [L, 2L-1] in the paper's "lm" layout (index
    m + L - 1), zero where |m| > l.  spectrum(l) defaults to 1/(l+1)^2.
    """
    if spectrum is None:
        spectrum = lambda l: 1.0 / (l + 1.0) ** 2  # noqa: E731
    flm = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    z = normals(key, 2 * L * L)
    k = 0
    for l in range(L):
        c = spectrum(l)
        flm[l, L - 1] = np.sqrt(c) * z[k]
        k += 2
        for m in range(1, l + 1):
            v = np.sqrt(c / 2.0) * (z[k] + 1j * z[k + 1])
            k += 2
            flm[l, L - 1 + m] = v
            flm[l, L - 1 - m] = (-1) ** m * np.conj(v)
    return flm


def spin_flm(L: int, s: int, key: int, spectrum=None) -> np.ndarray:
    """Harmonic coefficients of a complex band-limited spin-s Gaussian field on S^2:
    [L, 2L-1] ("lm" layout, index m + L - 1), every (l, m) with l >= max(|s|, |m|)
    independent complex normal with variance spectrum(l) (default 1/(l+1)^2), zero
    elsewhere."""
    if spectrum is None:
        spectrum = lambda l: 1.0 / (l + 1.0) ** 2  # noqa: E731
    flm = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    z = normals(key, 2 * L * (2 * L - 1))
    k = 0
    for l in range(abs(s), L):
        c = np.sqrt(spectrum(l) / 2.0)
        for m in range(-l, l + 1):
            flm[l, L - 1 + m] = c * (z[k] + 1j * z[k + 1])
            k += 2
    return flm


def ball_flmp(L: int, P: int, key: int) -> np.ndarray:
    """Spherical-Laguerre coefficients [P, L, 2L-1] of a real Gaussian field
    on the ball with E|f_lmp|^2 = 1/((l+1)^2 (p+1)^2)."""
    out = np.zeros((P, L, 2 * L - 1), dtype=np.complex128)
    for p in range(P):
        out[p] = sphere_flm(L, (key * 1000003 + p + 1) & 0xFFFFFFFFFFFFFFFF,
                            spectrum=lambda l, p=p: 1.0 / ((l + 1.0) ** 2 * (p + 1.0) ** 2))
    return out


def so3_flmn(L: int, N: int, key: int) -> np.ndarray:
    """Wigner coefficients [2N-1, L, 2L-1] ("nlm": index n+N-1, l, m+L-1) of a real
    band-limited Gaussian function on SO(3): complex Gaussian with variance 1/(l+1)^2 for
    |m|, |n| <= l, with f^l_{-m,-n} = (-1)^(m+n) conj(f^l_mn) (so the function is real;
    the (0, 0) coefficient real)."""
    out = np.zeros((2 * N - 1, L, 2 * L - 1), dtype=np.complex128)
    z = normals(key, 2 * (2 * N - 1) * L * (2 * L - 1))
    k = 0
    for l in range(L):
        s = 1.0 / (l + 1.0)
        for n in range(-min(N - 1, l), min(N - 1, l) + 1):
            for m in range(-l, l + 1):
                # one representative of each (m, n), (-m, -n) pair: n > 0, or n == 0 and m >= 0
                if n < 0 or (n == 0 and m < 0):
                    continue
                if n == 0 and m == 0:
                    v = s * z[k]
                else:
                    v = s * np.sqrt(0.5) * (z[k] + 1j * z[k + 1])
                k += 2
                out[n + N - 1, l, m + L - 1] = v
                out[-n + N - 1, l, -m + L - 1] = (-1) ** ((m + n) % 2) * np.conj(v)
    return out


def wl_flmnp(L: int, N: int, P: int, key: int) -> np.ndarray:
    """Wigner-Laguerre coefficients [P, 2N-1, L, 2L-1] of a real function on R+ x SO(3):
    per p the SO(3) coefficients of so3_flmn, scaled by 1/(p+1)."""
    return np.stack([so3_flmn(L, N, (key * 1000003 + p + 1) & 0xFFFFFFFFFFFFFFFF) / (p + 1.0)
                     for p in range(P)])
