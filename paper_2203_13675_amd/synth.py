"""Seeded synthetic wrapped-phase maps.

This module only *makes inputs*: a smooth phase field, additive Gaussian
noise, the wrapped measurement and an optional quality mask.  It holds none
of the unwrapping method's arithmetic (no wrapped differences, weights,
stencil or solver), so both the CPU oracle and the HIP path can consume the
same arrays without sharing code.

The wrapped measurement follows the signal model of Section 1 (a complex
signal whose argument is the phase): psi = arg(exp(i*phi)), folded into
(-pi, pi] as Eq. (1) requires.

Workloads (all seeded with numpy's default_rng):

* ``peaks_map``     -- MATLAB-style ``peaks`` surface on [-3, 3]^2, scaled.
* ``gaussians_map`` -- sum of random 2-D Gaussians.
* ``ramp_peaks_map``-- scaled peaks plus a linear ramp along x.
* ``batch_maps``    -- many uneven-sized random-Gaussian maps.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "peaks",
    "wrap_measurement",
    "peaks_map",
    "gaussians_map",
    "ramp_peaks_map",
    "hole_mask",
    "batch_sizes",
    "batch_maps",
    "batch_map",
    "random_phi0",
    "WORKLOADS",
    "workload",
]

BATCH_SIDES = (128, 256, 384, 512, 768, 1024)


def peaks(M: int, N: int) -> np.ndarray:
    """MATLAB ``peaks`` on x = linspace(-3,3,N) (columns), y = linspace(-3,3,M) (rows)."""
    x = np.linspace(-3.0, 3.0, N)
    y = np.linspace(-3.0, 3.0, M)
    X, Y = np.meshgrid(x, y)
    return (3.0 * (1.0 - X) ** 2 * np.exp(-X ** 2 - (Y + 1.0) ** 2)
            - 10.0 * (X / 5.0 - X ** 3 - Y ** 5) * np.exp(-X ** 2 - Y ** 2)
            - np.exp(-(X + 1.0) ** 2 - Y ** 2) / 3.0)


def wrap_measurement(phi: np.ndarray) -> np.ndarray:
    """Wrapped measurement arg(exp(i*phi)) in (-pi, pi] (signal model, Section 1)."""
    psi = np.angle(np.exp(1j * np.asarray(phi, dtype=np.float64)))
    psi[psi <= -np.pi] += 2.0 * np.pi  # arg() may return -pi; the range is half-open
    return np.ascontiguousarray(psi, dtype=np.float64)


def _noisy(phi: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    if sigma > 0:
        phi = phi + rng.normal(0.0, sigma, size=phi.shape)
    return phi


def peaks_map(M: int, N: int, *, scale: float | None = None, amplitude: float | None = None,
              sigma: float = 0.0, seed: int = 0):
    """Peaks surface: either multiplied by ``scale`` or scaled so max|phi| = ``amplitude``.

    Returns (psi, phi_true) with phi_true noise-free.
    """
    rng = np.random.default_rng(seed)
    p = peaks(M, N)
    if amplitude is not None:
        p = p * (amplitude / np.abs(p).max())
    elif scale is not None:
        p = p * scale
    phi = _noisy(p, sigma, rng)
    return wrap_measurement(phi), p


def gaussians_map(M: int, N: int, *, n_gauss: int = 20, amp=(5.0, 40.0), width=(50.0, 400.0),
                  sigma: float = 0.0, seed: int = 0):
    """Sum of ``n_gauss`` 2-D Gaussians, amplitude ~ U[amp], std ~ U[width] pixels,
    centres uniform over the map. Returns (psi, phi_true)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(amp[0], amp[1], n_gauss)
    S = rng.uniform(width[0], width[1], n_gauss)
    cy = rng.uniform(0, M, n_gauss)
    cx = rng.uniform(0, N, n_gauss)
    ii = np.arange(M, dtype=np.float64)[:, None]
    jj = np.arange(N, dtype=np.float64)[None, :]
    phi = np.zeros((M, N))
    for a, s, y0, x0 in zip(A, S, cy, cx):
        phi += a * np.exp(-((ii - y0) ** 2 + (jj - x0) ** 2) / (2.0 * s * s))
    noisy = _noisy(phi, sigma, rng)
    return wrap_measurement(noisy), phi


def ramp_peaks_map(M: int, N: int, *, amplitude: float = 60.0, ramp: float = 120.0,
                   sigma: float = 0.0, seed: int = 0):
    """Peaks scaled to max|.| = amplitude plus a linear ramp 0 -> ``ramp`` rad along x."""
    rng = np.random.default_rng(seed)
    p = peaks(M, N)
    p = p * (amplitude / np.abs(p).max()) + np.linspace(0.0, ramp, N)[None, :]
    phi = _noisy(p, sigma, rng)
    return wrap_measurement(phi), p


def hole_mask(M: int, N: int, frac: float = 0.10, seed: int = 0, margin: int = 1) -> np.ndarray:
    """Quality mask of ones with one square zero-quality hole covering ~``frac`` of the pixels,
    placed at a seeded position at least ``margin`` pixels from the border."""
    rng = np.random.default_rng(seed)
    side_y = int(round(np.sqrt(frac * M * N * M / N)))
    side_x = int(round(np.sqrt(frac * M * N * N / M)))
    side_y = min(side_y, M - 2 * margin)
    side_x = min(side_x, N - 2 * margin)
    y0 = int(rng.integers(margin, M - margin - side_y + 1))
    x0 = int(rng.integers(margin, N - margin - side_x + 1))
    m = np.ones((M, N), dtype=np.float32)
    m[y0:y0 + side_y, x0:x0 + side_x] = 0.0
    return m


def batch_sizes(n_maps: int = 256, seed: int = 3000):
    """Map shapes for the uneven batch: M and N drawn independently from BATCH_SIDES."""
    rng = np.random.default_rng(seed)
    Ms = rng.choice(BATCH_SIDES, n_maps)
    Ns = rng.choice(BATCH_SIDES, n_maps)
    return [(int(m), int(n)) for m, n in zip(Ms, Ns)]


def batch_maps(n_maps: int = 256, seed: int = 3000, sides=None):
    """Uneven batch of random-Gaussian maps with noise sigma ~ U[0.1, 0.8] rad.

    Returns a list of (psi, phi_true). ``sides`` overrides the drawn shapes.
    """
    shapes = sides if sides is not None else batch_sizes(n_maps, seed)
    rng = np.random.default_rng(seed + 1)
    out = []
    for k, (M, N) in enumerate(shapes):
        sig = float(rng.uniform(0.1, 0.8))
        out.append(gaussians_map(M, N, sigma=sig, seed=seed + 10 + k))
    return out


def batch_map(k: int, n_maps: int = 256, seed: int = 3000):
    """Map k of ``batch_maps(n_maps, seed)`` alone (same shape, noise level and
    phase), without generating the others.  Returns (psi, phi_true)."""
    M, N = batch_sizes(n_maps, seed)[k]
    rng = np.random.default_rng(seed + 1)
    sig = float(rng.uniform(0.1, 0.8, k + 1)[k])
    return gaussians_map(M, N, sigma=sig, seed=seed + 10 + k)


def random_phi0(M: int, N: int, seed: int = 0) -> np.ndarray:
    """Seeded random initial phase U(-pi, pi) (the random start of Algorithm 1)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(M, N))


# Named workloads with the shapes, sizes and distributions used throughout the
# tests and the benchmark.
WORKLOADS = {
    "peaks64": dict(kind="peaks", M=64, N=64, scale=4.0, sigma=0.3, seed=0, p=0.0, outer=10),
    "peaks1024": dict(kind="peaks", M=1024, N=1024, amplitude=60.0, sigma=0.5, seed=1000, p=0.0, outer=10),
    "gauss2048_hole": dict(kind="gauss", M=2048, N=2048, sigma=0.8, seed=2000, hole=0.10, p=0.0, outer=10),
    "batch256": dict(kind="batch", n_maps=256, seed=3000, p=0.0, outer=10),
    "ramp4096": dict(kind="ramp", M=4096, N=4096, sigma=0.5, seed=4000, p=0.0, outer=10),
}


def workload(name: str, *, M: int | None = None, N: int | None = None):
    """Return (psi, mask_or_None, phi_true) for a named single-map workload.

    ``M``/``N`` override the size (same recipe at another resolution)."""
    w = dict(WORKLOADS[name])
    M = M or w["M"]
    N = N or w["N"]
    if w["kind"] == "peaks":
        psi, phi = peaks_map(M, N, scale=w.get("scale"), amplitude=w.get("amplitude"),
                             sigma=w["sigma"], seed=w["seed"])
        return psi, None, phi
    if w["kind"] == "gauss":
        psi, phi = gaussians_map(M, N, sigma=w["sigma"], seed=w["seed"])
        mask = hole_mask(M, N, w["hole"], seed=w["seed"] + 1) if w.get("hole") else None
        return psi, mask, phi
    if w["kind"] == "ramp":
        psi, phi = ramp_peaks_map(M, N, sigma=w["sigma"], seed=w["seed"])
        return psi, None, phi
    raise ValueError(name)
