"""Seeded synthetic measures on regular grids.

This module only draws inputs: nonnegative float64 arrays of shape [N]^d
(C-contiguous), each normalised to total mass 1.  It contains none of the
bound computations, so both the CPU oracle and the GPU library's callers
(tests, benchmark) may import it.

Families follow the workloads the paper evaluates on (2D images of the
DOTmark kind, 3D density maps of the cryo-EM kind), replaced here by seeded
stand-ins because the datasets themselves are not available:

* ``blobs``      - sum of isotropic Gaussian blobs plus a uniform floor
* ``white_noise``- i.i.d. U(0,1) pixels
* ``grf``        - exponentiated Gaussian random field, squared-exponential
                   covariance with a given length scale (periodic, via FFT)
* ``cauchy``     - bivariate (or trivariate) Cauchy density
* ``shapes``     - 1..4 filled random ellipses / ellipsoids on a zero
                   background (exercises zero-mass pixels and blocks)
* ``gmm``        - Gaussian mixture with Dirichlet(1) weights

Every generator takes a ``numpy.random.Generator``; ``rng(seed)`` builds the
PCG64 generator used everywhere (seed = 1000 * config + image index).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

FAMILIES = ("white_noise", "grf", "cauchy", "shapes", "gmm")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _normalise(m: np.ndarray) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.float64)
    s = m.sum()
    if not (s > 0):
        raise ValueError("generated measure has no mass")
    return m / s


def _grid(N: int, d: int) -> np.ndarray:
    """Integer pixel coordinates, shape [N]^d x d (float64)."""
    axes = np.meshgrid(*([np.arange(N, dtype=np.float64)] * d), indexing="ij")
    return np.stack(axes, axis=-1)


def blobs(N: int, d: int, g: np.random.Generator, n_blobs: int = 3,
          sigma=(2.0, 6.0), floor: float = 1e-3) -> np.ndarray:
    """Sum of ``n_blobs`` unit-mass isotropic Gaussians plus a ``floor`` of total mass."""
    X = _grid(N, d)
    acc = np.zeros((N,) * d)
    for _ in range(n_blobs):
        c = g.uniform(0, N, size=d)
        s = g.uniform(*sigma)
        b = np.exp(-((X - c) ** 2).sum(-1) / (2 * s * s))
        acc += b / b.sum()
    m = (1.0 - floor) * acc / n_blobs + floor / N ** d
    return _normalise(m)


def white_noise(N: int, d: int, g: np.random.Generator) -> np.ndarray:
    return _normalise(g.uniform(0.0, 1.0, size=(N,) * d))


def grf(N: int, d: int, g: np.random.Generator, ell: float = 4.0) -> np.ndarray:
    """exp(z) for a unit-variance periodic field z with covariance exp(-r^2 / (2 ell^2))."""
    z = g.standard_normal((N,) * d)
    freqs = np.meshgrid(*([np.fft.fftfreq(N)] * d), indexing="ij")
    f2 = sum(f * f for f in freqs)
    amp = np.exp(-(math.pi ** 2) * ell * ell * f2)  # sqrt of the SE spectral density
    field = np.real(np.fft.ifftn(np.fft.fftn(z) * amp))
    field = (field - field.mean()) / field.std()
    return _normalise(np.exp(field))


def cauchy(N: int, d: int, g: np.random.Generator) -> np.ndarray:
    X = _grid(N, d)
    c = g.uniform(N / 4, 3 * N / 4, size=d)
    gam = g.uniform(N / 16, N / 8)
    r2 = ((X - c) ** 2).sum(-1)
    return _normalise((1.0 + r2 / (gam * gam)) ** (-1.5))


def _random_rotation(d: int, g: np.random.Generator) -> np.ndarray:
    if d == 2:
        th = g.uniform(0, math.pi)
        return np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    q, r = np.linalg.qr(g.standard_normal((d, d)))
    return q * np.sign(np.diag(r))


def shapes(N: int, d: int, g: np.random.Generator) -> np.ndarray:
    X = _grid(N, d)
    m = np.zeros((N,) * d)
    for _ in range(int(g.integers(1, 5))):
        c = g.uniform(N / 4, 3 * N / 4, size=d)
        semi = g.uniform(N / 16, N / 4, size=d)
        Rm = _random_rotation(d, g)
        loc = (X - c) @ Rm
        m[((loc / semi) ** 2).sum(-1) <= 1.0] = 1.0
    if m.sum() == 0:  # a shape always covers its centre pixel at these sizes
        m[(N // 2,) * d] = 1.0
    return _normalise(m)


def gmm(N: int, d: int, g: np.random.Generator) -> np.ndarray:
    X = _grid(N, d)
    k = int(g.integers(2, 6))
    w = g.dirichlet(np.ones(k))
    m = np.zeros((N,) * d)
    for j in range(k):
        c = g.uniform(0, N, size=d)
        s = g.uniform(2.0, max(2.0, N / 8))
        b = np.exp(-((X - c) ** 2).sum(-1) / (2 * s * s))
        m += w[j] * b / b.sum()
    return _normalise(m)


def family(name: str, N: int, d: int, g: np.random.Generator) -> np.ndarray:
    return {"white_noise": white_noise, "grf": grf, "cauchy": cauchy,
            "shapes": shapes, "gmm": gmm, "blobs": blobs}[name](N, d, g)


# --------------------------------------------------------------------------
# Pairs with known Wasserstein distance (closed forms that hold at any size)
# --------------------------------------------------------------------------

def translated_pair(N: int, d: int, shift, g: np.random.Generator):
    """(mu, nu) with nu = mu translated by the integer vector ``shift``.

    mu is a Gaussian mixture masked to a box that keeps the translate inside
    the grid, so nu is an exact translate (no wrap-around)."""
    shift = np.asarray(shift, dtype=np.int64)
    m = gmm(N, d, g)
    mask = np.ones((N,) * d, dtype=bool)
    for ax in range(d):
        lo, hi = max(0, -int(shift[ax])), N - max(0, int(shift[ax]))
        sl = [slice(None)] * d
        idx = np.arange(N)
        keep = (idx >= lo) & (idx < hi)
        shape = [1] * d
        shape[ax] = N
        mask &= keep.reshape(shape)
    mu = _normalise(np.where(mask, m, 0.0))
    nu = np.roll(mu, tuple(int(s) for s in shift), axis=tuple(range(d)))
    return mu, np.ascontiguousarray(nu)


def axis_constant_pair(N: int, d: int, g: np.random.Generator):
    """Measures that vary only along the last axis (profiles drawn at random)."""
    def profile():
        x = np.arange(N, dtype=np.float64)
        p = np.zeros(N)
        for _ in range(int(g.integers(1, 4))):
            c, s = g.uniform(0, N), g.uniform(1.0, max(1.5, N / 6))
            p += g.uniform(0.2, 1.0) * np.exp(-(x - c) ** 2 / (2 * s * s))
        p += 1e-3 * p.max()
        return p / p.sum()
    shape = [1] * (d - 1) + [N]
    mu = np.broadcast_to(profile().reshape(shape), (N,) * d) / N ** (d - 1)
    nu = np.broadcast_to(profile().reshape(shape), (N,) * d) / N ** (d - 1)
    return _normalise(mu), _normalise(nu)


def dirac_pair(N: int, d: int, g: np.random.Generator):
    mu = np.zeros((N,) * d)
    nu = np.zeros((N,) * d)
    x = tuple(int(v) for v in g.integers(0, N, size=d))
    y = tuple(int(v) for v in g.integers(0, N, size=d))
    mu[x] = 1.0
    nu[y] = 1.0
    return mu, nu, np.asarray(x), np.asarray(y)


# --------------------------------------------------------------------------
# The five workload configurations (stand-ins for the paper's data sets)
# --------------------------------------------------------------------------

def config1_pair():
    """One pair of 32x32 measures, three Gaussian blobs plus a 1e-3 floor; k=4, p=2."""
    mu = blobs(32, 2, rng(1000 + 0))
    nu = blobs(32, 2, rng(1000 + 1))
    return mu, nu


def config2_images():
    """Ten 64x64 images, two per family."""
    imgs = []
    for i in range(10):
        fam = FAMILIES[i // 2]
        imgs.append((fam, family(fam, 64, 2, rng(2000 + i))))
    return imgs


def config2_pairs():
    imgs = config2_images()
    return [(i, j, imgs[i][1], imgs[j][1]) for i, j in itertools.combinations(range(10), 2)]


def config3_pair(N: int, fam: str, idx: int = 0):
    """A single pair at N in {256, 512} from the GRF or Cauchy family."""
    base = 3000 + (0 if fam == "grf" else 100) + (0 if N == 256 else 10) + 2 * idx
    return family(fam, N, 2, rng(base)), family(fam, N, 2, rng(base + 1))


def config4_pairs(n_pairs: int = 64, N: int = 64):
    out = []
    for i in range(n_pairs):
        out.append((gmm(N, 2, rng(4000 + 2 * i)), gmm(N, 2, rng(4000 + 2 * i + 1))))
    return out


CONFIG5_GRIDS = ((32, 2), (64, 2), (128, 2), (16, 3), (32, 3))


def config5_jobs(n_jobs: int = 128):
    """Mixed jobs: (N, d, k, p, mu, nu) round-robin over grid x k x p, shuffled."""
    combos = [(N, d, k, p) for (N, d) in CONFIG5_GRIDS for k in (2, 4, 8) for p in (1, 2)]
    g = rng(5000)
    order = list(range(n_jobs))
    g.shuffle(order)
    jobs = []
    for j in order:
        N, d, k, p = combos[j % len(combos)]
        mu = grf(N, d, rng(5000 + 2 * j + 1), ell=4.0)
        nu = grf(N, d, rng(5000 + 2 * j + 2), ell=4.0)
        jobs.append((N, d, k, p, mu, nu))
    return jobs


# --------------------------------------------------------------------------
# Kernels for upscaling a coarse coupling (inputs, not part of the method)
# --------------------------------------------------------------------------

def random_plan_kernel(k: int, d: int, g: np.random.Generator, zero_frac: float = 0.0) -> np.ndarray:
    """A random nonnegative (k^d, k^d) kernel matrix with total 1: i.i.d.
    U(0.05, 1) entries, a fraction ``zero_frac`` of them set to 0 (every row
    and column keeps at least one positive entry)."""
    m = k ** d
    w = g.uniform(0.05, 1.0, size=(m, m))
    if zero_frac > 0:
        drop = g.uniform(size=(m, m)) < zero_frac
        keep = np.zeros((m, m), dtype=bool)
        keep[np.arange(m), g.permutation(m)] = True
        w = np.where(drop & ~keep, 0.0, w)
    return np.ascontiguousarray(w / w.sum())
