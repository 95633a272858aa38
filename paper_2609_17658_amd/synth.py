"""Seeded synthetic inputs shaped like the paper's cosmological boxes.

This module only draws particle sets; it holds none of the tree-force
arithmetic, and both the HIP path's tests/benchmark and the CPU oracle's
tests take their inputs from it.  All generators use
``numpy.random.default_rng(seed)`` and return positions wrapped into the
periodic box ``[0, box)^3`` and equal masses ``1/N`` (unit total mass, G = 1).

Workloads (every parameter set is scale-free in N: eps = 1/(40 N^(1/3)),
r_s = 1.25/(2 N^(1/3)), r_cut = 4.5 r_s):
  * ``mixture32k``   N = 32^3: half uniform, half in 8 Plummer spheres
                     (a = 0.01), theta = 0.5, leaf_max = 8.
  * ``mixture2m``    N = 128^3: half uniform, half in 64 Plummer spheres
                     (a = 0.005), theta in {0.3, 0.5, 0.7}.
  * ``zeldovich256`` N = 256^3 grid displaced by a Gaussian random field with
                     P(k) ~ k^-2 cut at the Nyquist wavenumber, rms 3-D
                     displacement 0.3 grid cells.
  * ``batch512``     512 independent boxes, N_b log-uniform in [1e3, 2e5],
                     8 spheres (a = 0.01) + uniform, box seed 1000 + b.
  * serving stream   Poisson arrivals, N log-uniform in [1e4, 4e6],
                     Zel'dovich or mixture by a seeded coin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class ForceParams:
    """Physical/numerical parameters of one short-range force evaluation."""
    G: float = 1.0
    eps: float = 0.0
    r_s: float = 0.0
    r_cut: float = 0.0          # 0 => 4.5 r_s
    theta: float = 0.5
    periodic: int = 1
    leaf_max: int = 8

    def as_dict(self):
        return asdict(self)


def scale_free_params(n: int, theta: float = 0.5, leaf_max: int = 8) -> ForceParams:
    """eps = 1/(40 n^(1/3)), r_s = 1.25/(2 n^(1/3)), r_cut = 4.5 r_s."""
    side = n ** (1.0 / 3.0)
    r_s = 1.25 / (2.0 * side)
    return ForceParams(G=1.0, eps=1.0 / (40.0 * side), r_s=r_s, r_cut=4.5 * r_s,
                       theta=theta, periodic=1, leaf_max=leaf_max)


def wrap(x: np.ndarray, box: float = 1.0) -> np.ndarray:
    """Map coordinates into [0, box); a value that rounds to box is the
    periodic image 0."""
    x = np.mod(x, box)
    x[x >= box] = 0.0
    return x


def plummer_offsets(rng, n: int, a: float) -> np.ndarray:
    """n offsets from a Plummer sphere of scale length a: radius from the
    inverted cumulative mass r = a (X^(-2/3) - 1)^(-1/2), X ~ U[0,1),
    isotropic direction."""
    X = rng.random(n)
    with np.errstate(divide="ignore"):
        r = a / np.sqrt(np.power(X, -2.0 / 3.0) - 1.0)
    r = np.where(X > 0, r, 0.0)
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([r * s * np.cos(phi), r * s * np.sin(phi), r * mu], axis=1)


def mixture(n_uniform: int, n_spheres: int, n_per_sphere, a: float, seed: int,
            box: float = 1.0) -> np.ndarray:
    """Uniform background plus Plummer spheres at seed-placed centres,
    wrapped periodically.  ``n_per_sphere`` is an int or a list of ints."""
    rng = np.random.default_rng(seed)
    parts = [rng.random((n_uniform, 3)) * box]
    centres = rng.random((n_spheres, 3)) * box
    if np.isscalar(n_per_sphere):
        n_per_sphere = [int(n_per_sphere)] * n_spheres
    for c, k in zip(centres, n_per_sphere):
        parts.append(c[None, :] + plummer_offsets(rng, k, a))
    return wrap(np.concatenate(parts, axis=0), box)


def plummer_sphere(n: int, a: float, seed: int, centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """An isolated (not wrapped) Plummer sphere."""
    rng = np.random.default_rng(seed)
    return np.asarray(centre)[None, :] + plummer_offsets(rng, n, a)


def zeldovich(n_grid: int, seed: int, rms_cells: float = 0.3, box: float = 1.0) -> np.ndarray:
    """Grid of n_grid^3 points displaced by psi = grad-potential field with
    psi_k = i k delta_k / k^2, delta_k Gaussian with <|delta_k|^2> ~ k^-2,
    zero mean, cut at |k| <= pi n / box; rms |psi| = rms_cells grid cells."""
    n = n_grid
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    dk = np.fft.rfftn(white)
    del white
    k1 = 2.0 * math.pi * np.fft.fftfreq(n, d=box / n)
    kz = 2.0 * math.pi * np.fft.rfftfreq(n, d=box / n)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kzz = kz[None, None, :]
    k2 = kx * kx + ky * ky + kzz * kzz
    knyq = math.pi * n / box
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where((k2 > 0) & (k2 <= knyq * knyq), 1.0 / np.sqrt(k2), 0.0)
        dk *= amp
        dk /= np.where(k2 > 0, k2, 1.0)
    del amp
    q1 = (np.arange(n) + 0.5) * box / n
    psi = np.empty((n, n, n, 3))
    psi[..., 0] = np.fft.irfftn(1j * kx * dk, s=(n, n, n), axes=(0, 1, 2))
    psi[..., 1] = np.fft.irfftn(1j * ky * dk, s=(n, n, n), axes=(0, 1, 2))
    psi[..., 2] = np.fft.irfftn(1j * kzz * dk, s=(n, n, n), axes=(0, 1, 2))
    del dk
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=-1))))
    psi *= (rms_cells * box / n) / rms
    q = np.stack(np.meshgrid(q1, q1, q1, indexing="ij"), axis=-1)
    pos = (q + psi).reshape(-1, 3)
    return wrap(pos, box)


def equal_masses(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n)


@dataclass
class Workload:
    name: str
    pos: np.ndarray
    mass: np.ndarray
    box: float
    params: ForceParams
    info: dict = field(default_factory=dict)


def mixture32k(seed: int = 1) -> Workload:
    n = 32 ** 3
    pos = mixture(n // 2, 8, (n - n // 2) // 8, 0.01, seed)
    p = scale_free_params(n, theta=0.5, leaf_max=8)
    return Workload("mixture32k", pos, equal_masses(n), 1.0, p,
                    {"N": n, "spheres": 8, "a": 0.01, "seed": seed})


def mixture2m(seed: int = 2, theta: float = 0.5) -> Workload:
    n = 128 ** 3
    pos = mixture(n // 2, 64, (n - n // 2) // 64, 0.005, seed)
    p = scale_free_params(n, theta=theta, leaf_max=8)
    return Workload("mixture2m", pos, equal_masses(n), 1.0, p,
                    {"N": n, "spheres": 64, "a": 0.005, "seed": seed, "theta": theta})


def zeldovich256(seed: int = 3, n_grid: int = 256) -> Workload:
    n = n_grid ** 3
    pos = zeldovich(n_grid, seed)
    p = scale_free_params(n, theta=0.5, leaf_max=8)
    return Workload("zeldovich%d" % n_grid, pos, equal_masses(n), 1.0, p,
                    {"N": n, "grid": n_grid, "seed": seed, "rms_cells": 0.3})


def box_sizes(n_boxes: int, seed: int, nmin: float, nmax: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_boxes))).astype(np.int64)


def mixture_box(n: int, seed: int, n_spheres: int = 8, a: float = 0.01) -> np.ndarray:
    """Half uniform, the rest spread over n_spheres Plummer spheres."""
    nu = n // 2
    rest = n - nu
    per = [rest // n_spheres + (1 if s < rest % n_spheres else 0) for s in range(n_spheres)]
    return mixture(nu, n_spheres, per, a, seed)


def batch512(n_boxes: int = 512, nmin: float = 1e3, nmax: float = 2e5, seed: int = 4,
             theta: float = 0.5, leaf_max: int = 8):
    """Independent periodic boxes of uneven N; box b uses seed 1000 + b."""
    sizes = box_sizes(n_boxes, seed, nmin, nmax)
    out = []
    for b, n in enumerate(sizes):
        n = int(n)
        pos = mixture_box(n, 1000 + b)
        out.append(Workload("box%d" % b, pos, equal_masses(n), 1.0,
                            scale_free_params(n, theta=theta, leaf_max=leaf_max),
                            {"N": n, "seed": 1000 + b}))
    return out


@dataclass
class Request:
    k: int
    t_arrive: float
    n: int
    kind: str       # "zeldovich" or "mixture"
    seed: int

    def workload(self, theta: float = 0.5) -> Workload:
        if self.kind == "zeldovich":
            g = max(2, int(round(self.n ** (1.0 / 3.0))))
            pos = zeldovich(g, self.seed)
        else:
            pos = mixture_box(self.n, self.seed)
        n = pos.shape[0]
        return Workload("req%d" % self.k, pos, equal_masses(n), 1.0,
                        scale_free_params(n, theta=theta), {"N": n, "seed": self.seed})


def request_stream(n_requests: int, rate_per_s: float, seed: int = 5, nmin: float = 1e4,
                   nmax: float = 4e6):
    """Poisson arrivals (exponential gaps at rate_per_s), N log-uniform,
    kind by a seeded coin; request k draws its particles with seed 100000+k."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_requests))).astype(np.int64)
    kinds = np.where(rng.random(n_requests) < 0.5, "zeldovich", "mixture")
    out = []
    for k in range(n_requests):
        n = int(ns[k])
        if kinds[k] == "zeldovich":
            g = max(2, int(round(n ** (1.0 / 3.0))))
            n = g ** 3
        out.append(Request(k, float(t[k]), n, str(kinds[k]), 100000 + k))
    return out


WORKLOADS = {
    "mixture32k": mixture32k,
    "mixture2m": mixture2m,
    "zeldovich256": zeldovich256,
}
