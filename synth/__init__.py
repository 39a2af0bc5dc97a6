"""Seeded synthetic inputs for the lattice Dyson problem.

This module only draws and shapes inputs: lattice geometry, the trap potential
V_i, the Matsubara grid and a model self-energy Sigma_i(i w_k).  It holds none
of the arithmetic of the method or of the oracle; both the CPU oracle and the
GPU library receive the very same arrays from here.

Input recipe (the paper's Falicov-Kimball self-energies are not published, so a
causal model stands in for them):

* open boundaries, real nearest-neighbour hopping t (entries of H are t, eq. (1)),
* trap V_i = v_c * r_i^2 with r_i measured from the lattice centre (L_d-1)/2,
* fermionic Matsubara frequencies w_n = (2n+1) pi / beta,
* Sigma_i(i w) = a_i / (i w + b_i), a_i ~ U[0,1), b_i ~ U[-1/2,1/2) drawn once
  per site from numpy's PCG64 with the given seed (shared by all frequencies).
  With a_i >= 0 this Sigma is causal: Im Sigma_i(i w) <= 0 for w > 0, so
  Im H_ii >= w > 0 and H is non-singular.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One Dyson problem: lattice, physics parameters and frequency list."""

    dims: tuple            # (Lx,) / (Lx, Ly) / (Lx, Ly, Lz); x fastest
    t: float               # hopping (matrix entry on every nearest-neighbour bond)
    mu: float              # chemical potential
    vc: float              # trap coefficient, V_i = vc * r_i^2
    beta: float            # inverse temperature of the Matsubara grid
    freq_index: tuple      # Matsubara indices n, w_n = (2n+1) pi / beta
    seed: int              # seed of the per-site self-energy parameters
    name: str = ""

    @property
    def n_sites(self) -> int:
        return int(np.prod(self.dims))

    @property
    def n_freq(self) -> int:
        return len(self.freq_index)


def coords(dims: Sequence[int]) -> np.ndarray:
    """Site coordinates, shape (N, D), natural order with x fastest."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n)
    out = np.empty((n, len(dims)), dtype=np.int64)
    for a, L in enumerate(dims):
        out[:, a] = idx % L
        idx = idx // L
    return out


def trap(dims: Sequence[int], vc: float) -> np.ndarray:
    """V_i = vc * sum_d (x_d - (L_d-1)/2)^2, float64 [N]."""
    c = coords(dims).astype(np.float64)
    centre = (np.asarray(dims, dtype=np.float64) - 1.0) / 2.0
    return vc * np.sum((c - centre) ** 2, axis=1)


def matsubara(beta: float, freq_index: Sequence[int]) -> np.ndarray:
    n = np.asarray(freq_index, dtype=np.float64)
    return (2.0 * n + 1.0) * math.pi / beta


def sigma_params(n_sites: int, seed: int):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, n_sites)
    b = rng.uniform(-0.5, 0.5, n_sites)
    return a, b


def sigma_table(a: np.ndarray, b: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Sigma_i(i w_k) = a_i / (i w_k + b_i), complex128 [K, N]."""
    return a[None, :] / (1j * omega[:, None] + b[None, :])


def make_inputs(w: Workload):
    """Returns (V [N] f64, omega [K] f64, sigma [K,N] c128)."""
    V = trap(w.dims, w.vc)
    omega = matsubara(w.beta, w.freq_index)
    a, b = sigma_params(w.n_sites, w.seed)
    return V, omega, sigma_table(a, b, omega)


# The synthetic workloads: the small single-frequency case, the 256^2 x 64
# frequency throughput case, the 3-D case and a few small shapes used by tests.
SMALL_32 = Workload(dims=(32, 32), t=-1.0, mu=0.5, vc=0.01, beta=10.0,
                    freq_index=(0,), seed=1, name="square 32x32, K=1")
SQUARE_256 = Workload(dims=(256, 256), t=-1.0, mu=0.5, vc=2e-4, beta=20.0,
                      freq_index=tuple(range(64)), seed=2,
                      name="square 256x256, K=64")
CUBIC_48 = Workload(dims=(48, 48, 48), t=-1.0, mu=1.0, vc=1e-3, beta=10.0,
                    freq_index=tuple(range(32)), seed=3,
                    name="cubic 48^3, K=32")


def scaled_square(L: int, K: int, seed: int = 2, beta: float = 20.0,
                  mu: float = 0.5) -> Workload:
    """A square lattice with the 256^2 trap rescaled so the edge potential
    stays the same: vc = 2e-4 * (256/L)^2."""
    return Workload(dims=(L, L), t=-1.0, mu=mu, vc=2e-4 * (256.0 / L) ** 2,
                    beta=beta, freq_index=tuple(range(K)), seed=seed,
                    name=f"square {L}x{L}, K={K}")


def rect(dims, K: int = 2, seed: int = 7, vc: float = 0.01, mu: float = 0.5,
         beta: float = 10.0, freq_index=None) -> Workload:
    fi = tuple(range(K)) if freq_index is None else tuple(freq_index)
    return Workload(dims=tuple(dims), t=-1.0, mu=mu, vc=vc, beta=beta,
                    freq_index=fi, seed=seed, name=f"lattice {dims}, K={len(fi)}")


def cubic(L: int, K: int, seed: int = 3, beta: float = 10.0, mu: float = 1.0) -> Workload:
    """A simple cubic lattice with the 48^3 trap rescaled to keep the edge
    potential: vc = 1e-3 * (48/L)^2."""
    return Workload(dims=(L, L, L), t=-1.0, mu=mu, vc=1e-3 * (48.0 / L) ** 2, beta=beta,
                    freq_index=tuple(range(K)), seed=seed, name=f"cubic {L}^3, K={K}")


def serving_trace(n: int, rate: float, squares=(128, 256, 512), cubes=(32, 64),
                  k_range=(16, 256), beta_range=(5.0, 40.0), seed: int = 5):
    """A seeded stream of solve requests as a self-consistency loop would emit
    them: Poisson arrivals at `rate` per second, the lattice drawn uniformly
    from the squares and cubes, K ~ U{k_range}, beta ~ U[beta_range], and a
    fresh self-energy per request (seed 1000 + request id).  Returns a list of
    (arrival time in s, Workload)."""
    rng = np.random.default_rng(seed)
    shapes = [("sq", L) for L in squares] + [("cu", L) for L in cubes]
    t, out = 0.0, []
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        kind, L = shapes[int(rng.integers(len(shapes)))]
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        beta = float(rng.uniform(*beta_range))
        if kind == "sq":
            w = scaled_square(L, K, seed=1000 + rid, beta=beta)
        else:
            w = cubic(L, K, seed=1000 + rid, beta=beta)
        out.append((t, w))
    return out


def real_axis_inputs(dims, K: int, eta: float = 0.1, w_range=(-3.0, 3.0), seed: int = 7,
                     vc: float = 0.01, mu: float = 0.5):
    """Inputs on the real-frequency axis: energies z_k = w_k + i eta on a
    uniform grid of w_range, the trap V = vc r^2 and the per-site self-energy
    model continued to z: Sigma_i(z) = a_i / (z + b_i) (Im Sigma <= 0).
    Returns (V [N], z [K] complex, sigma [K, N] complex, mu)."""
    n = int(np.prod(dims))
    V = trap(dims, vc)
    z = np.linspace(w_range[0], w_range[1], K) + 1j * eta
    a, b = sigma_params(n, seed)
    return V, z, a[None, :] / (z[:, None] + b[None, :]), mu
