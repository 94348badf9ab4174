"""Seeded synthetic inputs for the HISQ even-odd CG.

This module only *draws* inputs.  It holds none of the solver's arithmetic
(no Dslash, no CG, no force): both the FP64 CPU oracle and the HIP library
receive the arrays built here, and neither imports the other.

Inputs stand in for the finite-temperature HotQCD ensembles that the paper
measures on (Sec. 1 and Sec. 3, lattices N_s^3 x N_t with N_t << N_s); those
ensembles are not available, so links are drawn as follows:

* U_{x,mu} = eta_mu(x) * exp(i * eps * H_{x,mu}), with H = sum_a omega_a lambda_a / 2,
  omega ~ N(0, 1) i.i.d. and lambda_a the Gell-Mann matrices, so H is a Gaussian
  Hermitian traceless 3x3 matrix.  The exponential is taken through the FP64
  eigen-decomposition of H.
* eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) is the staggered phase, folded into the
  links (the kernels never see it).
* N_{x,mu} = -(1/24) U_{x,mu} U_{x+mu,mu} U_{x+2mu,mu}: a three-link product
  standing in for the Naik link of Sec. 1, eq. (3).  It is s*V with s = 1/24 and
  V unitary, so it is exactly representable in the compressed 14-real Naik format.
* Sources: complex Gaussian, real and imaginary parts i.i.d. N(0, 1).

Layouts (the library's canonical ones):
  site index  s = x0 + L0*(x1 + L1*(x2 + L2*x3)), x0 fastest;
  links       [4][V][3][3] complex128 (mu, site, row, col);
  half field  [V/2][3][n] complex128, the index within a parity is s // 2.

Random numbers come from numpy.random.Generator(PCG64(seed)); the draw order
for the links is [mu][x3][x2][x1][x0][a].
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

__all__ = [
    "gell_mann", "staggered_phases", "make_links", "free_links", "make_sources",
    "random_su3", "plane_wave", "volume", "half_volume", "Config", "CONFIGS",
    "links_seed", "sources_seed", "even_mask", "to_half", "from_half",
]


def volume(L: Sequence[int]) -> int:
    return int(np.prod([int(v) for v in L]))


def half_volume(L: Sequence[int]) -> int:
    return volume(L) // 2


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0, 0, 1] = g[0, 1, 0] = 1
    g[1, 0, 1] = -1j
    g[1, 1, 0] = 1j
    g[2, 0, 0] = 1
    g[2, 1, 1] = -1
    g[3, 0, 2] = g[3, 2, 0] = 1
    g[4, 0, 2] = -1j
    g[4, 2, 0] = 1j
    g[5, 1, 2] = g[5, 2, 1] = 1
    g[6, 1, 2] = -1j
    g[6, 2, 1] = 1j
    g[7, 0, 0] = g[7, 1, 1] = 1 / np.sqrt(3)
    g[7, 2, 2] = -2 / np.sqrt(3)
    return g


def _coords(L: Sequence[int]) -> np.ndarray:
    """Coordinates of every site, shape (4, V), x0 fastest."""
    L = [int(v) for v in L]
    s = np.arange(volume(L), dtype=np.int64)
    out = np.empty((4, s.size), dtype=np.int64)
    for mu in range(4):
        out[mu] = s % L[mu]
        s = s // L[mu]
    return out


def even_mask(L: Sequence[int]) -> np.ndarray:
    """Boolean (V,) array, True where x0+x1+x2+x3 is even."""
    return (_coords(L).sum(axis=0) % 2) == 0


def staggered_phases(L: Sequence[int]) -> np.ndarray:
    """eta_mu(x) = (-1)^(x_0+...+x_{mu-1}), shape (4, V) float64."""
    c = _coords(L)
    eta = np.ones((4, c.shape[1]))
    for mu in range(1, 4):
        eta[mu] = np.where(c[:mu].sum(axis=0) % 2 == 0, 1.0, -1.0)
    return eta


def _roll_site(field: np.ndarray, L: Sequence[int], mu: int, hop: int) -> np.ndarray:
    """Return g with g[s] = field[s + hop*mu_hat] (periodic); field is (V, ...)."""
    L = [int(v) for v in L]
    shaped = field.reshape((L[3], L[2], L[1], L[0]) + field.shape[1:])
    axis = 3 - mu
    return np.roll(shaped, -hop, axis=axis).reshape(field.shape)


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def make_links(L: Sequence[int], eps: float, seed: int, phases: bool = True,
               chunk: int = 1 << 18) -> tuple[np.ndarray, np.ndarray]:
    """Seeded smeared links U and Naik links N, each [4][V][3][3] complex128."""
    L = [int(v) for v in L]
    V = volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    lam_half = gell_mann() / 2
    U = np.empty((4, V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        omega = rng.standard_normal((V, 8))
        for a in range(0, V, chunk):
            b = min(V, a + chunk)
            H = np.tensordot(omega[a:b], lam_half, axes=([1], [0]))
            U[mu, a:b] = _expi_hermitian(H, eps)
    if phases:
        U *= staggered_phases(L)[:, :, None, None]
    N = np.empty_like(U)
    for mu in range(4):
        U1 = _roll_site(U[mu], L, mu, 1)
        U2 = _roll_site(U[mu], L, mu, 2)
        N[mu] = -(1.0 / 24.0) * (U[mu] @ U1 @ U2)
    return U, N


def free_links(L: Sequence[int], c: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Free field without phases: U = 1, N = c * 1."""
    V = volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:, :, [0, 1, 2], [0, 1, 2]] = 1.0
    return U, c * U.copy()


def make_sources(L: Sequence[int], n: int, seed: int) -> np.ndarray:
    """Complex Gaussian half-lattice bundle, [V/2][3][n] complex128."""
    Vh = half_volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((Vh, 3, n, 2))
    return g[..., 0] + 1j * g[..., 1]


def random_su3(count: int, seed: int) -> np.ndarray:
    """Haar-like random SU(3) matrices, shape (count, 3, 3) complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.standard_normal((count, 3, 3)) + 1j * rng.standard_normal((count, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[:, None, None]


def make_noise(L: Sequence[int], n: int, seed: int, kind: str = "z2") -> tuple[np.ndarray, np.ndarray]:
    """Random vectors for the trace estimator of eq. (2), split into the even and
    odd half fields ([V/2][3][n] complex128 each): "z2" draws every component
    from {+1, -1}, "gauss" from a unit complex Gaussian."""
    Vh = half_volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "z2":
        f = 1.0 - 2.0 * rng.integers(0, 2, size=(2, Vh, 3, n))
        f = f.astype(np.complex128)
    elif kind == "gauss":
        g = rng.standard_normal((2, Vh, 3, n, 2)) / np.sqrt(2.0)
        f = g[..., 0] + 1j * g[..., 1]
    else:
        raise ValueError("kind must be 'z2' or 'gauss'")
    return np.ascontiguousarray(f[0]), np.ascontiguousarray(f[1])


def plane_wave(L: Sequence[int], k: Sequence[int], xi: Sequence[complex]) -> np.ndarray:
    """Full-lattice field e^{i p.x} xi with p_mu = 2 pi k_mu / L_mu, shape (V, 3, 1)."""
    c = _coords(L)
    phase = np.zeros(c.shape[1])
    for mu in range(4):
        phase += 2 * np.pi * k[mu] * c[mu] / L[mu]
    return (np.exp(1j * phase)[:, None] * np.asarray(xi, dtype=np.complex128)[None, :])[:, :, None]


def to_half(full: np.ndarray, L: Sequence[int], parity: int) -> np.ndarray:
    """Restrict a full field (V, 3, n) to one parity, in the s // 2 ordering."""
    m = even_mask(L) if parity == 0 else ~even_mask(L)
    return np.ascontiguousarray(full[m])


def from_half(half: np.ndarray, L: Sequence[int], parity: int) -> np.ndarray:
    """Embed a half field into a full one (zeros on the other parity)."""
    V = volume(L)
    out = np.zeros((V,) + half.shape[1:], dtype=half.dtype)
    m = even_mask(L) if parity == 0 else ~even_mask(L)
    out[m] = half
    return out


@dataclasses.dataclass(frozen=True)
class Config:
    """One synthetic workload: lattice, bundle sizes, mass and link spread."""
    name: str
    L: tuple
    nrhs: tuple
    mass: float
    eps: float
    tol: float = 1e-10


# Workloads shaped like the paper's finite-temperature lattices (N_t << N_s).
CONFIGS = {
    1: Config("8^4 plain FP64", (8, 8, 8, 8), (1,), 0.1, 0.3),
    2: Config("32^3x8 dslash+cg sweep", (32, 32, 32, 8), (1, 2, 4, 8), 0.02, 0.3),
    3: Config("48^3x12 mixed 8-rhs", (48, 48, 48, 12), (8,), 0.01, 0.2),
    4: Config("batched 16^3x4/24^3x6/32^3x8", (16, 16, 16, 4), (3, 5, 8), 0.05, 0.3),
    5: Config("gradient 24^3x6", (24, 24, 24, 6), (4,), 0.05, 0.3),
}

# Batched workload: (lattice, nrhs) pairs, each at two masses.
BATCHED_PROBLEMS = [((16, 16, 16, 4), 3), ((24, 24, 24, 6), 5), ((32, 32, 32, 8), 8)]
BATCHED_MASSES = (0.05, 0.01)


def links_seed(config: int, solve_index: int = 0) -> int:
    return 1000 * config + solve_index


def sources_seed(config: int, solve_index: int = 0) -> int:
    return 1000 * config + 500 + solve_index
