"""Seeded synthetic inputs for the Exp-ParaDiag workloads.

This module only draws random numbers and builds initial conditions and
instance descriptors.  It holds none of the method's arithmetic, so both the
CPU reference and the GPU library can be fed from it without sharing solver
code.  Every array is float64, C-contiguous, row-major with the last spatial
index fastest, on the periodic grid x_j = 2*pi*j/n.

Workloads (all on periodic [0, 2*pi)^d):
  heat1d       1D heat u_t = u_xx, n=64, Nt=16, T=1, alpha=1e-2;
               u0 = sin x + sum_{k=1..8} (a_k cos kx + b_k sin kx),
               a_k, b_k ~ N(0, 0.1) (standard deviation 0.1).
  allen_cahn2d 2D Allen-Cahn u_t = eps^2 Lap u + u - u^3, eps=0.05, n=256,
               Nt=64, T=2, alpha=1e-3; u0 ~ U[-0.9, 0.9] i.i.d. per point.
  diffusion2d_ebdf2  allen_cahn2d's grid, window and u0 without the
               reaction (u_t = eps^2 Lap u), second-order exponential BDF.
  advection2d  allen_cahn2d with an advection term -b.grad u, b = (2, 1)
               (complex symbol, real state).
  schroedinger2d  u_t = i Lap u - 2i u (complex state), n=256, Nt=64, T=1,
               alpha=1e-3, u0 = Gaussian wave packet (width 0.4,
               wavenumber 5) centred in the box.
  rd2d         2D reaction-diffusion u_t = 0.1 Lap u + u - u^3, n=512,
               Nt=128, T=1, ETD2; u0 = sum of 32 periodic Gaussians with
               amplitude U[-1,1], width U[0.1,0.5], centre U[0,2pi)^2.
  batch        heterogeneous 2D Allen-Cahn instances: n in {64,128,256},
               Nt in {16,32,64,128}, eps ~ U[0.02,0.1], alpha in {1e-2,1e-3},
               T=2, u0 ~ U[-0.9,0.9]; instance i uses default_rng([seed, i]).
  served       Poisson arrival times over a mix of batch-shaped 2D requests
               and 3D 128^3 heat / Allen-Cahn requests (Nt=32, T=1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Instance", "grid_coords", "heat1d", "allen_cahn2d", "rd2d", "batch",
    "diffusion2d_ebdf2", "advection2d", "schroedinger2d", "wave_packet",
    "served_stream", "uniform_field", "gaussians_field", "low_mode_field",
    "scaled",
]


@dataclasses.dataclass
class Instance:
    """Plain description of one solve: grid, time window and PDE coefficients.

    u_t = a*Lap(u) - c*u + n1*u + n2*u^2 + n3*u^3 on periodic [0,2pi)^dim.
    scheme is 1 (ETD1) or 2 (ETD2); precision is 0 (fp64) or 1 (mixed).
    """
    name: str
    dim: int
    n: int
    Nt: int
    T: float
    alpha: float
    a: float
    c: float = 0.0
    n1: float = 0.0
    n2: float = 0.0
    n3: float = 0.0
    scheme: int = 1
    precision: int = 0
    u0: Optional[np.ndarray] = None
    b: tuple = (0.0, 0.0, 0.0)
    a_im: float = 0.0
    c_im: float = 0.0
    cstate: bool = False
    jac: int = 1

    @property
    def dt(self) -> float:
        return self.T / self.Nt

    @property
    def shape(self):
        return (self.n,) * self.dim

    @property
    def Ns(self) -> int:
        return self.n ** self.dim

    @property
    def dof(self) -> int:
        return self.Ns * self.Nt

    @property
    def nonlinear(self) -> bool:
        return (self.n1, self.n2, self.n3) != (0.0, 0.0, 0.0)


def grid_coords(dim: int, n: int):
    x = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    return np.meshgrid(*([x] * dim), indexing="ij")


def uniform_field(rng, dim, n, lo=-0.9, hi=0.9):
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(n,) * dim))


def low_mode_field(rng, n, kmax=8, sigma=0.1):
    (x,) = grid_coords(1, n)
    u = np.sin(x)
    a = rng.normal(0.0, sigma, size=kmax)
    b = rng.normal(0.0, sigma, size=kmax)
    for k in range(1, kmax + 1):
        u = u + a[k - 1] * np.cos(k * x) + b[k - 1] * np.sin(k * x)
    return np.ascontiguousarray(u)


def gaussians_field(rng, dim, n, count=32, wlo=0.1, whi=0.5):
    """Sum of periodic Gaussian bumps, minimum-image distance on the torus."""
    X = grid_coords(dim, n)
    u = np.zeros((n,) * dim)
    amp = rng.uniform(-1.0, 1.0, size=count)
    wid = rng.uniform(wlo, whi, size=count)
    cen = rng.uniform(0.0, 2.0 * np.pi, size=(count, dim))
    for g in range(count):
        d2 = np.zeros_like(u)
        for ax in range(dim):
            d = np.abs(X[ax] - cen[g, ax])
            d = np.minimum(d, 2.0 * np.pi - d)
            d2 += d * d
        u += amp[g] * np.exp(-d2 / (2.0 * wid[g] ** 2))
    return np.ascontiguousarray(u)


def heat1d(seed: int = 0, n: int = 64, Nt: int = 16, T: float = 1.0,
           alpha: float = 1e-2) -> Instance:
    rng = np.random.default_rng(seed)
    return Instance("heat1d", 1, n, Nt, T, alpha, a=1.0,
                    u0=low_mode_field(rng, n))


def allen_cahn2d(seed: int = 0, n: int = 256, Nt: int = 64, T: float = 2.0,
                 alpha: float = 1e-3, eps: float = 0.05,
                 precision: int = 0, scheme: int = 1) -> Instance:
    rng = np.random.default_rng(seed)
    return Instance("allen_cahn2d", 2, n, Nt, T, alpha, a=eps * eps,
                    n1=1.0, n3=-1.0, scheme=scheme, precision=precision,
                    u0=uniform_field(rng, 2, n))


def diffusion2d_ebdf2(seed: int = 0, n: int = 256, Nt: int = 64,
                      T: float = 2.0, alpha: float = 1e-3,
                      eps: float = 0.05) -> Instance:
    """The Allen-Cahn grid and window without the reaction term, for the
    second-order exponential BDF (scheme 3, linear problems)."""
    rng = np.random.default_rng(seed)
    return Instance("diffusion2d_ebdf2", 2, n, Nt, T, alpha, a=eps * eps,
                    scheme=3, u0=uniform_field(rng, 2, n))


def diffusion2d_ebdf(order: int, seed: int = 0, n: int = 256,
                     Nt: int = 64, T: float = 2.0, alpha: float = 1e-3,
                     eps: float = 0.05) -> Instance:
    """diffusion2d_ebdf2's problem stepped by the exponential BDF of order
    2..6 (schemes 3, 5, 6, 7, 8)."""
    rng = np.random.default_rng(seed)
    scheme = 3 if order == 2 else order + 2
    return Instance(f"diffusion2d_ebdf{order}", 2, n, Nt, T, alpha,
                    a=eps * eps, scheme=scheme, u0=uniform_field(rng, 2, n))


def heat2d_table(a: float, seed: int = 0, n: int = 256, Nt: int = 64,
                 dt: float = 0.01, alpha: float = 1e-3,
                 scheme: int = 1) -> Instance:
    """The purely diffusive problem of Table cpu_time_combined (u_t = a Lap
    u, a in {1e-1, 1e-5}, dt = 0.01) on the periodic 256^2 box, Nt steps,
    first-order (scheme 1) or EBDF2 (scheme 3) time stepping."""
    rng = np.random.default_rng(seed)
    return Instance("heat2d_table", 2, n, Nt, Nt * dt, alpha, a=a,
                    scheme=scheme, u0=uniform_field(rng, 2, n))


def advection2d(seed: int = 0, n: int = 256, Nt: int = 64, T: float = 2.0,
                alpha: float = 1e-3, eps: float = 0.05,
                b: tuple = (2.0, 1.0), nonlinear: bool = True) -> Instance:
    """allen_cahn2d's grid, window and u0 with an advection term
    -b.grad(u) (complex symbol, real state); without the reaction term when
    nonlinear is False."""
    rng = np.random.default_rng(seed)
    return Instance("advection2d", 2, n, Nt, T, alpha, a=eps * eps,
                    n1=1.0 if nonlinear else 0.0,
                    n3=-1.0 if nonlinear else 0.0,
                    u0=uniform_field(rng, 2, n), b=tuple(b) + (0.0,))


def wave_packet(dim: int, n: int, k0: float = 5.0, width: float = 0.4,
                centre: float = math.pi) -> np.ndarray:
    """Gaussian packet exp(-|x - centre|^2 / (2 width^2)) e^{-i k0 (x_0 -
    centre)} (complex128), periodic box, no randomness."""
    g = grid_coords(dim, n)
    r2 = sum((gi - centre) ** 2 for gi in g)
    return (np.exp(-r2 / (2.0 * width * width))
            * np.exp(-1j * k0 * (g[0] - centre))).astype(np.complex128)


def schroedinger2d(n: int = 256, Nt: int = 64, T: float = 1.0,
                   alpha: float = 1e-3, c_im: float = 2.0,
                   scheme: int = 1) -> Instance:
    """u_t = i Lap u - i c_im u (a = i, the Schroedinger equation of the
    paper's Sec. 6) on the periodic box, complex state, from a Gaussian wave
    packet (width 0.4, wavenumber 5)."""
    return Instance("schroedinger2d", 2, n, Nt, T, alpha, a=0.0,
                    scheme=scheme, u0=wave_packet(2, n), a_im=1.0,
                    c_im=c_im, cstate=True)


def rd2d(seed: int = 0, n: int = 512, Nt: int = 128, T: float = 1.0,
         alpha: float = 1e-3, precision: int = 1) -> Instance:
    rng = np.random.default_rng(seed)
    return Instance("rd2d", 2, n, Nt, T, alpha, a=0.1, n1=1.0, n3=-1.0,
                    scheme=2, precision=precision,
                    u0=gaussians_field(rng, 2, n))


def batch(count: int = 256, seed: int = 0,
          ns: Sequence[int] = (64, 128, 256),
          nts: Sequence[int] = (16, 32, 64, 128),
          alphas: Sequence[float] = (1e-2, 1e-3),
          T: float = 2.0, precision: int = 1) -> List[Instance]:
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.choice(ns))
        Nt = int(rng.choice(nts))
        alpha = float(rng.choice(alphas))
        eps = float(rng.uniform(0.02, 0.1))
        out.append(Instance(f"ac2d_{i}", 2, n, Nt, T, alpha, a=eps * eps,
                            n1=1.0, n3=-1.0, precision=precision,
                            u0=uniform_field(rng, 2, n)))
    return out


def served_stream(count: int, rate: float, seed: int = 0,
                  frac3d: float = 0.1, n3d: int = 128, Nt3d: int = 32,
                  batch_kw: Optional[dict] = None):
    """Poisson arrivals: returns (arrival_times_seconds, instances).

    A fraction frac3d of the requests are 3D (half heat with a=1 and
    Gaussian u0, half Allen-Cahn with eps ~ U[0.02,0.1] and uniform u0), the
    rest are batch-shaped 2D Allen-Cahn instances.
    """
    rng = np.random.default_rng([seed, 10_000_019])
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    base = batch(count, seed=seed, **(batch_kw or {}))
    out = []
    for i in range(count):
        r = np.random.default_rng([seed, i, 3])
        if r.uniform() < frac3d:
            if r.uniform() < 0.5:
                out.append(Instance(f"heat3d_{i}", 3, n3d, Nt3d, 1.0, 1e-3,
                                    a=1.0, precision=base[i].precision,
                                    u0=gaussians_field(r, 3, n3d, count=8)))
            else:
                eps = float(r.uniform(0.02, 0.1))
                out.append(Instance(f"ac3d_{i}", 3, n3d, Nt3d, 1.0, 1e-3,
                                    a=eps * eps, n1=1.0, n3=-1.0,
                                    precision=base[i].precision,
                                    u0=uniform_field(r, 3, n3d)))
        else:
            out.append(base[i])
    return t, out


def scaled(inst: Instance, n: int, Nt: int, seed: int = 0) -> Instance:
    """Same PDE and time window on a smaller grid (for oracle-sized cases)."""
    rng = np.random.default_rng([seed, n, Nt])
    if inst.name.startswith("heat1d"):
        u0 = low_mode_field(rng, n, kmax=min(8, n // 2 - 1))
    elif inst.name.startswith("rd2d"):
        u0 = gaussians_field(rng, inst.dim, n)
    else:
        u0 = uniform_field(rng, inst.dim, n)
    return dataclasses.replace(inst, n=n, Nt=Nt, u0=u0)
