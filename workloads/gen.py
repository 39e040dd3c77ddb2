"""Seeded synthetic workloads for the DG-in-time multigrid solve.

Only random draws and DG load vectors live here (no part of the multigrid).
The load vector of slab n (length tau, midpoint c_n) is
    f_n[m] = int_{t_{n-1}}^{t_n} f(t) P_m(xi(t)) dt,  xi = 2(t - t_{n-1})/tau - 1,
for the unnormalised Legendre basis; the initial value u0 is *not* folded in
(the solver adds it to slab 0).  Layout: float64, [instance][slab][m].

Recipes (name, seed; draws in the order listed):
  fourier_small (1)      u'+u=f on (0,10], u0=1, p=1, N=1024; f = sum_{k=1..8} a_k sin(k t + phi_k),
     a = standard_normal(8), then phi = uniform(0, 2pi, 8).
  fourier_scalar (2)     lambda=1, T=1000, u0=1, N=2^22, p in {0..5}; same
     form with 16 modes.
  eigenmode_batch (3)    4096 instances: kappa = uniform(0.01, 1) (one draw), lambda_j = pi^2 j^2 kappa,
     N_j = 2^integers(12, 19), T_j = 1, p = 1, u0 = 1; load vector M_tau c with
     c ~ standard_normal per (slab, coefficient), drawn instance by instance.
  adjoint_batch (4)      256 instances, N = 2^20, p = 2, T = 100: lambda_b = uniform(0.1, 10, 256),
     then per instance a (16), phi (16); then targets y ~ standard_normal(256 x N).
  long_horizon (5)       N = 2^24, p = 3, T = 1e4: lambda = uniform(0.5, 50, B) (B = 1 or 64), then
     per instance a (16), phi (16).
Smaller N (same recipe) serve the parity tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Instance", "Workload", "sph_jn", "fourier_load", "fourier_load_torch",
           "quadrature_load",
           "gaussian_legendre_load", "fourier_small", "fourier_scalar", "eigenmode_batch", "adjoint_batch", "long_horizon",
           "fourier_batch", "fourier_params", "eigenmode_sizes", "adjoint_params", "long_horizon_params"]


def sph_jn(m: int, x: np.ndarray) -> np.ndarray:
    """Spherical Bessel j_m(x): power series for |x| <= 1, scipy otherwise."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) <= 1.0
    if np.any(small):
        xs = x[small]
        t = xs ** m / np.prod(np.arange(1, 2 * m + 2, 2, dtype=np.float64))
        tot = np.zeros_like(xs)
        for j in range(40):
            tot += t
            t = t * (-xs * xs / 2.0) / ((j + 1) * (2 * m + 2 * j + 3))
        out[small] = tot
    if np.any(~small):
        from scipy.special import spherical_jn
        out[~small] = spherical_jn(m, x[~small])
    return out


def fourier_load(p: int, N: int, T: float, a, phi) -> np.ndarray:
    """Load vector of f(t) = sum_k a_k sin(k t + phi_k), k = 1..len(a), exact:
    int_{-1}^{1} e^{i b xi} P_m(xi) dxi = 2 i^m j_m(b) gives
    f_n[m] = tau sum_k a_k j_m(k tau/2) sin(k c_n + phi_k + m pi/2)."""
    P = p + 1
    tau = T / N
    c = (np.arange(N, dtype=np.float64) + 0.5) * tau
    f = np.zeros((N, P))
    for k, (ak, pk) in enumerate(zip(a, phi), start=1):
        th = k * c + pk
        s, co = np.sin(th), np.cos(th)
        for m in range(P):
            jm = float(sph_jn(m, np.array([k * tau / 2.0]))[0])
            trig = (s, co, -s, -co)[m % 4]
            f[:, m] += tau * ak * jm * trig
    return f.reshape(-1)


def fourier_load_torch(p: int, N: int, T: float, a, phi, device="cuda", out=None):
    """The same load vector as :func:`fourier_load` (up to the order of the
    sum over modes), evaluated with torch on `device` (for large workloads):
    the sines and cosines of every mode in one pass each and the sum over
    modes as two small matrix products.  Returns a flat float64 tensor, or
    fills `out` (a flat view of N*(p+1) elements)."""
    import torch
    P = p + 1
    tau = T / N
    K = len(a)
    kk = torch.arange(1, K + 1, dtype=torch.float64, device=device)
    c = (torch.arange(N, dtype=torch.float64, device=device) + 0.5) * tau
    th = torch.addcmul(torch.as_tensor(np.asarray(phi, dtype=np.float64), device=device)[:, None],
                       kk[:, None], c[None, :])
    S, C = torch.sin(th), torch.cos(th)
    del th
    # f_n[m] = tau sum_k a_k j_m(k tau/2) sin(k c_n + phi_k + m pi/2)
    cs = np.zeros((P, K))
    cc = np.zeros((P, K))
    for k, ak in enumerate(a, start=1):
        for m in range(P):
            w = tau * float(ak) * float(sph_jn(m, np.array([k * tau / 2.0]))[0])
            (cs if m % 2 == 0 else cc)[m, k - 1] = w * (1.0 if m % 4 < 2 else -1.0)
    f = torch.as_tensor(cs, device=device) @ S
    f += torch.as_tensor(cc, device=device) @ C
    del S, C
    if out is not None:
        out.view(N, P).copy_(f.t())
        return out
    return f.t().contiguous().reshape(-1)


def quadrature_load(p: int, N: int, T: float, fn, q: int | None = None) -> np.ndarray:
    """Load vector of a callable f by q-point Gauss-Legendre per slab."""
    P = p + 1
    q = q or P + 8
    x, w = np.polynomial.legendre.leggauss(q)
    tau = T / N
    t0 = np.arange(N, dtype=np.float64) * tau
    t = t0[:, None] + 0.5 * tau * (x[None, :] + 1.0)
    fv = fn(t)
    V = np.stack([np.polynomial.legendre.legval(x, np.eye(P)[m]) for m in range(P)], axis=1)
    return (0.5 * tau * (fv * w[None, :]) @ V).reshape(-1)


def gaussian_legendre_load(p: int, N: int, T: float, rng) -> np.ndarray:
    """Load vector M_tau c of f = sum_m c_m P_m(xi) with c ~ N(0, 1)."""
    P = p + 1
    tau = T / N
    c = rng.standard_normal((N, P))
    return (c * (tau / (2.0 * np.arange(P) + 1.0))[None, :]).reshape(-1)


@dataclass
class Instance:
    p: int
    N: int
    T: float
    lam: float
    u0: float
    f: np.ndarray          # unfolded load vector, N*(p+1)


@dataclass
class Workload:
    name: str
    p: int
    instances: list = field(default_factory=list)
    targets: list | None = None     # per-instance targets y (adjoint batch)

    @property
    def unknowns(self) -> int:
        return sum(i.N * (i.p + 1) for i in self.instances)


def fourier_small(N: int = 1024, seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(8)
    phi = rng.uniform(0.0, 2.0 * math.pi, 8)
    return Workload("fourier_small", 1, [Instance(1, N, 10.0, 1.0, 1.0, fourier_load(1, N, 10.0, a, phi))])


def fourier_scalar(p: int, N: int = 1 << 22, T: float = 1000.0, seed: int = 2) -> Workload:
    """Scalar, lambda = 1.  The default T keeps tau = 1000 / 2^22 also when a
    smaller N is asked for only if T is scaled by the caller."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(16)
    phi = rng.uniform(0.0, 2.0 * math.pi, 16)
    return Workload(f"fourier_scalar_p{p}", p, [Instance(p, N, T, 1.0, 1.0, fourier_load(p, N, T, a, phi))])


def eigenmode_batch(n_inst: int = 4096, log2_range=(12, 19), seed: int = 3, take=None) -> Workload:
    """Eigenmode batch.  `take` (an iterable of instance indices) keeps a
    subset; draws for all n_inst instances are still made in order so that a
    subset equals the corresponding instances of the full batch."""
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.01, 1.0)
    lam = (math.pi ** 2) * (np.arange(1, n_inst + 1, dtype=np.float64) ** 2) * kappa
    Ns = 2 ** rng.integers(log2_range[0], log2_range[1], size=n_inst)
    keep = set(range(n_inst)) if take is None else set(take)
    inst = []
    for j in range(n_inst):
        if j in keep:
            f = gaussian_legendre_load(1, int(Ns[j]), 1.0, rng)
            inst.append(Instance(1, int(Ns[j]), 1.0, float(lam[j]), 1.0, f))
        else:
            rng.standard_normal(int(Ns[j]) * 2)   # keep the stream aligned
    return Workload("eigenmode_batch", 1, inst)


def fourier_batch(name: str, p: int, N: int, T: float, lam: np.ndarray, rng, modes: int = 16):
    inst = []
    for lb in lam:
        a = rng.standard_normal(modes)
        phi = rng.uniform(0.0, 2.0 * math.pi, modes)
        inst.append(Instance(p, N, T, float(lb), 1.0, fourier_load(p, N, T, a, phi)))
    return Workload(name, p, inst)


def fourier_params(lam: np.ndarray, rng, modes: int = 16):
    """Per-instance (lambda, a, phi) draws of a Fourier batch, without load
    vectors (for generation on the GPU with fourier_load_torch)."""
    out = []
    for lb in lam:
        a = rng.standard_normal(modes)
        phi = rng.uniform(0.0, 2.0 * math.pi, modes)
        out.append((float(lb), a, phi))
    return out


def adjoint_params(B: int = 256, seed: int = 4):
    rng = np.random.default_rng(seed)
    return fourier_params(rng.uniform(0.1, 10.0, B), rng), rng


def long_horizon_params(B: int = 1, seed: int = 5):
    rng = np.random.default_rng(seed)
    return fourier_params(rng.uniform(0.5, 50.0, B), rng)


def eigenmode_sizes(n_inst: int = 4096, log2_range=(12, 19), seed: int = 3):
    """(lambda_j, N_j) of the eigenmode batch, drawn as in eigenmode_batch."""
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.01, 1.0)
    lam = (math.pi ** 2) * (np.arange(1, n_inst + 1, dtype=np.float64) ** 2) * kappa
    Ns = 2 ** rng.integers(log2_range[0], log2_range[1], size=n_inst)
    return lam, Ns


def adjoint_batch(B: int = 256, N: int = 1 << 20, T: float = 100.0, seed: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.1, 10.0, B)
    w = fourier_batch("adjoint_batch", 2, N, T, lam, rng)
    w.targets = [rng.standard_normal(N) for _ in range(B)]
    return w


def long_horizon(B: int = 1, N: int = 1 << 24, T: float = 1e4, seed: int = 5) -> Workload:
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.5, 50.0, B)
    return fourier_batch(f"long_horizon_b{B}", 3, N, T, lam, rng)


def heat_problem(p: int = 1, nx: int = 255, N: int = 1 << 14, T: float = 0.1, seed: int = 7):
    """Space-time heat equation u_t - u_xx = f on (0,1), u = 0 at both ends,
    nx interior points: u0 = sin(pi x) and a load M_tau c with Gaussian
    Legendre coefficients c ~ N(0, 1) at every point (layout
    [point][slab][k]).  Returns (u0, f)."""
    rng = np.random.default_rng(seed)
    P = p + 1
    tau = T / N
    x = np.arange(1, nx + 1) / (nx + 1.0)
    c = rng.standard_normal((nx, N, P))
    f = (c * (tau / (2.0 * np.arange(P) + 1.0))[None, None, :]).reshape(-1)
    return np.sin(np.pi * x), f
