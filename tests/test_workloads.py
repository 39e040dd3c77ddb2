"""The seeded input generators (workloads/gen.py), CPU only: the exact
Fourier load vector against Gauss-Legendre quadrature of the same f, the
torch generator (used on the GPU for the large workloads) against the NumPy
one, and the eigenmode subsets against the full batch's draws."""
import math

import numpy as np
import pytest

from workloads import gen


@pytest.mark.parametrize("p", [0, 1, 3, 5, 10])
def test_fourier_load_is_the_integral(p):
    rng = np.random.default_rng(11)
    a, phi = rng.standard_normal(6), rng.uniform(0.0, 2.0 * math.pi, 6)
    N, T = 40, 7.0
    exact = gen.fourier_load(p, N, T, a, phi)
    fn = lambda t: sum(ak * np.sin((k + 1) * t + pk) for k, (ak, pk) in enumerate(zip(a, phi)))
    quad = gen.quadrature_load(p, N, T, fn, q=p + 16)
    assert np.max(np.abs(exact - quad)) <= 1e-13 * np.max(np.abs(quad))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_torch_load_equals_numpy_load(p):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12 + p)
    a, phi = rng.standard_normal(16), rng.uniform(0.0, 2.0 * math.pi, 16)
    N, T = 3000, 1e4 * 3000 / (1 << 24)
    ref = gen.fourier_load(p, N, T, a, phi)
    t = gen.fourier_load_torch(p, N, T, a, phi, device="cpu").numpy()
    out = torch.empty(N * (p + 1), dtype=torch.float64)
    gen.fourier_load_torch(p, N, T, a, phi, device="cpu", out=out)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(t - ref)) <= 1e-14 * scale
    assert np.array_equal(out.numpy(), t)


def test_eigenmode_subset_equals_full_batch():
    full = gen.eigenmode_batch(n_inst=64, log2_range=(2, 6))
    take = [0, 5, 17, 63]
    sub = gen.eigenmode_batch(n_inst=64, log2_range=(2, 6), take=take)
    for i, j in enumerate(take):
        a, b = sub.instances[i], full.instances[j]
        assert (a.N, a.lam) == (b.N, b.lam) and np.array_equal(a.f, b.f)
    lam, Ns = gen.eigenmode_sizes(64, log2_range=(2, 6))
    assert np.array_equal(lam, [i.lam for i in full.instances])
    assert np.array_equal(Ns, [i.N for i in full.instances])
