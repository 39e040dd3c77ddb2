"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-derives the oracle's
own formula: the oracle builds its matrices by quadrature of the integral
definitions, while the checks use printed closed forms, exact identities,
dense brute force and the Fourier symbol of the two-grid cycle.
"""
import math
import os

import numpy as np
import pytest

from oracle import analysis as an
from oracle import core
from workloads import gen


def _golden_pade(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "pade_subdiagonal.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            p, num, den = (s.strip() for s in line.split("|"))
            rows[int(p)] = ([float(x) for x in num.split()], [float(x) for x in den.split()])
    return rows


def _golden_const(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "paper_constants.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


# --------------------------------------------------------------------------
# Discretisation (section 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam,T,N", [(1.0, 1.0, 16), (3.5, 2.0, 40)])
def test_p0_is_backward_euler(lam, T, N):
    """Section 2.1: constant polynomials give backward Euler,
    u_n = (u_{n-1} + int_{slab n} f) / (1 + lam tau)."""
    rng = np.random.default_rng(0)
    f = rng.standard_normal(N)            # = int f over each slab for p = 0
    u0 = 0.7
    u = core.direct_solve(0, T, lam, u0, f)
    tau = T / N
    ref = np.empty(N)
    prev = u0
    for n in range(N):
        prev = (prev + f[n]) / (1.0 + lam * tau)
        ref[n] = prev
    assert np.max(np.abs(u - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_stability_function_is_pade(p, golden_dir):
    """Corollary chap4_corollary1 / Lemma chap4_theorem2: for f = 0 the end
    value after one slab is R(-lam tau) u0 with R the (p, p+1) subdiagonal
    Pade approximant of e^z, and alpha (the nonzero eigenvalue of
    (K + M)^{-1} N) equals the same value."""
    num, den = _golden_pade(golden_dir)[p]
    for z in [1e-6, 1e-3, 0.1, 1.0, 3.0, 10.0, 1e3]:
        R = an.pade(num, den, -z)
        t = core.tables(p, 1.0, z)
        assert abs(t["alpha"] - R) <= 1e-13 * max(1.0, abs(R))
        N = 5
        u = core.direct_solve(p, float(N), z, 1.0, np.zeros(N * (p + 1)))
        w = u.reshape(N, p + 1).sum(axis=1)          # end values P_k(1) = 1
        assert np.allclose(w, R ** np.arange(1, N + 1), rtol=1e-12, atol=1e-14)


def test_alpha_range_minimum(golden_dir):
    """Lemma chap4_lemma7 proof: alpha >= (5 - 3 sqrt 3)/2 ~ -0.0980762, attained
    for p = 1 at z = 3 + 3 sqrt 3; every alpha lies in [alpha_min, 1]."""
    c = _golden_const(golden_dir)
    zs = np.logspace(-6, 6, 400)
    for p in range(4):
        al = np.array([core.tables(p, 1.0, z)["alpha"] for z in zs])
        assert np.all(al <= 1.0) and np.all(al >= c["alpha_min"] - 1e-7)
    zstar = 3.0 + 3.0 * math.sqrt(3.0)
    amin = core.tables(1, 1.0, zstar)["alpha"]
    assert abs(amin - c["alpha_min"]) < 1e-7
    assert abs(amin - (5.0 - 3.0 * math.sqrt(3.0)) / 2.0) < 1e-14
    assert core.tables(1, 1.0, zstar * 1.01)["alpha"] > amin
    assert core.tables(1, 1.0, zstar * 0.99)["alpha"] > amin


def test_alpha_zero_for_odd_degree():
    """Section 4.2: for odd p the Pade approximant of e^{-z} has exactly one
    positive zero (p = 1: z = 3); for even p alpha stays positive."""
    assert abs(core.tables(1, 1.0, 3.0)["alpha"]) < 1e-15
    zs = np.logspace(-4, 5, 300)
    for p in (0, 2):
        assert min(core.tables(p, 1.0, z)["alpha"] for z in zs) > 0.0
    for p in (1, 3):
        al = np.array([core.tables(p, 1.0, z)["alpha"] for z in zs])
        assert np.count_nonzero(np.diff(np.sign(al))) == 1


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_polynomial_solution_is_reproduced(p):
    """Variational problem chap4_discreteVarFormODE: if the exact solution is
    a polynomial of degree <= p, it lies in the trial space and satisfies the
    DG equations with no jumps, so the DG solution equals it on every slab."""
    rng = np.random.default_rng(p)
    c = rng.standard_normal(p + 1)
    lam, T, N = 2.3, 3.0, 12
    u_ex = lambda t: sum(c[j] * t ** j for j in range(p + 1))
    du_ex = lambda t: sum(j * c[j] * t ** (j - 1) for j in range(1, p + 1)) + 0 * t
    f = gen.quadrature_load(p, N, T, lambda t: du_ex(t) + lam * u_ex(t), q=p + 6)
    u = core.direct_solve(p, T, lam, u_ex(0.0), f).reshape(N, p + 1)
    x, w = np.polynomial.legendre.leggauss(p + 6)
    tau = T / N
    V = an.legendre_values(p + 1, x)
    for n in range(N):
        vals = u_ex(n * tau + 0.5 * tau * (x + 1.0))
        coef = (V * w[:, None]).T @ vals * (2.0 * np.arange(p + 1) + 1.0) / 2.0
        assert np.allclose(u[n], coef, rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(coef))))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_radau_ia_collocation(p):
    """Theorem chap4_theorem1a: with the load vector taken by the left Radau
    rule with p+1 points, the DG solution satisfies the discontinuous
    collocation equations (the jump equation at t_{n-1} and the ODE at
    c_2..c_{p+1}); here with lam in place of 1."""
    s = p + 1
    c, b = an.radau_ia(s)
    lam, T, N, u0 = 1.7, 2.0, 8, 0.4
    tau = T / N
    fn = lambda t: np.sin(3.0 * t) + t * t
    V = an.legendre_values(s, 2.0 * c - 1.0)                  # psi_k(t_{n-1} + c_i tau)
    dV = np.stack([np.polynomial.legendre.legval(2.0 * c - 1.0,
                   np.polynomial.legendre.legder(np.eye(s)[k])) for k in range(s)], axis=1)
    f = np.concatenate([tau * (b * fn(n * tau + c * tau)) @ V for n in range(N)])
    u = core.direct_solve(p, T, lam, u0, f).reshape(N, s)
    prev = u0
    for n in range(N):
        val = V @ u[n]
        der = (2.0 / tau) * (dV @ u[n])
        t0 = n * tau
        jump = val[0] - prev
        assert abs(jump - tau * b[0] * (fn(t0) - der[0] - lam * val[0])) < 1e-13
        for i in range(1, s):
            assert abs(der[i] + lam * val[i] - fn(t0 + c[i] * tau)) < 1e-11
        prev = u[n].sum()


@pytest.mark.parametrize("p,N", [(0, 64), (1, 16), (2, 8), (3, 4)])
def test_nodal_order(p, N):
    """Theorem chap4_theorem2a: Radau IA with s = p+1 stages has order
    2s - 1 = 2p + 1 at the nodes; u = e^{-t} (f = 0, u0 = 1)."""
    errs = []
    for n in (N, 2 * N):
        u = core.direct_solve(p, 1.0, 1.0, 1.0, np.zeros(n * (p + 1)))
        errs.append(abs(u.reshape(n, p + 1)[-1].sum() - math.exp(-1.0)))
    order = math.log2(errs[0] / errs[1])
    assert abs(order - (2 * p + 1)) < 0.1


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_direct_against_dense(p):
    """Eq. chap4_generalLinearSystemODE assembled densely from the closed-form
    Legendre matrices and solved by numpy; also L u and L^T z."""
    rng = np.random.default_rng(10 + p)
    N, tau, lam = 13, 0.37, 1.9
    L = an.dense_L(p, N, tau, lam)
    f = rng.standard_normal(N * (p + 1))
    assert np.allclose(core.direct(p, tau, lam, f), np.linalg.solve(L, f), rtol=1e-12, atol=1e-13)
    assert np.allclose(core.direct(p, tau, lam, f, trans=True), np.linalg.solve(L.T, f),
                       rtol=1e-12, atol=1e-13)
    u = rng.standard_normal(N * (p + 1))
    assert np.allclose(core.apply(p, tau, lam, u), L @ u, rtol=1e-13, atol=1e-13)
    assert np.allclose(core.apply(p, tau, lam, u, trans=True), L.T @ u, rtol=1e-13, atol=1e-13)
    # the initial value enters as the upwind term of slab 1
    u0 = 0.3
    full = core.direct_solve(p, N * tau, lam, u0, f)
    rhs = f.copy()
    rhs[:p + 1] += u0 * (-1.0) ** np.arange(p + 1)
    assert np.allclose(full, np.linalg.solve(L, rhs), rtol=1e-12, atol=1e-13)


def test_operator_depends_on_lambda_tau_only():
    """The slab operator K + lam M_tau depends on lam and tau only through
    z = lam tau (M_tau = tau M_1), so lambda > 0 is the paper's lambda = 1
    with tau -> lam tau."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal(32 * 3)
    a = core.direct(2, 0.01, 7.0, f)
    b = core.direct(2, 0.07, 1.0, f)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Transfers (section 4.2, eqs. chap4_restrictionTime / chap4_prolongationTime)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_galerkin_identity(p):
    """R L_tau P = L_{2 tau}: for coarse trial and test functions the fine jump
    terms inside a coarse slab cancel, so the fine bilinear form restricted to
    coarse functions is the coarse one."""
    Nc, tau, lam = 6, 0.2, 1.3
    P = p + 1
    G = np.zeros((Nc * P, Nc * P))
    for j in range(Nc * P):
        e = np.zeros(Nc * P)
        e[j] = 1.0
        v = core.prolong_add(p, e, np.zeros(2 * Nc * P))
        G[:, j] = core.restrict(p, core.apply(p, tau, lam, v))
    assert np.allclose(G, an.dense_L(p, Nc, 2 * tau, lam), rtol=0, atol=2e-14)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_restriction_of_load_vector(p):
    """R is the transpose of the L2-embedding, so R f_tau = f_{2 tau} exactly
    for load vectors of any f."""
    rng = np.random.default_rng(7)
    a, phi = rng.standard_normal(5), rng.uniform(0, 2 * np.pi, 5)
    fine = gen.fourier_load(p, 64, 4.0, a, phi)
    coarse = gen.fourier_load(p, 32, 4.0, a, phi)
    assert np.allclose(core.restrict(p, fine), coarse, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_prolongation_is_exact_embedding(p):
    """P maps a coarse polynomial to the same function on both fine slabs."""
    rng = np.random.default_rng(8)
    P = p + 1
    e = rng.standard_normal(3 * P)
    v = core.prolong_add(p, e, np.zeros(6 * P)).reshape(6, P)
    x = np.linspace(-1, 1, 7)
    Vx = an.legendre_values(P, x)
    for m in range(3):
        for half, xc in ((0, (x - 1) / 2), (1, (x + 1) / 2)):
            coarse_vals = an.legendre_values(P, xc) @ e[m * P:(m + 1) * P]
            assert np.allclose(Vx @ v[2 * m + half], coarse_vals, atol=1e-14)


def test_transfer_matrices_closed_form():
    """Legendre re-expansion of P_l((xi -+ 1)/2): upper triangular with
    diagonal 2^{-l}; p = 1 gives [[1, -1/2], [0, 1/2]] and [[1, 1/2], [0, 1/2]]."""
    t = core.tables(1, 1.0, 1.0)
    assert np.allclose(t["R1T"], [[1, -0.5], [0, 0.5]], atol=1e-15)
    assert np.allclose(t["R2T"], [[1, 0.5], [0, 0.5]], atol=1e-15)
    t3 = core.tables(3, 1.0, 1.0)
    assert np.allclose(np.diag(t3["R1T"]), 2.0 ** -np.arange(4), atol=1e-15)
    assert np.allclose(np.tril(t3["R1T"], -1), 0, atol=1e-15)


# --------------------------------------------------------------------------
# Smoother (eq. chap4_ODESmoother, Lemmas chap4_lemma4..8)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 3])
def test_jacobi_with_unit_damping_is_nilpotent(p):
    """Section 4.1: for omega = 1 the block Jacobi iteration matrix is strictly
    block lower triangular, so N sweeps from any start give the exact solution."""
    rng = np.random.default_rng(1)
    N, tau, lam = 16, 0.3, 1.0
    f = rng.standard_normal(N * (p + 1))
    u = core.sweeps(p, tau, lam, f, rng.standard_normal(N * (p + 1)), N, omega=1.0)
    assert np.allclose(u, core.direct(p, tau, lam, f), rtol=1e-12, atol=1e-12)


def test_optimal_damping_and_smoothing_bound(golden_dir):
    """Lemma chap4_lemma7: omega* = 1/(1 + alpha^2) (alpha >= 0) or 1, and the
    smoothing factor stays below 1/sqrt(2); Lemma chap4_lemma8 bound
    |alpha| (1 + |alpha|) / (1 + alpha^2) over all frequencies."""
    bound = _golden_const(golden_dir)["smoothing_bound"]
    for p in range(4):
        for z in np.logspace(-6, 6, 25):
            t = core.tables(p, 1.0, z)
            a = t["alpha"]
            assert t["omega"] == pytest.approx(1 / (1 + a * a) if a >= 0 else 1.0, rel=1e-15)
            assert a == pytest.approx(an.alpha_of(p, z), rel=1e-12, abs=1e-15)
            assert an.smoothing_factor(p, z, t["omega"], N=256) <= bound + 1e-12
            _, _, Nm, A = an.slab_closed_form(p, 1.0, z)
            G = np.linalg.solve(A, Nm)
            lemma8 = abs(a) * (1 + abs(a)) / (1 + a * a)
            for th in np.linspace(-np.pi, np.pi, 33):
                S = (1 - t["omega"]) * np.eye(p + 1) + np.exp(-1j * th) * t["omega"] * G
                assert np.max(np.abs(np.linalg.eigvals(S))) <= lemma8 + 1e-12


def test_levels_and_damping_fourier_small():
    """Per-level alpha_l = R(-lam tau_l) and omega_l = omega*(alpha_l) on the
    hierarchy N, N/2, ..., 2 (config-1 sizes)."""
    al, om = core.levels(1, 1024, 10.0, 1.0)
    assert len(al) == 10
    for l in range(10):
        z = 10.0 / (1024 >> l)
        R = (6 - 2 * z) / (6 + 4 * z + z * z)
        assert al[l] == pytest.approx(R, rel=1e-13)
        assert om[l] == pytest.approx(1 / (1 + R * R) if R >= 0 else 1.0, rel=1e-14)


# --------------------------------------------------------------------------
# Two-grid cycle (eq. chap4_errorTwoGridCycle, Theorem chap4_theorem4)
# --------------------------------------------------------------------------

def test_two_grid_closed_form_p0(golden_dir):
    """Section 4.2: p = 0, nu1 = nu2 = 1 with omega*(tau) gives
    rho(M) = 1/(2 + 2 tau + tau^2) <= 1/2."""
    bound = _golden_const(golden_dir)["two_grid_p0_bound"]
    for z in [1e-6, 1e-2, 0.5, 1.0, 4.0, 30.0]:
        rho = an.two_grid_rho(0, z, 1, 1, N=256)
        assert rho == pytest.approx(1.0 / (2 + 2 * z + z * z), rel=1e-10)
        assert rho <= bound


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_symbol_matches_dense_periodic_two_grid(p):
    """Theorem chap4_theorem4 is exact for the time-periodic problem: the
    largest eigenvalue modulus of the dense periodic two-grid operator equals
    the maximum of rho(M^(theta)) over the low frequencies (coarse symbol at
    2 tau)."""
    for z in (0.05, 1.0, 7.0):
        for nu in (1, 2):
            om = an.omega_opt(an.alpha_of(p, z))
            Md = an.dense_two_grid(p, 32, z, nu, nu, om)
            rd = np.max(np.abs(np.linalg.eigvals(Md)))
            rs = an.two_grid_rho(p, z, nu, nu, om, N=32)
            assert rd == pytest.approx(rs, rel=1e-8, abs=1e-13)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("z", [1e-3, 1.0])
@pytest.mark.parametrize("nu", [1, 2])
def test_measured_two_grid_contraction(p, z, nu):
    """Section 4.2 experiment: N = 1024 slabs, f = 0, random start in [0, 1];
    the measured asymptotic residual contraction of the oracle's two-grid cycle
    (tail geometric mean) lies under the Fourier estimate, up to a
    finite-window bias of 1e-5 relative (the last ratios oscillate about the
    estimate by up to that much), and above 0.9 of it."""
    N = 1024
    rng = np.random.default_rng(100 + p)
    opts = core.Opts(nu1=nu, nu2=nu, gamma=1, n_coarse=N // 2)
    u = rng.uniform(0.0, 1.0, N * (p + 1))
    f = np.zeros_like(u)
    r = [np.linalg.norm(core.residual(p, z, 1.0, f, u))]
    while len(r) < 40 and r[-1] > 1e-200 * r[0]:
        u = core.cycles(p, z * N, 1.0, f, u, 1, opts)
        r.append(np.linalg.norm(core.residual(p, z, 1.0, f, u)))
    K = len(r) - 1
    assert K >= 8
    tail = (r[K] / r[K // 2]) ** (1.0 / (K - K // 2))
    est = an.two_grid_rho(p, z, nu, nu, N=N)
    assert 0.9 * est <= tail <= (1.0 + 1e-5) * est


# --------------------------------------------------------------------------
# Multigrid solve, adjoint and mixed precision
# --------------------------------------------------------------------------

def test_vcycle_solve_fourier_small():
    """Stopping rule of section 4.2 (relative residual reduction): the V-cycle
    reaches 1e-10 and the result is within the residual bound of the direct
    solve."""
    inst = gen.fourier_small().instances[0]
    ud = core.direct_solve(1, inst.T, inst.lam, inst.u0, inst.f)
    u, k, rr, hist = core.solve(1, inst.T, inst.lam, inst.u0, inst.f)
    assert rr <= 1e-10 and 5 <= k <= 20
    assert np.all(np.diff(np.log(hist)) < 0)
    assert np.max(np.abs(u - ud)) <= 1e-8 * np.max(np.abs(ud))
    uw, kw, rrw, _ = core.solve(1, inst.T, inst.lam, inst.u0, inst.f, opts=core.Opts(gamma=2))
    assert rrw <= 1e-10 and kw <= k
    assert np.max(np.abs(uw - ud)) <= 1e-8 * np.max(np.abs(ud))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_adjoint_dot_product_and_solves(p):
    """<L u, z> = <u, L^T z>; the backward substitution and the multigrid
    cycle on L^T solve the transposed system."""
    rng = np.random.default_rng(20 + p)
    N, T, lam = 64, 3.0, 2.0
    tau = T / N
    u = rng.standard_normal(N * (p + 1))
    z = rng.standard_normal(N * (p + 1))
    lhs = core.apply(p, tau, lam, u) @ z
    rhs = u @ core.apply(p, tau, lam, z, trans=True)
    assert lhs == pytest.approx(rhs, rel=1e-13)
    g = rng.standard_normal(N * (p + 1))
    zd = core.direct(p, tau, lam, g, trans=True)
    assert np.allclose(core.apply(p, tau, lam, zd, trans=True), g, atol=1e-12)
    zm, k, rr, _ = core.solve_folded(p, T, lam, g, trans=True)
    assert rr <= 1e-10
    assert np.max(np.abs(zm - zd)) <= 1e-8 * np.max(np.abs(zd))


@pytest.mark.parametrize("p", [1, 2])
def test_gradients_against_finite_differences(p):
    """J = 1/2 sum (w_n - y_n)^2 with w_n = u_n(t_n^-): the adjoint gradients
    match central differences (h = 1e-6) of direct forward solves."""
    rng = np.random.default_rng(30 + p)
    N, T, lam, u0 = 32, 2.0, 1.5, 0.8
    tau = T / N
    f = rng.standard_normal(N * (p + 1)) * 0.1
    y = rng.standard_normal(N)

    def J(f_, u0_, lam_):
        u = core.direct_solve(p, T, lam_, u0_, f_)
        return core.adjoint_rhs(p, u, y)[1]

    u = core.direct_solve(p, T, lam, u0, f)
    g, _ = core.adjoint_rhs(p, u, y)
    z = core.direct(p, tau, lam, g, trans=True)
    dlam, du0 = core.gradients(p, tau, lam, u, z)
    h = 1e-6
    fd_lam = (J(f, u0, lam + h) - J(f, u0, lam - h)) / (2 * h)
    fd_u0 = (J(f, u0 + h, lam) - J(f, u0 - h, lam)) / (2 * h)
    d = rng.standard_normal(f.size)
    fd_f = (J(f + h * d, u0, lam) - J(f - h * d, u0, lam)) / (2 * h)
    assert dlam == pytest.approx(fd_lam, rel=1e-6)
    assert du0 == pytest.approx(fd_u0, rel=1e-6)
    assert z @ d == pytest.approx(fd_f, rel=1e-6)


def test_mixed_precision_reference():
    """FP32 inner cycle with FP64 residual / coarsest solve / outer update
    reaches 1e-10 with (about) as many cycles as FP64 and the same solution
    to the tolerance."""
    w = gen.long_horizon(B=1, N=1 << 12, T=1e4 * 2 ** -12)
    inst = w.instances[0]
    u64, k64, rr64, _ = core.solve(3, inst.T, inst.lam, inst.u0, inst.f)
    um, km, rrm, _ = core.solve_mixed(3, inst.T, inst.lam, inst.u0, inst.f)
    assert rrm <= 1e-10 and abs(km - k64) <= 1
    ud = core.direct_solve(3, inst.T, inst.lam, inst.u0, inst.f)
    assert np.max(np.abs(um - ud)) <= 1e-8 * np.max(np.abs(ud))
