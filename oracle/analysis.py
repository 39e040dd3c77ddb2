"""NumPy tools from the paper's analysis, used to pin the C oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is built independently of ``tmg_oracle.c``: the slab matrices
come from their closed forms for the Legendre basis (not from quadrature),
the transfer matrices from Legendre series re-expansion (not from the
projection integrals), so that agreement between the two is evidence, not
tautology.

* :func:`pade` -- the (p, p+1) subdiagonal Pade approximant of e^z from its
  printed coefficients (section 2.2, remark after Theorem chap4_theorem2a);
* :func:`radau_ia` -- left Radau nodes and weights (c_1 = 0), section 2.2;
* :func:`slab_closed_form`, :func:`transfer_series`, :func:`dense_L`,
  :func:`dense_R` -- dense global operators (eqs. chap4_equationLinearSystemODE,
  chap4_circulantMatrix, chap4_restrictionTime, chap4_prolongationTime);
* :func:`two_grid_symbol`, :func:`two_grid_rho` -- the 2P x 2P two-grid
  iteration matrix of Theorem chap4_theorem4 and its maximum spectral radius
  over the low frequencies (the asymptotic two-grid convergence factor);
* :func:`smoothing_factor` -- max over high frequencies of rho(S(theta)).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def pade(num, den, z):
    """Evaluate sum(num[i] z^i) / sum(den[i] z^i)."""
    z = np.asarray(z, dtype=np.complex128 if np.iscomplexobj(z) else np.float64)
    return np.polyval(np.asarray(num, float)[::-1], z) / np.polyval(np.asarray(den, float)[::-1], z)


def radau_ia(s: int):
    """Left Radau quadrature (c_1 = 0) with s points on [0, 1], exact to
    degree 2s - 2 (order 2s - 1).  Nodes: zeros of P_s(2x-1) + P_{s-1}(2x-1)."""
    coef = np.zeros(s + 1)
    coef[s] = 1.0
    coef[s - 1] += 1.0
    y = np.sort(np.real(npleg.legroots(coef)))
    c = (y + 1.0) / 2.0
    c[0] = 0.0
    V = np.vander(c, s, increasing=True).T          # V[j, i] = c_i^j
    b = np.linalg.solve(V, 1.0 / np.arange(1, s + 1))
    return c, b


def legendre_values(P: int, x):
    """Matrix V[i, k] = P_k(x_i) for k < P."""
    x = np.asarray(x, dtype=float)
    return np.stack([npleg.legval(x, np.eye(P)[k]) for k in range(P)], axis=-1)


def slab_closed_form(p: int, tau: float, lam: float):
    """K, M, N, A for the Legendre basis in closed form:
    K[k,l] = 1 - 2[l < k and k + l odd], M = tau diag(1/(2k+1)), N = v_L 1^T
    with v_L[k] = (-1)^k, A = K + lam M."""
    P = p + 1
    k = np.arange(P)
    K = np.ones((P, P)) - 2.0 * ((k[None, :] < k[:, None]) & ((k[:, None] + k[None, :]) % 2 == 1))
    M = np.diag(tau / (2.0 * k + 1.0))
    vL = (-1.0) ** k
    N = np.outer(vL, np.ones(P))
    return K, M, N, K + lam * M


def transfer_series(p: int):
    """R1T[:, l] / R2T[:, l]: Legendre coefficients of the coarse basis function
    P_l restricted to the first / second fine slab, in fine coordinates:
    P_l((xi - 1)/2) and P_l((xi + 1)/2)."""
    from numpy.polynomial import Legendre, Polynomial
    P = p + 1
    R1T = np.zeros((P, P))
    R2T = np.zeros((P, P))
    for l in range(P):
        pl = Legendre.basis(l).convert(kind=Polynomial)   # power series of P_l(y)
        for shift, R in ((-1.0, R1T), (1.0, R2T)):
            comp = pl(Polynomial([shift / 2.0, 0.5]))      # P_l((xi + shift)/2)
            c = comp.convert(kind=Legendre).coef
            R[:len(c), l] = c
    return R1T, R2T


def dense_L(p: int, N: int, tau: float, lam: float, periodic: bool = False):
    """Global matrix I (x) A + U_N (x) N (or the circulant U~_N if periodic)."""
    _, _, Nm, A = slab_closed_form(p, tau, lam)
    U = -np.eye(N, k=-1)
    if periodic:
        U[0, N - 1] = -1.0
    return np.kron(np.eye(N), A) + np.kron(U, Nm)


def dense_R(p: int, Nc: int):
    """Restriction R (Nc P x 2 Nc P): block row m = [.. R_1 R_2 ..] at fine
    slabs 2m, 2m+1; the prolongation is its transpose."""
    P = p + 1
    R1T, R2T = transfer_series(p)
    R = np.zeros((Nc * P, 2 * Nc * P))
    for m in range(Nc):
        R[m * P:(m + 1) * P, (2 * m) * P:(2 * m + 1) * P] = R1T.T
        R[m * P:(m + 1) * P, (2 * m + 1) * P:(2 * m + 2) * P] = R2T.T
    return R


def omega_opt(alpha: float) -> float:
    """Lemma chap4_lemma7."""
    return 1.0 / (1.0 + alpha * alpha) if alpha >= 0 else 1.0


def alpha_of(p: int, z: float) -> float:
    """alpha = the nonzero eigenvalue of A^{-1} N (Lemma chap4_theorem2),
    computed as 1^T A^{-1} v_L from the closed-form matrices (tau = 1)."""
    _, _, Nm, A = slab_closed_form(p, 1.0, z)
    return float(np.ones(p + 1) @ np.linalg.solve(A, Nm[:, 0]))


def two_grid_symbol(p: int, z: float, nu1: int, nu2: int, omega: float, theta: float):
    """The 2P x 2P iteration matrix M^(theta) of Theorem chap4_theorem4 for the
    fine step z = lambda tau (coarse step 2z), theta in the low frequencies.
    gamma(theta) = theta - sign(theta) pi, with gamma(0) = -pi (the harmonic
    partner of the zero mode)."""
    P = p + 1
    _, _, Nm, A = slab_closed_form(p, 1.0, z)
    _, _, _, Ac = slab_closed_form(p, 1.0, 2.0 * z)
    R1T, R2T = transfer_series(p)
    I = np.eye(P)

    def Lhat(A_, th):
        return A_ - np.exp(-1j * th) * Nm

    def Shat(th):
        return (1 - omega) * I + np.exp(-1j * th) * omega * np.linalg.solve(A, Nm)

    def Rhat(th):
        return np.exp(-1j * th) * R1T.T + R2T.T

    def Phat(th):
        return 0.5 * (np.exp(1j * th) * R1T + R2T)

    g = theta - np.sign(theta) * np.pi if theta != 0 else -np.pi
    Lf = np.block([[Lhat(A, theta), np.zeros((P, P))], [np.zeros((P, P)), Lhat(A, g)]])
    Pm = np.vstack([Phat(theta), Phat(g)])
    Rm = np.hstack([Rhat(theta), Rhat(g)])
    K = np.eye(2 * P) - Pm @ np.linalg.solve(Lhat(Ac, 2 * theta), Rm @ Lf)
    S = lambda th, nu: np.linalg.matrix_power(Shat(th), nu)
    S1 = np.block([[S(theta, nu1), np.zeros((P, P))], [np.zeros((P, P)), S(g, nu1)]])
    S2 = np.block([[S(theta, nu2), np.zeros((P, P))], [np.zeros((P, P)), S(g, nu2)]])
    return S2 @ K @ S1


def two_grid_rho(p: int, z: float, nu1: int, nu2: int, omega: float | None = None,
                 N: int = 1024) -> float:
    """Asymptotic two-grid factor: max over theta_k = 2 k pi / N,
    k = 1 - N/4 .. N/4, of rho(M^(theta_k))."""
    if omega is None:
        omega = omega_opt(alpha_of(p, z))
    ks = np.arange(1 - N // 4, N // 4 + 1)
    best = 0.0
    for k in ks:
        th = 2.0 * np.pi * k / N
        ev = np.linalg.eigvals(two_grid_symbol(p, z, nu1, nu2, omega, th))
        best = max(best, float(np.max(np.abs(ev))))
    return best


def smoothing_factor(p: int, z: float, omega: float, N: int = 1024) -> float:
    """max over high frequencies of rho(S(theta, omega)) (Lemma chap4_lemma4)."""
    _, _, Nm, A = slab_closed_form(p, 1.0, z)
    G = np.linalg.solve(A, Nm)
    best = 0.0
    for k in range(1 - N // 2, N // 2 + 1):
        th = 2.0 * np.pi * k / N
        if -np.pi / 2 < th <= np.pi / 2:
            continue
        S = (1 - omega) * np.eye(p + 1) + np.exp(-1j * th) * omega * G
        best = max(best, float(np.max(np.abs(np.linalg.eigvals(S)))))
    return best


def dense_two_grid(p: int, N: int, z: float, nu1: int, nu2: int, omega: float,
                   periodic: bool = True):
    """Dense two-grid error propagator S^nu2 (I - P Lc^{-1} R L) S^nu1 on N
    fine slabs of length z (lambda = 1), coarse operator rediscretised at 2z."""
    L = dense_L(p, N, z, 1.0, periodic)
    Lc = dense_L(p, N // 2, 2 * z, 1.0, periodic)
    R = dense_R(p, N // 2)
    _, _, _, A = slab_closed_form(p, z, 1.0)
    D = np.kron(np.eye(N), A)
    S = np.eye(N * (p + 1)) - omega * np.linalg.solve(D, L)
    K = np.eye(N * (p + 1)) - R.T @ np.linalg.solve(Lc, R @ L)
    return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)


def level_steps(N: int, n_coarse: int):
    """Slab counts N, N/2, ..., n_coarse of the hierarchy (N = n_coarse 2^k)."""
    out = [N]
    while out[-1] > n_coarse:
        assert out[-1] % 2 == 0
        out.append(out[-1] // 2)
    assert out[-1] == n_coarse
    return out


def dense_cycle(p: int, N: int, T: float, lam: float, nu1: int, nu2: int, gamma: int,
                n_coarse: int = 2, omega: float | None = None, trans: bool = False,
                periodic: bool = False):
    """Dense error propagator M_0 of one multigrid cycle on level 0.

    The two-grid error propagator of eq. chap4_errorTwoGridCycle,
    S^nu2 (I - P L_c^{-1} R L) S^nu1, with the exact coarse solve replaced by
    gamma cycles from a zero initial guess on the coarse error equation,
    which leaves the coarse error M_{l+1}^gamma L_{l+1}^{-1} R L e:

        M_l = S_l^nu2 (I - P (I - M_{l+1}^gamma) L_{l+1}^{-1} R L_l) S_l^nu1,

    M = 0 on the coarsest level (an exact solve).  L_l is rediscretised at
    tau_l = T / N_l, S_l = I - omega_l D_l^{-1} L_l is damped block Jacobi
    (eq. chap4_ODESmoother) with omega_l from Lemma chap4_lemma7 at
    alpha(lam tau_l) (or the fixed omega), R the restriction of
    eq. chap4_restrictionTime and P = R^T.  trans: the same cycle applied to
    L^T (smoother I - omega D^{-T} L^T, the same R and P).  periodic: every
    level's operator is the circulant one of
    eq. chap4_equationLinearSystemODEPeriodic.  Every matrix comes from the
    closed forms above, none from the C oracle."""
    Ns = level_steps(N, n_coarse)
    P_ = p + 1

    def Lmat(Nl):
        L = dense_L(p, Nl, T / Nl, lam, periodic)
        return L.T if trans else L

    def smoother(Nl):
        L = Lmat(Nl)
        _, _, _, A = slab_closed_form(p, T / Nl, lam)
        D = np.kron(np.eye(Nl), A.T if trans else A)
        om = omega_opt(alpha_of(p, lam * T / Nl)) if omega is None else omega
        return np.eye(Nl * P_) - om * np.linalg.solve(D, L)

    def M(l):
        Nl = Ns[l]
        if l == len(Ns) - 1:
            return np.zeros((Nl * P_, Nl * P_))
        Lf, Lc = Lmat(Nl), Lmat(Ns[l + 1])
        R = dense_R(p, Ns[l + 1])
        Mc = np.linalg.matrix_power(M(l + 1), gamma)
        K = np.eye(Nl * P_) - R.T @ (np.eye(Mc.shape[0]) - Mc) @ np.linalg.solve(Lc, R @ Lf)
        S = smoother(Nl)
        return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)

    return M(0)
