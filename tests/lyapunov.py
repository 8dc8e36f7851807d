"""Linear fluctuation theory of the lattice scheme, per wavevector.

Test helper, independent of the oracle's code: it linearises the FLBE update
(Eqs. (84)-(87)) about the homogeneous rest state f_i = w_i rho0_sigma and
writes one time step for a Fourier mode k as

    x(n+1) = P(k) [ (I + C(k)) x(n) + eta(n) ],   <eta eta^H> = Xi,

x = (delta f_1, delta f_2) in C^{2Q}, P(k) = diag(exp(-i k.c_i)) (streaming),
C(k) the linearised collision and Xi the per-site covariance of the noise of
Eq. (74) mapped to populations.  The stationary covariance solves the discrete
Lyapunov equation Sigma = M Sigma M^H + P Xi P^H with M = P (I + C): the
lattice counterpart of Eq. (13) of Sec. II.  Because the noise is white in
space, Sigma is directly the equal-time structure factor normalised per site.

The linearised collision is written in population space without a mode basis
(completeness, Eq. (79), turns the sum over the non-hydrodynamic modes into
f - w rho - 3 w c.j), so it does not depend on the choice of ghost modes:
  f*_i = f_i - lambda_sigma (f_i - w_i rho - 3 w_i c_i.j) + 3 w_i c_i.R,
  R = lambda_d (rho0 u - j) + (1 - lambda_d/2) F,
  u = (j_1 + j_2)/rho_t0 + (F_1 + F_2)/(2 rho_t0),
  F_sigma = rho0_sigma a_sigma,  a_sigma(k) = -G g(k) delta rho_sigma'(k),
  g(k) = sum_i w_i c_i exp(i k.c_i);
the equilibrium and second-order forcing terms are quadratic and drop out.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import linalg


def lattice(name: str):
    """(c [Q, D] float, w [Q]) for "d2q9" or "d3q19" with c_s^2 = 1/3."""
    if name == "d2q9":
        c = [v for v in itertools.product((-1, 0, 1), repeat=2)]
    elif name == "d3q19":
        c = [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(abs(x) for x in v) <= 2]
    else:
        raise ValueError(name)
    c = np.array(c, dtype=float)
    c2 = (c ** 2).sum(1)
    if name == "d2q9":
        w = np.select([c2 == 0, c2 == 1, c2 == 2], [4 / 9, 1 / 9, 1 / 36])
    else:
        w = np.select([c2 == 0, c2 == 1, c2 == 2], [1 / 3, 1 / 18, 1 / 36])
    return c, w


class LinearFLBE:
    def __init__(self, name="d2q9", rho0=(1.0, 1.0), tau=(1.0, 1.0), tau_d=1.0, G=0.0, kT=1e-5,
                 sdf=True):
        self.c, self.w = lattice(name)
        self.Q, self.D = self.c.shape
        self.rho0 = np.array(rho0, float)
        self.lam = 1.0 / np.array(tau, float)
        self.lam_d = 1.0 / tau_d
        self.G = G
        self.kT = kT
        self.sdf = sdf

    def operators(self, k):
        """(M, Xi_streamed) for the wavevector k (length-D array)."""
        c, w, Q = self.c, self.w, self.Q
        k = np.asarray(k, float)
        phase = np.exp(1j * (c @ k))
        P = np.diag(np.conj(phase))              # streaming: f(r + c) <- f*(r)
        g = (w[:, None] * c * phase[:, None]).sum(0)  # sum_i w_i c_i e^{i k.c_i}
        rt = self.rho0.sum()
        ones = np.ones(Q)
        # linear functionals on one species' populations
        Erho = ones[None, :]                     # 1 x Q
        Ej = c.T                                 # D x Q
        # build C as a 2Q x 2Q matrix column by column (action on unit vectors)
        n = 2 * Q
        A = np.zeros((n, n), complex)
        for col in range(n):
            x = np.zeros(n, complex)
            x[col] = 1.0
            f = [x[:Q], x[Q:]]
            rho = [(Erho @ fs)[0] for fs in f]
            j = [Ej @ fs for fs in f]
            a = [-self.G * g * rho[1], -self.G * g * rho[0]]
            F = [self.rho0[s] * a[s] for s in range(2)]
            u = (j[0] + j[1]) / rt + 0.5 * (F[0] + F[1]) / rt
            out = []
            for s in range(2):
                R = self.lam_d * (self.rho0[s] * u - j[s]) + (1 - 0.5 * self.lam_d) * F[s]
                neq = f[s] - w * rho[s] - 3 * w * (c @ j[s])
                out.append(f[s] - self.lam[s] * neq + 3 * w * (c @ R))
            A[:, col] = np.concatenate(out)
        M = np.kron(np.eye(2), P) @ A
        # noise covariance in population space
        mu = 3.0 * self.kT
        Xi = np.zeros((n, n))
        Pi = np.diag(w) - np.outer(w, w) - 3 * np.outer(w, w) * (c @ c.T)
        for s in range(2):
            Xi[s * Q:(s + 1) * Q, s * Q:(s + 1) * Q] = (2 * self.lam[s] - self.lam[s] ** 2) * mu * self.rho0[s] * Pi
        if self.sdf:
            sd2 = (2 * self.lam_d - self.lam_d ** 2) * self.kT * self.rho0[0] * self.rho0[1] / rt
            B = 3 * w[:, None] * c                  # Q x D, f_i += 3 w_i c_i . xi
            blk = sd2 * (B @ B.T)
            Xi[:Q, :Q] += blk
            Xi[Q:, Q:] += blk
            Xi[:Q, Q:] -= blk
            Xi[Q:, :Q] -= blk
        PP = np.kron(np.eye(2), P)
        return M, PP @ Xi @ PP.conj().T

    def covariance(self, k):
        """Sigma = M Sigma M^H + N, solved directly as a linear system in
        vec(Sigma) (I - conj(M) kron M) vec(Sigma) = vec(N)."""
        M, N = self.operators(k)
        n = M.shape[0]
        A = np.eye(n * n) - np.kron(np.conj(M), M)
        vecS = linalg.solve(A, N.reshape(-1, order="F"))
        S = vecS.reshape(n, n, order="F")
        return 0.5 * (S + S.conj().T)

    def observables(self, k):
        """Linear functionals e (complex, 2Q) with X_hat(k) = e . x(k)."""
        c, w, Q = self.c, self.w, self.Q
        k = np.asarray(k, float)
        phase = np.exp(1j * (c @ k))
        g = (w[:, None] * c * phase[:, None]).sum(0)
        z = np.zeros(Q)
        rt = self.rho0.sum()
        e = {"rho1": np.concatenate([np.ones(Q), z]), "rho2": np.concatenate([z, np.ones(Q)])}
        for al in range(self.D):
            e[f"j1_{al}"] = np.concatenate([c[:, al], z])
            e[f"j2_{al}"] = np.concatenate([z, c[:, al]])
            # physical barycentric velocity (J_bar + F_t/2)/rho_t0
            F1 = self.rho0[0] * (-self.G * g[al]) * e["rho2"]
            F2 = self.rho0[1] * (-self.G * g[al]) * e["rho1"]
            e[f"vb_{al}"] = (e[f"j1_{al}"] + e[f"j2_{al}"] + 0.5 * (F1 + F2)) / rt
        return e

    def structure_factors(self, k):
        """Dict of S_XY(k) = <X_hat conj(Y_hat)> / N for the stationary state."""
        S = self.covariance(k)
        e = self.observables(k)

        def s(a, b):
            return (e[a] @ S @ np.conj(e[b])).real

        out = {"rho1rho1": s("rho1", "rho1"), "rho2rho2": s("rho2", "rho2"),
               "rho1rho2": s("rho1", "rho2")}
        out["j1j1"] = np.mean([s(f"j1_{a}", f"j1_{a}") for a in range(self.D)])
        out["j1j2"] = np.mean([s(f"j1_{a}", f"j2_{a}") for a in range(self.D)])
        out["vbvb"] = np.mean([s(f"vb_{a}", f"vb_{a}") for a in range(self.D)])
        return out

    def mode_variance_ratios(self, T, N, L=13):
        """Stationary <m_a^2> / (N_a mu rho0_s) of the pre-collision modes
        m_a = sum_i T_ai f_i of each species ([2][Q]), averaged over the
        wavevectors of an L^D grid with k = 0 left out: the equipartition
        check of Sec. VI A including the corrections the mean-field force
        brings at G > 0 (exactly 1 at G = 0).  L is odd so that no grid point
        has a component pi, where some lattice modes do not relax and the
        stationary covariance is undefined.  T's columns follow this module's
        velocity order."""
        if L % 2 == 0:
            raise ValueError("use an odd grid size")
        Q, D = self.Q, self.D
        ks = 2 * np.pi * np.fft.fftfreq(L)
        grid = np.stack(np.meshgrid(*([ks] * D), indexing="ij"), -1).reshape(-1, D)
        acc = np.zeros((2, Q))
        cnt = 0
        for k in grid:
            if not np.any(k):
                continue
            S = self.covariance(k)
            for s in range(2):
                blk = S[s * Q:(s + 1) * Q, s * Q:(s + 1) * Q]
                acc[s] += np.real(np.einsum("ai,ij,aj->a", T, blk, T))
            cnt += 1
        return acc / cnt / (np.asarray(N)[None, :] * 3.0 * self.kT * self.rho0[:, None])

    def spectral_radius(self, k):
        M, _ = self.operators(k)
        return np.max(np.abs(np.linalg.eigvals(M)))

    def eigenvalues(self, k):
        M, _ = self.operators(k)
        return np.linalg.eigvals(M)


class LinearMultiFLBE:
    """The same linearisation for N species (Apps. C and D): pair couplings
    G[N][N] (a_sigma(k) = -g(k) sum_s' G_sigma,s' delta rho_s'(k)), u =
    (sum j + sum F / 2) / rho_t0, and the momentum noise with covariance
    (2 lambda_d - lambda_d^2) k_B T (rho_sigma delta - rho_sigma rho_s' / rho_t)
    per component, mapped to populations.  Uses the covariance itself, not
    any way of sampling it."""

    def __init__(self, name="d2q9", rho0=(1.0, 1.0, 1.0), tau=(1.0, 1.0, 1.0), tau_d=1.0, G=None, kT=1e-5,
                 sdf=True):
        self.c, self.w = lattice(name)
        self.Q, self.D = self.c.shape
        self.rho0 = np.array(rho0, float)
        self.N = len(self.rho0)
        self.lam = 1.0 / np.array(tau, float)
        self.lam_d = 1.0 / tau_d
        self.G = np.zeros((self.N, self.N)) if G is None else np.array(G, float)
        self.kT = kT
        self.sdf = sdf

    def operators(self, k):
        c, w, Q, NS = self.c, self.w, self.Q, self.N
        k = np.asarray(k, float)
        phase = np.exp(1j * (c @ k))
        P = np.diag(np.conj(phase))
        g = (w[:, None] * c * phase[:, None]).sum(0)
        rt = self.rho0.sum()
        n = NS * Q
        A = np.zeros((n, n), complex)
        for col in range(n):
            x = np.zeros(n, complex)
            x[col] = 1.0
            f = [x[s * Q:(s + 1) * Q] for s in range(NS)]
            rho = np.array([fs.sum() for fs in f])
            j = [c.T @ fs for fs in f]
            F = [self.rho0[s] * (-g * (self.G[s] @ rho)) for s in range(NS)]
            u = sum(j) / rt + 0.5 * sum(F) / rt
            out = []
            for s in range(NS):
                R = self.lam_d * (self.rho0[s] * u - j[s]) + (1 - 0.5 * self.lam_d) * F[s]
                neq = f[s] - w * rho[s] - 3 * w * (c @ j[s])
                out.append(f[s] - self.lam[s] * neq + 3 * w * (c @ R))
            A[:, col] = np.concatenate(out)
        PP = np.kron(np.eye(NS), P)
        M = PP @ A
        mu = 3.0 * self.kT
        Xi = np.zeros((n, n))
        Pi = np.diag(w) - np.outer(w, w) - 3 * np.outer(w, w) * (c @ c.T)
        for s in range(NS):
            Xi[s * Q:(s + 1) * Q, s * Q:(s + 1) * Q] = (2 * self.lam[s] - self.lam[s] ** 2) * mu * self.rho0[s] * Pi
        if self.sdf:
            B = 3 * w[:, None] * c
            K = (2 * self.lam_d - self.lam_d ** 2) * self.kT * (np.diag(self.rho0) - np.outer(self.rho0, self.rho0) / rt)
            Xi += np.kron(K, B @ B.T)
        return M, PP @ Xi @ PP.conj().T

    def covariance(self, k):
        M, N = self.operators(k)
        n = M.shape[0]
        vecS = linalg.solve(np.eye(n * n) - np.kron(np.conj(M), M), N.reshape(-1, order="F"))
        S = vecS.reshape(n, n, order="F")
        return 0.5 * (S + S.conj().T)

    def density_structure(self, k):
        """S_rho_sigma rho_s'(k), N x N."""
        Q = self.Q
        E = np.kron(np.eye(self.N), np.ones((1, Q)))
        return (E @ self.covariance(k) @ E.T).real

    def momentum_structure(self, k):
        """S_j_sigma j_s'(k) averaged over the D components, N x N."""
        Q, c = self.Q, self.c
        S = self.covariance(k)
        out = np.zeros((self.N, self.N))
        for al in range(self.D):
            E = np.kron(np.eye(self.N), c[:, al][None, :])
            out += (E @ S @ E.T).real
        return out / self.D

    def spectral_radius(self, k):
        M, _ = self.operators(k)
        return np.max(np.abs(np.linalg.eigvals(M)))


def appendix_structure_factor(k_mag, G, rho0, kT, cs2=1.0 / 3.0):
    """Density structure factors of the homogeneous multicomponent mixture,
    from the self-consistency condition of App. D (mu alpha + Gamma R alpha
    + Gamma = 0) inserted into App. C's S = mu R + R Gamma R, which gives
    S(k) = mu (R^-1 + alpha(k))^-1, R = diag(rho0), alpha = G sin k / k
    (lattice form along an axis, Sec. VI A); for two species this is
    Eq. (57)."""
    mu = kT / cs2
    alpha = np.asarray(G, float) * np.sinc(k_mag / np.pi)
    return mu * np.linalg.inv(np.diag(1.0 / np.asarray(rho0, float)) + alpha)


def eq57(k_mag, G, kT, rho0=1.0, rho0p=1.0, cs2=1.0 / 3.0):
    """Eq. (57) with the lattice alpha(k) = G sin k / k for k along an axis
    (Sec. VI A): S_rho_rho and S_rho_rho'."""
    k_mag = np.asarray(k_mag, float)
    alpha = G * np.sinc(k_mag / np.pi)
    den = 1.0 - rho0 * rho0p * alpha ** 2
    return kT / cs2 * rho0 / den, -kT / cs2 * rho0 * rho0p * alpha / den
