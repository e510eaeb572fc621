"""A second, independent transcription of one time step of the ternary colour-gradient
LBM (arXiv:1808.08555, Sec. 2), in NumPy, FP64.

TEST INFRASTRUCTURE ONLY: the test suite is its only user.  It is written straight from the
paper's displays, as whole-lattice array expressions, and shares nothing with the C oracle
(``lbm3_oracle.c``) beyond the readings of the paper that both must take (the guard on
|G_kl|, the snap of g(X) at |X| -> 1, the choice of the third fluid in X_kl, the triangle
test of the comparison laws).  Where the C oracle groups a sum one way, this file takes the
printed form: the difference of Eq. (12) as the full nine-term sum, the stress of Eq. (7)
as the ordered double sum with its factor 1/2, Eq. (13) as the ordered sum over l != k,
IEEE division everywhere.  Its purpose is to pin the C oracle's constants and stages that no
closed form fixes (the 35 of C_t, the 10^6 of C_kl, the comparison laws, the perturbation
operator) by agreement of two codes written apart.

Layout: the post-streaming state ``f[k, i, y, x]`` (fluids k = red, green, blue; D2Q9
direction i), periodic in x and y; ``sigma = (sigma_rg, sigma_rb, sigma_gb)``.
"""
from __future__ import annotations

import math

import numpy as np

# D2Q9 (Sec. 2, after Eq. 3): e_0 = 0, e_{1,3} = (+-1, 0), e_{2,4} = (0, +-1),
# e_{5,7} = (+-1, +-1), e_{6,8} = (-+1, +-1); weights 4/9, 1/9, 1/36; c_s^2 = 1/3.
E = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))
W = (4.0 / 9.0,) + (1.0 / 9.0,) * 4 + (1.0 / 36.0,) * 4
CS2 = 1.0 / 3.0
# perturbation operator, Eq. (5): the B_i the paper quotes
B = (-4.0 / 27.0,) + (2.0 / 27.0,) * 4 + (5.0 / 108.0,) * 4
GUARD = 1e-12  # |G_kl| at or below which n_kl is taken as 0 (the paper leaves it undefined)
LAWS = ("paper", "spencer", "leclaire", "constant")


def _sigma(sigma, k, l):
    """sigma_kl for an unordered pair of distinct fluids."""
    a, b = min(k, l), max(k, l)
    return {(0, 1): sigma[0], (0, 2): sigma[1], (1, 2): sigma[2]}[(a, b)]


def _at(phi, e):
    """phi(x + e) on the periodic lattice (arrays indexed [..., y, x])."""
    return np.roll(phi, shift=(-e[1], -e[0]), axis=(-2, -1))


def derivative(phi):
    """Eq. (12): d_alpha phi(x) = (1/c_s^2) sum_i w_i phi(x + e_i) e_i,alpha, all nine terms."""
    dx = np.zeros_like(phi)
    dy = np.zeros_like(phi)
    for i in range(9):
        val = _at(phi, E[i])
        dx = dx + W[i] * val * E[i][0]
        dy = dy + W[i] * val * E[i][1]
    return dx / CS2, dy / CS2


def X_of(sigma, k, l):
    """Eq. (18), with m the fluid other than k and l."""
    m = 3 - k - l
    smk, sml, skl = _sigma(sigma, m, k), _sigma(sigma, m, l), _sigma(sigma, k, l)
    return (smk ** 2 + sml ** 2 - skl ** 2) / (2.0 * smk * sml)


def g_of(X):
    """Eq. (20), with |X| within 1e-12 of 1 taken as exactly +-1."""
    if X <= -1.0 + 1e-12:
        return 1.0
    if X >= 1.0 - 1e-12:
        return -1.0
    s = math.sin(math.acos(X))
    return 1.0 - s if X < 0.0 else s - 1.0


def _phi(sigma, k, l):
    """phi_kl of Eq. (14): the Neumann angle opposite sigma_kl (cosine clamped to [-1, 1])."""
    return math.acos(min(1.0, max(-1.0, X_of(sigma, k, l))))


def beta_field(law, sigma, beta0, k, l, rho_r, rho_g, rho_b, rho):
    """beta_kl over the lattice for the chosen segregation law: the proposed law of
    Eqs. (19)-(20), or Eq. (15) (Spencer et al.), Eq. (16) (Leclaire et al.), Eq. (17)."""
    k, l = min(k, l), max(k, l)
    prod = rho_r * rho_g * rho_b / rho ** 3
    if law == "paper":
        return beta0 + beta0 * np.minimum(35.0 * prod, 1.0) * g_of(X_of(sigma, k, l))
    if law == "constant":
        return beta0 + 0.0 * rho
    if law == "spencer":
        if (k, l) == (0, 1):
            return beta0 + 0.0 * rho
        other = (1, 2) if (k, l) == (0, 2) else (0, 2)  # beta_rb takes phi_gb, beta_gb takes phi_rb
        return beta0 * (1.0 + 27.0 * prod * (math.sin(_phi(sigma, *other)) - 1.0))
    if law == "leclaire":
        pairs = [(0, 1), (0, 2), (1, 2)]
        if not all(abs(X_of(sigma, a, b)) < 1.0 - 1e-12 for a, b in pairs):
            return beta0 + 0.0 * rho  # no Neumann triangle
        phis = [_phi(sigma, a, b) for a, b in pairs]
        big = max(phis)
        largest = pairs[phis.index(big)]  # the first of equal maxima
        if (k, l) == largest:
            return beta0 + 0.0 * rho
        Ct = np.minimum(35.0 * prod, 1.0)
        return beta0 + beta0 * Ct * (math.sin(math.pi - big - _phi(sigma, k, l)) - 1.0)
    raise ValueError(law)


def step(f, sigma, tau, rho0=(1.0, 1.0, 1.0), beta0=0.7, law="paper", forcing="guo"):
    """One collision, recolouring and streaming step of the post-streaming state f[3, 9, ny, nx]."""
    f = np.asarray(f, dtype=np.float64)
    rho_k = [f[k].sum(axis=0) for k in range(3)]           # rho_k = sum_i f_{i,k}
    rho = rho_k[0] + rho_k[1] + rho_k[2]                    # rho = sum_k rho_k
    ftot = f[0] + f[1] + f[2]                               # f_i = sum_k f_{i,k}
    c = [rho_k[k] / rho for k in range(3)]
    grad = [derivative(c[k]) for k in range(3)]

    # colour gradients, unit normals and concentration factors of every ordered pair
    G, n, mag, C = {}, {}, {}, {}
    for k in range(3):
        for l in range(3):
            if l == k:
                continue
            Gx = c[l] * grad[k][0] - c[k] * grad[l][0]
            Gy = c[l] * grad[k][1] - c[k] * grad[l][1]
            m = np.sqrt(Gx * Gx + Gy * Gy)
            ok = m > GUARD
            safe = np.where(ok, m, 1.0)
            G[k, l] = (Gx, Gy)
            mag[k, l] = np.where(ok, m, 0.0)
            n[k, l] = (np.where(ok, Gx / safe, 0.0), np.where(ok, Gy / safe, 0.0))
            C[k, l] = np.minimum(1e6 * rho_k[k] * rho_k[l] / (rho0[k] * rho0[l]), 1.0)

    # relaxation time from the harmonic viscosity mean, Eqs. (10)-(11)
    nu_k = [(tau[k] - 0.5) * CS2 for k in range(3)]
    nu = rho / (rho_k[0] / nu_k[0] + rho_k[1] / nu_k[1] + rho_k[2] / nu_k[2])
    tau_f = nu / CS2 + 0.5

    if forcing == "guo":
        # Eq. (7): F = sum_k sum_{l != k} div[(sigma_kl C_kl / 2) |G_kl| (I - n_kl n_kl)]
        S = [[np.zeros_like(rho) for _ in range(2)] for _ in range(2)]
        for (k, l), (nx_, ny_) in n.items():
            a = _sigma(sigma, k, l) * C[k, l] / 2.0 * mag[k, l]
            nn = ((nx_ * nx_, nx_ * ny_), (ny_ * nx_, ny_ * ny_))
            for p in range(2):
                for q in range(2):
                    S[p][q] = S[p][q] + a * ((1.0 if p == q else 0.0) - nn[p][q])
        Fx = derivative(S[0][0])[0] + derivative(S[1][0])[1]  # d_x S_xx + d_y S_yx
        Fy = derivative(S[0][1])[0] + derivative(S[1][1])[1]  # d_x S_xy + d_y S_yy
    else:
        Fx = np.zeros_like(rho)
        Fy = np.zeros_like(rho)

    # velocity with the half force, Eq. (9)
    mx = sum(ftot[i] * E[i][0] for i in range(9))
    my = sum(ftot[i] * E[i][1] for i in range(9))
    ux = (mx + 0.5 * Fx) / rho
    uy = (my + 0.5 * Fy) / rho
    uu = ux * ux + uy * uy

    fdag = np.empty_like(ftot)
    for i in range(9):
        eu = E[i][0] * ux + E[i][1] * uy
        feq = W[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))  # Eq. (3)
        omega = -(ftot[i] - feq) / tau_f                                                     # Eq. (2)
        if forcing == "guo":
            # Eq. (8)
            ax = (E[i][0] - ux) / CS2 + eu / (CS2 * CS2) * E[i][0]
            ay = (E[i][1] - uy) / CS2 + eu / (CS2 * CS2) * E[i][1]
            phi = W[i] * (1.0 - 1.0 / (2.0 * tau_f)) * (ax * Fx + ay * Fy)
        else:
            # Eqs. (4)-(5), A_kl = A_lk = 9 sigma_kl / (2 tau_f)
            phi = np.zeros_like(rho)
            for (k, l), (Gx, Gy) in G.items():
                A = 9.0 * _sigma(sigma, k, l) / (2.0 * tau_f)
                m = mag[k, l]
                safe = np.where(m > 0.0, m, 1.0)
                eG = E[i][0] * Gx + E[i][1] * Gy
                term = A * C[k, l] / 2.0 * m * (W[i] * eG * eG / (safe * safe) - B[i])
                phi = phi + np.where(m > 0.0, term, 0.0)
        fdag[i] = ftot[i] + omega + phi                                                      # Eq. (1)

    # recolouring, Eq. (13), then streaming, Eq. (22)
    out = np.empty_like(f)
    for k in range(3):
        for i in range(9):
            v = rho_k[k] / rho * fdag[i]
            for l in range(3):
                if l == k:
                    continue
                beta = beta_field(law, sigma, beta0, k, l, rho_k[0], rho_k[1], rho_k[2], rho)
                ne = n[k, l][0] * E[i][0] + n[k, l][1] * E[i][1]
                v = v + beta * W[i] * rho_k[k] * rho_k[l] / rho * ne
            out[k, i] = _at(v, (-E[i][0], -E[i][1]))  # f(x + e_i) = f_ddag(x)
    return out


def run(f, nsteps, **kw):
    for _ in range(nsteps):
        f = step(f, **kw)
    return f


def init_at_rest(rho):
    """f_{i,k} = w_i rho_k: the rest equilibrium split by colour (the paper prints no initial
    populations; the C oracle takes the same reading)."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.stack([np.stack([W[i] * rho[k] for i in range(9)]) for k in range(3)])
