"""Karhunen-Loeve random fields for the oracle (TEST INFRASTRUCTURE).

Porosity and permeability are the uncertain fields of Sec. 2.2 of the paper;
this module gives them as truncated KL expansions of Gaussian fields with
the separable squared-exponential covariance
    C(x, x') = exp(-|x - x'|^2 / (2 l^2)) = C1(x1, x1') C2(x2, x2'),
on D = [0,2] x [-1,0], correlation length l = 0.3 m:
    Z(x) = sum_{k < 20} sqrt(lam_k) e_k(x) xi_k,  xi_k ~ N(0,1),
    phi = phi0 (1 + 0.1 Z_phi),  log K = log k0 + 0.5 Z_K,
    q = q_in (1 + 0.2 xi_41),  xi_41 ~ U[-1,1].
1D eigenpairs by the Nystrom method with Gauss-Legendre quadrature
(numpy's leggauss / eigh as library steps); eigenfunctions normalised to
unit L2 norm under the quadrature, signed positive at the first node, and
evaluated off the nodes by Nystrom interpolation
    e(x) = (1/lam) sum_j w_j C(x, x_j) e(x_j).
2D modes are products e^x_a(x) e^y_b(y) with eigenvalue lam^x_a lam^y_b,
ordered by decreasing eigenvalue, ties by (a + b, a).

Gaussian coefficients: Box-Muller on Philox uniforms.  Pair g (components
2g, 2g+1) takes Philox block counter (100 + g, level, index lo, index hi),
key (seed lo, seed hi); words (0,1) and (2,3) give 53-bit integers x1, x2;
u1 = (x1 + 1) 2^-53 in (0, 1], u2 = x2 2^-53; r = sqrt(-2 ln u1),
z = (r cos 2 pi u2, r sin 2 pi u2).  The recharge component uses block
(200, level, index lo, index hi), words (0,1), mapped to x 2^-52 - 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox4x32_10

CORR_LEN = 0.3
NMODES = 20
NQUAD = 200
SIGMA_PHI = 0.1
SIGMA_LOGK = 0.5


def nystrom_1d(a: float, b: float, corr_len: float = CORR_LEN, nquad: int = NQUAD):
    """Eigenpairs of the 1D kernel exp(-(s-t)^2/(2 l^2)) on [a, b]:
    returns (lam descending, nodes, weights, values at the nodes [k][i])."""
    t, w = np.polynomial.legendre.leggauss(nquad)
    x = 0.5 * (b - a) * t + 0.5 * (b + a)
    w = 0.5 * (b - a) * w
    C = np.exp(-(x[:, None] - x[None, :]) ** 2 / (2 * corr_len ** 2))
    sw = np.sqrt(w)
    lam, V = np.linalg.eigh(sw[:, None] * C * sw[None, :])
    order = np.argsort(-lam)
    lam = lam[order]
    E = (V[:, order] / sw[:, None]).T          # e_k(x_i), unit norm under the quadrature
    E *= np.sign(E[:, :1])                     # positive at the first node
    return lam, x, w, E


def eval_1d(lam, x, w, E, pts, corr_len: float = CORR_LEN):
    """Nystrom interpolation of the eigenfunctions at `pts`: [k][len(pts)]."""
    C = np.exp(-(np.asarray(pts)[:, None] - x[None, :]) ** 2 / (2 * corr_len ** 2))
    return (C @ (w[:, None] * E.T)).T / lam[:, None]


def basis(nx: int, ny: int, nmodes: int = NMODES, corr_len: float = CORR_LEN, nquad: int = NQUAD):
    """(lam[nmodes], modes[nmodes][ny][nx]) of the 2D expansion at cell centres."""
    h = 1.0 / ny
    xc = (np.arange(nx) + 0.5) * h
    yc = -1.0 + (np.arange(ny) + 0.5) * h
    lx, X, WX, EX = nystrom_1d(0.0, 2.0, corr_len, nquad)
    ly, Y, WY, EY = nystrom_1d(-1.0, 0.0, corr_len, nquad)
    m1 = nmodes
    cand = [(lx[a] * ly[b], a + b, a, b) for a in range(m1) for b in range(m1)]
    cand.sort(key=lambda t: (-t[0], t[1], t[2]))
    cand = cand[:nmodes]
    ex = eval_1d(lx, X, WX, EX, xc, corr_len)
    ey = eval_1d(ly, Y, WY, EY, yc, corr_len)
    lam = np.array([c[0] for c in cand])
    modes = np.array([np.outer(ey[c[3]], ex[c[2]]) for c in cand])
    return lam, modes


def fields(phys, lam, modes, xi41):
    """phi, K [ny][nx] and q from the 41 coefficients."""
    s = np.sqrt(lam)
    zphi = np.tensordot(s * np.asarray(xi41[:20]), modes, axes=1)
    zk = np.tensordot(s * np.asarray(xi41[20:40]), modes, axes=1)
    phi = phys["phi0"] * (1.0 + SIGMA_PHI * zphi)
    K = np.exp(math.log(phys["k0"]) + SIGMA_LOGK * zk)
    q = phys["q_in"] * (1.0 + 0.2 * xi41[40])
    return phi, K, q


def _words(seed, ctr0, level, index):
    return philox4x32_10((ctr0, level, index & 0xFFFFFFFF, index >> 32), (seed & 0xFFFFFFFF, seed >> 32))


def sample_xi41(seed: int, level: int, first: int, count: int) -> np.ndarray:
    out = np.empty((count, 41))
    for s in range(count):
        idx = first + s
        for g in range(20):
            w = _words(seed, 100 + g, level, idx)
            x1 = ((w[1] << 32) | w[0]) >> 11
            x2 = ((w[3] << 32) | w[2]) >> 11
            u1 = (x1 + 1) * 2.0 ** -53
            u2 = x2 * 2.0 ** -53
            r = math.sqrt(-2.0 * math.log(u1))
            out[s, 2 * g] = r * math.cos(2.0 * math.pi * u2)
            out[s, 2 * g + 1] = r * math.sin(2.0 * math.pi * u2)
        w = _words(seed, 200, level, idx)
        out[s, 40] = (((w[1] << 32) | w[0]) >> 11) * 2.0 ** -52 - 1.0
    return out


def solve_kl(phys, nx, ny, nsteps, xi41, lam, modes):
    """(Q, c) of one solve with KL fields."""
    from . import solve
    phi, K, q = fields(phys, lam, modes, xi41)
    out = solve(phys, nsteps, phi, K, q)
    return out["qoi"], out["c"]


def adjoint_kl(phys, nsteps, xi41, lam, modes):
    """(Q, dQ/dxi[41]): the oracle's discrete adjoint (gradients with
    respect to phi, K and q) composed with the field map by the chain rule:
    dphi/dxi_k = phi0 s_phi sqrt(lam_k) e_k, dK/dxi_{20+k} = K s_K sqrt(lam_k) e_k,
    dq/dxi_41 = 0.2 q_in."""
    from . import adjoint
    phi, K, q = fields(phys, lam, modes, xi41)
    Q, gphi, gK, gq = adjoint(phys, nsteps, phi, K, q)
    s = np.sqrt(lam)
    g = np.empty(41)
    g[:20] = phys["phi0"] * SIGMA_PHI * s * np.tensordot(modes, gphi, axes=([1, 2], [0, 1]))
    g[20:40] = SIGMA_LOGK * s * np.tensordot(modes, gK * K, axes=([1, 2], [0, 1]))
    g[40] = gq * phys["q_in"] * 0.2
    return Q, g
