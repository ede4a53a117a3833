"""Discrete-ordinates quadrature and real spherical harmonics, for building
moment matrices L[NM][D] and L+[D][NM] with L * L+ = I_NM.

This is input construction (textbook material, not the contraction itself):

* real spherical harmonics Y_n^m, n = 0..Lmax, m = -n..n, orthonormal on the
  unit sphere (integral of Y^2 over the sphere = 1), built from the
  associated-Legendre three-term recurrence;
* a product quadrature: n_mu Gauss-Legendre polar nodes mu_i (weights w_i,
  sum 2) times n_phi equispaced azimuths phi_j = 2 pi (j + 1/2) / n_phi
  (weights 2 pi / n_phi); direction d = i * n_phi + j, weight w_d summing to 4 pi.

The product rule integrates Y_n^m Y_n'^m' exactly when n + n' <= 2 Lmax,
n_mu >= Lmax + 1 and n_phi >= 2 Lmax + 1, so with
    L[nm, d] = w_d * Y_nm(Omega_d),   L+[d, nm] = Y_nm(Omega_d)
the moment-to-moment product L * L+ is the identity on the NM = (Lmax+1)^2
moments, and L+ * L is an idempotent projector on direction space.
Moment index: nm = n^2 + n + m.
"""
from __future__ import annotations

import math

import numpy as np


def assoc_legendre(nmax: int, x: np.ndarray) -> np.ndarray:
    """P[n, m, :] = P_n^m(x) for 0 <= m <= n <= nmax, without the Condon-Shortley
    phase, by the standard recurrences:
        P_m^m     = (2m-1)!! (1-x^2)^(m/2)
        P_{m+1}^m = x (2m+1) P_m^m
        P_n^m     = ((2n-1) x P_{n-1}^m - (n+m-1) P_{n-2}^m) / (n-m)
    """
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((nmax + 1, nmax + 1) + x.shape)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for m in range(nmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        P[m, m] = pmm
        if m + 1 <= nmax:
            P[m + 1, m] = x * (2 * m + 1) * pmm
        for n in range(m + 2, nmax + 1):
            P[n, m] = ((2 * n - 1) * x * P[n - 1, m] - (n + m - 1) * P[n - 2, m]) / (n - m)
    return P


def real_sph_harm(lmax: int, mu: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Y[nm, k] for directions k given by (mu_k = cos theta_k, phi_k)."""
    mu = np.asarray(mu, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    P = assoc_legendre(lmax, mu)
    Y = np.zeros(((lmax + 1) ** 2,) + mu.shape)
    for n in range(lmax + 1):
        for m in range(-n, n + 1):
            am = abs(m)
            norm = math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - am) / math.factorial(n + am))
            if m > 0:
                ang = math.sqrt(2.0) * np.cos(m * phi)
            elif m < 0:
                ang = math.sqrt(2.0) * np.sin(am * phi)
            else:
                ang = np.ones_like(phi)
            Y[n * n + n + m] = norm * P[n, am] * ang
    return Y


def product_quadrature(n_mu: int, n_phi: int):
    """(mu[D], phi[D], w[D]) with D = n_mu * n_phi, d = i * n_phi + j."""
    x, wx = np.polynomial.legendre.leggauss(n_mu)
    az = 2.0 * math.pi * (np.arange(n_phi) + 0.5) / n_phi
    mu = np.repeat(x, n_phi)
    ph = np.tile(az, n_mu)
    w = np.repeat(wx, n_phi) * (2.0 * math.pi / n_phi)
    return mu, ph, w


def moment_matrices(lmax: int, n_mu: int, n_phi: int):
    """(L[NM][D], Lplus[D][NM]) as row-major float64 arrays."""
    mu, ph, w = product_quadrature(n_mu, n_phi)
    Y = real_sph_harm(lmax, mu, ph)          # [NM][D]
    L = Y * w[None, :]
    Lplus = np.ascontiguousarray(Y.T)
    return np.ascontiguousarray(L), Lplus


# Quadrature sets matching the benchmark shapes: (lmax, n_mu, n_phi) -> D, NM.
SETS = {
    (48, 16): (3, 4, 12),
    (96, 16): (3, 8, 12),
    (128, 64): (7, 8, 16),
}
