"""Seeded one- and two-electron integrals for the long-range Hamiltonian (Eq. 1).

The Hamiltonian is read in the spin-free chemists' form
``H = sum h_ij c+_is c_js + 1/2 sum (ij|kl) c+_is c+_kt c_lt c_js`` with real
orbitals; these routines only draw the integral arrays.
"""

import numpy as np


def molecular_integrals(L, seed):
    """Random integrals shaped like molecular ones.

    * ``h_ij = h_ji`` Gaussian with standard deviation ``exp(-|i-j|/4)``.
    * ``(ij|kl) = sum_mu B^mu_ij B^mu_kl`` with ``B^mu`` symmetric,
      ``B^mu_ij = a_ij g^mu_ij``, ``g ~ N(0,1)``,
      ``a_ij = sqrt(0.5/sqrt(M)) exp(-|i-j|/4)`` and ``M = L(L+1)/2``.
      This gives the 8-fold permutational symmetry, a positive semi-definite
      pair supermatrix, and a standard deviation of about
      ``0.5 exp(-(|i-j|+|k-l|)/4)``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.arange(L)
    dist = np.abs(idx[:, None] - idx[None, :]).astype(np.float64)
    g = rng.standard_normal((L, L))
    h = np.triu(g) + np.triu(g, 1).T
    h = h * np.exp(-dist / 4.0)
    M = L * (L + 1) // 2
    gm = rng.standard_normal((M, L, L))
    gm = np.triu(gm) + np.transpose(np.triu(gm, 1), (0, 2, 1))
    a = np.sqrt(0.5 / np.sqrt(M)) * np.exp(-dist / 4.0)
    B = gm * a[None, :, :]
    eri = np.einsum("mij,mkl->ijkl", B, B, optimize=True)
    return h, eri


def hubbard_integrals(L, t, U, periodic=False):
    """Hubbard chain written as integrals: ``h`` = -t on nearest neighbours,
    ``(ii|ii) = U`` on site, every other two-electron integral zero."""
    h = np.zeros((L, L))
    for i in range(L - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    if periodic and L > 2:
        h[0, L - 1] = h[L - 1, 0] = -t
    eri = np.zeros((L, L, L, L))
    for i in range(L):
        eri[i, i, i, i] = U
    return h, eri
