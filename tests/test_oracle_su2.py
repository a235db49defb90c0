"""Pins of the oracle's spin-adapted (SU(2)) product.

* The terms coef [O_L x O_R]^0 of the instance sum to the same operator as
  the Hamiltonian written directly in spin orbitals (hopping, Heisenberg
  and density couplings between the blocks, block Hamiltonians): this pins
  every tensor-operator component and the -sqrt2, -sqrt3 factors.
* The coupled states are orthonormal eigenstates of the total S^2 with
  S(S+1) and of Sz with M = S.
* Without truncation the spectrum of V^T H V equals the eigenvalues of the
  Fock-space Hamiltonian on its (N, Sz = S) states of total spin S, and with
  truncation V^T H V is the compression of H (symmetric, its eigenvalues
  inside the untruncated ones' range).
"""
import numpy as np
import pytest

from synth.su2 import su2_instance
from oracle import su2 as osu


CASES = {"2x2 N=4 S=0": (2, 2, (4, 0)), "3x2 N=5 S=1/2": (3, 2, (5, 1)), "2x2 N=3 S=3/2": (2, 2, (3, 3)),
         "3x2 N=4 S=1": (3, 2, (4, 2))}


@pytest.mark.parametrize("case", list(CASES))
def test_terms_equal_direct_hamiltonian(case):
    lL, lR, target = CASES[case]
    inst = su2_instance(lL, lR, target, seed=11)
    F = osu.FullSpace(lL + lR)
    H = osu.hamiltonian(inst, F)
    Hd = osu.direct_hamiltonian(inst, F)
    assert abs(H - Hd).max() < 1e-12
    assert abs(H - H.T).max() < 1e-12


@pytest.mark.parametrize("case", list(CASES))
def test_coupled_states(case):
    lL, lR, target = CASES[case]
    inst = su2_instance(lL, lR, target, seed=12, keep_frac=0.7)
    F = osu.FullSpace(lL + lR)
    V = osu.coupled_basis(inst)
    assert V.shape[1] == inst.psi_dim > 0
    assert np.allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-12)
    S2, Sz = osu.total_spin(F, lL + lR)
    S = target[1] / 2
    assert np.allclose(S2 @ V, S * (S + 1) * V, atol=1e-12)
    assert np.allclose(Sz @ V, S * V, atol=1e-12)
    N = np.array([bin(d).count("1") for d in range(F.dim)])
    assert np.all(np.abs(V[N != target[0]]) < 1e-14)


@pytest.mark.parametrize("case", list(CASES))
def test_spectrum_equals_fock_multiplets(case):
    lL, lR, (N, twoS) = CASES[case]
    inst = su2_instance(lL, lR, (N, twoS), seed=13)
    F = osu.FullSpace(lL + lR)
    H = osu.hamiltonian(inst, F)
    V = osu.coupled_basis(inst)
    e_su2 = np.linalg.eigvalsh(V.T @ (H @ V))
    # Fock sector (N, 2Sz = 2S), then its states of total spin S
    occ = np.array([[(d >> p) & 1 for p in range(2 * (lL + lR))] for d in range(F.dim)])
    sel = np.nonzero((occ.sum(1) == N) & (occ[:, 0::2].sum(1) - occ[:, 1::2].sum(1) == twoS))[0]
    S2, _ = osu.total_spin(F, lL + lR)
    w, U = np.linalg.eigh(S2[np.ix_(sel, sel)].toarray())
    S = twoS / 2
    Q = U[:, np.abs(w - S * (S + 1)) < 1e-8]
    Hs = H[np.ix_(sel, sel)].toarray()
    e_fock = np.linalg.eigvalsh(Q.T @ Hs @ Q)
    assert len(e_su2) == len(e_fock) == inst.psi_dim
    assert np.allclose(e_su2, e_fock, atol=1e-10)


def test_truncated_compression():
    inst = su2_instance(3, 2, (5, 1), seed=14, keep_frac=0.5)
    full = su2_instance(3, 2, (5, 1), seed=14)
    H = osu.hamiltonian(inst)
    V = osu.coupled_basis(inst)
    A = V.T @ (H @ V)
    assert np.allclose(A, A.T, atol=1e-12)
    Vf = osu.coupled_basis(full)
    ef = np.linalg.eigvalsh(Vf.T @ (osu.hamiltonian(full) @ Vf))
    e = np.linalg.eigvalsh(A)
    assert ef[0] - 1e-10 <= e[0] and e[-1] <= ef[-1] + 1e-10
    psi = np.random.default_rng(0).standard_normal(inst.psi_dim)
    assert np.allclose(osu.sigma(inst, psi, H, V), A @ psi, atol=1e-12)


@pytest.mark.parametrize("case", list(CASES))
def test_reduced_route_equals_projection(case):
    """The Wigner-Eckart route on reduced blocks equals V^T H V psi."""
    lL, lR, target = CASES[case]
    for keep in (1.0, 0.6):
        inst = su2_instance(lL, lR, target, seed=15, keep_frac=keep)
        psi = np.random.default_rng(1).standard_normal(inst.psi_dim)
        want = osu.sigma(inst, psi)
        got = osu.sigma_reduced(inst, psi)
        assert np.allclose(got, want, atol=1e-12 * np.linalg.norm(want))
