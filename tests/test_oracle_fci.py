"""Pins of the brute-force FCI Hamiltonian (Eq. 1, spin-free reading) against
closed forms and invariants that do not reuse its code."""
import numpy as np
import pytest

from synth import molecular_integrals, hubbard_integrals
from oracle.fock import (fci_hamiltonian, string_matrix, number_strings, s2_strings,
                         determinants, apply_string)


def lowest(H):
    return np.linalg.eigvalsh(H.toarray())


def test_jordan_wigner_anticommutation():
    # {c_p, c+_q} = delta_pq on every determinant of 3 orbitals
    for p in range(6):
        for q in range(6):
            for det in range(64):
                s1, d1 = apply_string([(p, 0), (q, 1)], det)
                s2, d2 = apply_string([(q, 1), (p, 0)], det)
                acc = {}
                if s1:
                    acc[d1] = acc.get(d1, 0) + s1
                if s2:
                    acc[d2] = acc.get(d2, 0) + s2
                acc = {k: v for k, v in acc.items() if v}
                assert acc == ({det: 1} if p == q else {})


def test_hubbard_dimer_closed_form():
    # two sites, two electrons, singlet ground state: U/2 - sqrt(U^2/4 + 4 t^2)
    for t, U in ((1.0, 4.0), (0.7, 1.3), (1.0, 0.0)):
        h, eri = hubbard_integrals(2, t, U)
        H, _ = fci_hamiltonian(h, eri, 2, 0)
        e = lowest(H)
        assert abs(e[0] - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-12


def test_two_orbital_two_electron_spectrum():
    # h diagonal (e1, e2), J=(11|22), K=(12|12) with 8-fold symmetry, U1=(11|11), U2=(22|22)
    e1, e2, U1, U2, J, K = -1.3, -0.4, 0.9, 0.7, 0.5, 0.2
    h = np.diag([e1, e2])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0], eri[1, 1, 1, 1] = U1, U2
    eri[0, 0, 1, 1] = eri[1, 1, 0, 0] = J
    for idx in ((0, 1, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1)):
        eri[idx] = K
    H, _ = fci_hamiltonian(h, eri, 2, 0)
    got = np.sort(lowest(H))
    closed = np.linalg.eigvalsh(np.array([[2 * e1 + U1, K], [K, 2 * e2 + U2]]))
    want = np.sort(np.concatenate([closed, [e1 + e2 + J - K, e1 + e2 + J + K]]))
    assert np.allclose(got, want, atol=1e-12)


def test_free_fermions_closed_form():
    h, _ = molecular_integrals(6, 5)
    eps = np.linalg.eigvalsh(h)
    H, _ = fci_hamiltonian(h, np.zeros((6,) * 4), 6, 0)
    assert abs(lowest(H)[0] - 2 * eps[:3].sum()) < 1e-12
    # odd electron number: N=5, 2Sz=1 -> doubly fill 2 levels, singly the third
    H, _ = fci_hamiltonian(h, np.zeros((6,) * 4), 5, 1)
    assert abs(lowest(H)[0] - (2 * eps[:2].sum() + eps[2])) < 1e-12


def test_hermitian_number_spin_and_reversal():
    L, N = 5, 5
    h, eri = molecular_integrals(L, 3)
    H, dets = fci_hamiltonian(h, eri, N, 1)
    assert abs(H - H.T).max() < 1e-14
    # particle number and S^2 commute with H; N is diagonal with value N
    Nop = string_matrix(number_strings(L), dets)
    assert np.allclose(Nop.toarray(), N * np.eye(len(dets)))
    S2 = string_matrix(s2_strings(L), dets)
    assert abs(H @ S2 - S2 @ H).max() < 1e-12
    e, v = np.linalg.eigh(H.toarray())
    s2 = v[:, 0] @ (S2 @ v[:, 0])
    S = (-1 + np.sqrt(1 + 4 * s2)) / 2
    assert abs(S - round(2 * S) / 2) < 1e-8
    # orbital reversal leaves the spectrum unchanged
    r = np.arange(L)[::-1]
    H2, _ = fci_hamiltonian(h[np.ix_(r, r)], eri[np.ix_(r, r, r, r)], N, 1)
    assert abs(np.linalg.eigvalsh(H2.toarray())[0] - e[0]) < 1e-12


def test_determinant_count():
    from math import comb
    assert len(determinants(8, 8, 0)) == comb(8, 4) ** 2 == 4900
    assert len(determinants(6, 5, 1)) == comb(6, 3) * comb(6, 2)
