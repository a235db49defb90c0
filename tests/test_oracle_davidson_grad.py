"""Pins of the oracle's Davidson iteration and gradients."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from synth import molecular_integrals, synthetic_problem, gaussian_psi, gapped_guess
from oracle.blocks import Construction
from oracle.fock import fci_hamiltonian, rdms
from oracle import heff, grad
from oracle.davidson import davidson


def diag_of(P, tasks):
    return heff.diagonal(P, tasks)


def test_cfg1_davidson_equals_fci(cfg1):
    P, H = cfg1["P"], cfg1["H"]
    tasks = heff.enumerate_tasks(P)
    e_fci = sla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    d = diag_of(P, tasks)
    # the task-derived diagonal is the FCI diagonal
    assert np.allclose(d, H.diagonal()[cfg1["idx"]], atol=1e-13)
    th, x, info = davidson(lambda v: heff.sigma(P, v, tasks), d, gaussian_psi(P, 1), tol_res=1e-7)
    assert abs(th - e_fci) < 1e-10
    assert info["res"] <= 1e-7


def test_synthetic_davidson_vs_eigsh():
    P = synthetic_problem(14, 14, 0, 64, 6, 16, 40, seed=8, gapped=True)
    tasks = heff.enumerate_tasks(P)
    mv = lambda v: heff.sigma(P, v, tasks)
    op = sla.LinearOperator((P.psi_dim, P.psi_dim), matvec=mv, dtype=np.float64)
    e_ref = sla.eigsh(op, k=1, which="SA", tol=1e-13)[0][0]
    d = diag_of(P, tasks)
    assert abs(np.argmin(d) - np.argmax(np.abs(gapped_guess(P, 2)))) == 0
    th, x, info = davidson(mv, d, gapped_guess(P, 2), tol_res=1e-8)
    assert abs(th - e_ref) < 1e-10 and info["iters"] < 40
    # non-gapped random instance from a random start
    P2 = synthetic_problem(14, 14, 0, 64, 6, 16, 40, seed=8)
    t2 = heff.enumerate_tasks(P2)
    mv2 = lambda v: heff.sigma(P2, v, t2)
    op2 = sla.LinearOperator((P2.psi_dim, P2.psi_dim), matvec=mv2, dtype=np.float64)
    e2 = sla.eigsh(op2, k=1, which="SA", tol=1e-13)[0][0]
    th2, _, _ = davidson(mv2, diag_of(P2, t2), gaussian_psi(P2, 2), tol_res=1e-8)
    assert abs(th2 - e2) < 1e-10
    assert np.linalg.norm(mv(x) - th * x) < 1e-7


def test_restart_path():
    P = synthetic_problem(14, 14, 0, 64, 6, 16, 40, seed=18, gapped=True)
    tasks = heff.enumerate_tasks(P)
    mv = lambda v: heff.sigma(P, v, tasks)
    d = diag_of(P, tasks)
    a = davidson(mv, d, gapped_guess(P, 3), tol_res=1e-8, max_sub=6, keep=2)
    b = davidson(mv, d, gapped_guess(P, 3), tol_res=1e-8)
    assert abs(a[0] - b[0]) < 1e-10


def _fd(f, x, h=1e-6):
    return (f(x + h) - f(x - h)) / (2 * h)


def test_gradients_central_fd():
    P = synthetic_problem(10, 10, 0, 24, 4, 8, 16, seed=61)
    tasks = heff.enumerate_tasks(P)
    psi = gaussian_psi(P, 1)
    G = gaussian_psi(P, 2)
    loss = lambda Q, x: float(G @ heff.sigma(Q, x, tasks))
    dpsi, dvals, dcoef = grad.backward(P, psi, G, tasks)
    rng = np.random.default_rng(0)
    for i in rng.choice(P.psi_dim, 8, replace=False):
        e = np.zeros(P.psi_dim)
        e[i] = 1.0
        fd = _fd(lambda t: loss(P, psi + t * e), 0.0)
        assert abs(fd - dpsi[i]) < 1e-7 * max(1, abs(dpsi[i]))
    used = np.nonzero(np.abs(dvals) > 0)[0]
    for j in rng.choice(used, 8, replace=False):
        orig = P.op_vals[j]

        def f(t):
            P.op_vals[j] = orig + t
            v = loss(P, psi)
            P.op_vals[j] = orig
            return v
        assert abs(_fd(f, 0.0) - dvals[j]) < 1e-7 * max(1, abs(dvals[j]))
    for k in range(min(P.nTerms, 6)):
        orig = P.term_coef[k]

        def g(t):
            P.term_coef[k] = orig + t
            tk = heff.enumerate_tasks(P)
            v = float(G @ heff.sigma(P, psi, tk))
            P.term_coef[k] = orig
            return v
        assert abs(_fd(g, 0.0) - dcoef[k]) < 1e-7 * max(1, abs(dcoef[k]))


def test_energy_gradient_is_rdm():
    L, N = 6, 6
    h, eri = molecular_integrals(L, 11)
    C = Construction(h, eri, N, 0, l=2)
    P = C.problem()
    H, dets = fci_hamiltonian(h, eri, N, 0)
    e, v = np.linalg.eigh(H.toarray())
    idx = C.fci_map(P, dets)
    x = v[idx, 0]
    tasks = heff.enumerate_tasks(P)
    dpsi, dvals, dcoef = grad.backward(P, x, x, tasks)
    # through sigma only: H^T x = H x = E x
    assert np.linalg.norm(dpsi - e[0] * x) < 1e-11
    dh, dv = grad.integral_gradients(C, P, dvals, dcoef, h.shape)
    g1, g2 = rdms(v[:, 0], dets, L)
    assert abs(dh - g1).max() < 1e-10
    assert abs(dv - 0.5 * g2).max() < 1e-10
    assert abs(np.trace(g1) - N) < 1e-10
    assert abs(np.einsum("iijj->", g2) - N * (N - 1)) < 1e-9
    assert abs((h * g1).sum() + 0.5 * (eri * g2).sum() - e[0]) < 1e-10
