"""FP64 Davidson iteration for the lowest eigenpair of H_eff.

Section III (implementation): the effective Hamiltonian is diagonalised
iteratively with the Lanczos or Davidson method, whose matrix-vector product
is the sum of Eq. (2).  The paper gives no further detail; the iteration here
is Davidson's method (1975) in the form below (a reading):

* ``V = [x0/|x0|]``, ``W = [H V]``.
* Repeat: ``S = (V^T W + W^T V)/2``; ``(theta, y)`` = lowest eigenpair of S;
  ``x = V y``, ``w = W y``, ``r = w - theta x``; stop when ``|r| <= tol_res``
  and ``|theta - theta_prev| <= tol_e``; correction ``t = r / (theta - d)``
  with ``d = diag(H)`` (denominators below 1e-12 in magnitude replaced by a
  signed 1e-12); two passes of classical Gram-Schmidt against V; stop on
  breakdown (``|t| < 1e-10``); append ``t/|t|`` and ``H t``; when V reaches
  ``max_sub`` columns restart from the ``keep`` lowest Ritz vectors.
"""

import numpy as np


def davidson(matvec, diag, x0, tol_res=1e-6, tol_e=1e-10, max_sub=32, keep=8, max_iter=500):
    """Returns ``(theta, x, info)`` with ``info = dict(iters, matvecs, res)``."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    V = [x]
    W = [matvec(x)]
    nmv = 1
    theta_prev = None
    res = np.inf
    it = 0
    theta = None
    for it in range(1, max_iter + 1):
        Vm = np.array(V).T
        Wm = np.array(W).T
        S = Vm.T @ Wm
        S = 0.5 * (S + S.T)
        evals, evecs = np.linalg.eigh(S)
        theta = evals[0]
        y = evecs[:, 0]
        x = Vm @ y
        w = Wm @ y
        r = w - theta * x
        res = np.linalg.norm(r)
        if res <= tol_res and theta_prev is not None and abs(theta - theta_prev) <= tol_e:
            break
        theta_prev = theta
        den = theta - diag
        small = np.abs(den) < 1e-12
        den = np.where(small, np.where(den < 0, -1e-12, 1e-12), den)
        t = r / den
        for _ in range(2):
            t = t - Vm @ (Vm.T @ t)
        nt = np.linalg.norm(t)
        if nt < 1e-10:
            break
        t = t / nt
        if len(V) >= max_sub:
            k = min(keep, len(V))
            Vm_new = Vm @ evecs[:, :k]
            Wm_new = Wm @ evecs[:, :k]
            V = [Vm_new[:, i] for i in range(k)]
            W = [Wm_new[:, i] for i in range(k)]
            t = t - np.array(V).T @ (np.array(V) @ t)
            t = t - np.array(V).T @ (np.array(V) @ t)
            t = t / np.linalg.norm(t)
        V.append(t)
        W.append(matvec(t))
        nmv += 1
    return theta, x / np.linalg.norm(x), dict(iters=it, matvecs=nmv, res=res)
