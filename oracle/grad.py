"""Gradients of a scalar loss on sigma (FP64, by definition).

Not in the paper; the derivative of Eq. (2).  For a loss with
``G = dloss/dsigma`` and every task ``sigma_out += alpha L psi_in R^T``:

* ``dpsi_in  += alpha L^T G_out R``
* ``dL       += alpha G_out R psi_in^T``
* ``dR       += alpha G_out^T L psi_in``
* ``dcoef_k  += (alpha / c_k) <G_out, L psi_in R^T>``  (Frobenius)

An identity side contributes no operator gradient.  For the energy loss
``<psi, H psi>`` with symmetric H, ``dpsi = 2 H psi``; the loss is quadratic
in psi and linear in every block and coefficient, so central finite
differences are exact up to rounding.

Integral gradients: the complementary operators of :mod:`oracle.blocks` are
linear in the integrals, so ``dE/dw_S`` for each Hamiltonian string ``S`` is
the Frobenius product of the gradient of the operator that carries ``w_S``
with the string's own block matrix (times its reordering sign).
"""

import numpy as np

from .heff import enumerate_tasks


def backward(P, psi, G, tasks=None):
    """Returns ``(dpsi, dvals, dcoef)``; ``dvals`` has the layout of
    ``P.op_vals`` (padding stays zero)."""
    if tasks is None:
        tasks = enumerate_tasks(P)
    dpsi = np.zeros(P.psi_dim)
    dvals = np.zeros_like(P.op_vals)
    dcoef = np.zeros(P.nTerms)
    for (s2, s, k, lb, rb, order, alpha, _) in tasks:
        X = P.psi_sector_view(psi, s)
        Gs = P.psi_sector_view(G, s2)
        Lm = P.block(lb) if lb >= 0 else None
        Rm = P.block(rb) if rb >= 0 else None
        GR = Gs @ Rm if Rm is not None else Gs              # q x n
        dX = (Lm.T @ GR) if Lm is not None else GR          # m x n
        dpsi[P.psi_off[s]:P.psi_off[s + 1]] += alpha * dX.reshape(-1)
        if Lm is not None:
            _add_block(P, dvals, lb, alpha * (GR @ X.T))
        if Rm is not None:
            LX = Lm @ X if Lm is not None else X            # q x n
            _add_block(P, dvals, rb, alpha * (Gs.T @ LX))
        c = float(P.term_coef[k])
        if c != 0.0:
            prod = X
            if Lm is not None:
                prod = Lm @ prod
            if Rm is not None:
                prod = prod @ Rm.T
            dcoef[k] += (alpha / c) * float(np.sum(Gs * prod))
    return dpsi, dvals, dcoef


def _add_block(P, dvals, b, M):
    o, r, c, ld = int(P.blk_off[b]), int(P.blk_rows[b]), int(P.blk_cols[b]), int(P.blk_ld[b])
    dvals[o:o + r * ld].reshape(r, ld)[:, :c] += M


def block_frobenius(P, dvals, op, blocks):
    """``sum_in <dvals[op block on in], blocks[in]>``."""
    tot = 0.0
    for b in np.nonzero(P.blk_op == op)[0]:
        i = int(P.blk_in[b])
        if i in blocks:
            o, r, c, ld = int(P.blk_off[b]), int(P.blk_rows[b]), int(P.blk_cols[b]), int(P.blk_ld[b])
            tot += float(np.sum(dvals[o:o + r * ld].reshape(r, ld)[:, :c] * blocks[i]))
    return tot


def integral_gradients(construction, P, dvals, dcoef, h_shape):
    """Contract operator-block and coefficient gradients to ``dE/dh_ij`` and
    ``dE/d(ij|kl)`` (each of the L^2 and L^4 entries treated as independent).

    A string whose weight sits in a term coefficient (naive table, or a term
    with identity on both blocks) gets ``f * dcoef``; one summed into an
    operator gets ``f * <d operator, string blocks>``; ``f`` is the string's
    reordering and monomial sign."""
    L = h_shape[0]
    dh = np.zeros((L, L))
    dv = np.zeros((L, L, L, L))
    for (wi, term, side, op, f, blocks) in construction.provenance:
        if side is None:
            g = f * float(dcoef[term])
        else:
            g = f * block_frobenius(P, dvals, op, blocks)
        lab = construction.labels[wi]
        if lab[0] == "h":
            dh[lab[1], lab[2]] += g
        else:
            dv[lab[1], lab[2], lab[3], lab[4]] += 0.5 * g
    return dh, dv
