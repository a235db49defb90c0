"""Renormalisation (blocking) of block operators, by definition (FP64).

Section II.A / IV.D: after a two-site step the left block grows by one site
and its operators are carried over to the new, truncated basis.  Every new
operator is a sum of terms ``coef * (O ⊗ m)`` with ``O`` an operator of the
old block (or the identity) and ``m`` a site monomial; on the enlarged basis
it is a dense matrix, and the renormalised operator is ``U^T O' U`` with the
isometry ``U`` whose columns span the kept states.  Unlike the effective
Hamiltonian's product, the terms of different new operators are never summed
together: each new operator is an output of its own (the paper's note that
the position sum is left out).

Readings (the paper defers to reviews for the details):

* The enlarged block is the old block followed by one site; its product
  state ``|l, s> = C_l C_s |0>`` (old-block creators first), so a term acting
  as ``O ⊗ m`` picks up ``(-1)^(parity(m) N_l)`` from moving the site
  factor past ``C_l`` (``N_l`` the old block's particle number of the input).
* Enlarged sectors ``Q = q(i) + q(s)`` in ascending (N, 2Sz) order; inside a
  sector the product basis lists the components ``(i, s)`` (old sector,
  site state) in ascending order, each with the ``dim(i)`` states of old
  sector ``i``.  ``U_Q`` is a ``full(Q) x keep(Q)`` matrix with orthonormal
  columns on that basis.

Functions here build the dense operator on the whole enlarged basis and apply
the isometry with plain matrix products; no block task list is involved.
"""

import numpy as np

from .blocks import MONO, SITE_Q


def _parity(m):
    nz = np.nonzero(MONO[m])
    if len(nz[0]) == 0:
        return 0
    o, i = nz[0][0], nz[1][0]
    return int(abs(int(SITE_Q[o][0] - SITE_Q[i][0])) % 2)


def enlarged_sectors(qL, dimL):
    """Sectors of the enlarged block: ``(qQ[nQ, 2], comps)`` with ``comps[Q]``
    the list of ``(i, s, dim(i))`` components in ascending ``(i, s)`` order."""
    comps = {}
    for i in range(len(dimL)):
        for s in range(4):
            q = (int(qL[i][0]) + int(SITE_Q[s][0]), int(qL[i][1]) + int(SITE_Q[s][1]))
            comps.setdefault(q, []).append((i, s, int(dimL[i])))
    qQ = sorted(comps)
    return np.array(qQ, dtype=np.int32).reshape(-1, 2), [comps[q] for q in qQ]


def full_basis_offsets(comps):
    """Offsets of each enlarged sector and of each component inside the
    concatenated full product basis."""
    sec_off, comp_off = [], []
    o = 0
    for cs in comps:
        sec_off.append(o)
        co = {}
        for (i, s, d) in cs:
            co[(i, s)] = o
            o += d
        comp_off.append(co)
    return sec_off + [o], comp_off


def dense_old(qL, dimL, blocks):
    """Dense matrix of an old-block operator given as ``{in_sector: (out_sector,
    block)}`` on the concatenated old-block basis (or the identity for None)."""
    off = np.concatenate([[0], np.cumsum(dimL)]).astype(np.int64)
    n = int(off[-1])
    if blocks is None:
        return np.eye(n), off
    M = np.zeros((n, n))
    for i, (j, B) in blocks.items():
        M[off[j]:off[j + 1], off[i]:off[i + 1]] = B
    return M, off


def dense_enlarged(qL, dimL, terms, op_blocks):
    """The new operator ``sum_t coef_t (O_t ⊗ m_t) * sign`` as a dense matrix
    on the full enlarged basis (sector-major, components ascending).
    ``terms``: list of ``(op, mono, coef)`` (op -1 = identity);
    ``op_blocks[op]``: ``{in_sector: (out_sector, block)}``."""
    qQ, comps = enlarged_sectors(qL, dimL)
    sec_off, comp_off = full_basis_offsets(comps)
    n = sec_off[-1]
    M = np.zeros((n, n))
    NL = np.asarray(qL)[:, 0]
    for (op, m, coef) in terms:
        O, off = dense_old(qL, dimL, None if op < 0 else op_blocks[op])
        pm = _parity(m)
        for i in range(len(dimL)):
            for s in range(4):
                col = np.nonzero(MONO[m][:, s])[0]
                if len(col) == 0:
                    continue
                s2 = int(col[0])
                val = float(MONO[m][s2, s])
                sign = -1.0 if (pm * int(NL[i])) % 2 else 1.0
                Qi = _sector_of(qQ, qL[i], s)
                c_in = comp_off[Qi][(i, s)]
                for j in range(len(dimL)):
                    blk = O[off[j]:off[j + 1], off[i]:off[i + 1]]
                    if not blk.any():
                        continue
                    Qj = _sector_of(qQ, qL[j], s2)
                    c_out = comp_off[Qj][(j, s2)]
                    M[c_out:c_out + dimL[j], c_in:c_in + dimL[i]] += coef * val * sign * blk
    return M, qQ, comps, sec_off


def _sector_of(qQ, qi, s):
    q = (int(qi[0]) + int(SITE_Q[s][0]), int(qi[1]) + int(SITE_Q[s][1]))
    for k, x in enumerate(qQ):
        if int(x[0]) == q[0] and int(x[1]) == q[1]:
            return k
    raise KeyError(q)


def renormalize(qL, dimL, terms, op_blocks, U):
    """``U^T O' U`` of one new operator, returned as
    ``{(Q_in, Q_out): keep(Q_out) x keep(Q_in) block}`` (non-zero blocks
    only); ``U[Q]`` is the isometry of enlarged sector Q."""
    M, qQ, comps, sec_off = dense_enlarged(qL, dimL, terms, op_blocks)
    out = {}
    for a in range(len(qQ)):
        for b in range(len(qQ)):
            blk = M[sec_off[b]:sec_off[b + 1], sec_off[a]:sec_off[a + 1]]
            if not blk.any():
                continue
            R = U[b].T @ blk @ U[a]
            out[(a, b)] = R
    return out
