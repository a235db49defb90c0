"""sigma = H_eff psi by definition, the canonical task table, and the full-form check.

Section III.A.2, Eq. (2): with the site factors reduced to scalars, each term
adds ``alpha * L_i A R_i^T`` into an output sector of the wavefunction, where
``alpha`` is the precalculated product of the term coefficient, the two site
matrix elements and the fermionic sign.  Section III.A.1 (levels 1 and 2):
the sector and task tables list, for every term and input sector, the output
sector and the blocks involved.  Level 4 is a full-form representation used
as a self-check; :func:`dense_heff` builds it.  Section III.B: each matrix
chain is evaluated in its cheaper parenthesisation.

Fermionic sign (reading): a term ``c * O_L O_a O_b O_R`` acting on
``|l, sa, sb, r> = C_l C_a C_b C_r |0>`` moves ``O_a`` past ``C_l``, ``O_b``
past ``C_l C_a`` and ``O_R`` past ``C_l C_a C_b``, so the sign is
``(-1)^(pa*Nl + pb*(Nl+Na) + pR*(Nl+Na+Nb))`` with the parities ``p`` of the
operators and the particle numbers ``N`` of the *input* state.

Task record (40 bytes, little endian): ``out, in, term, lblk, rblk, order``
(int32), ``alpha`` (float64), ``cost`` (int64).  ``cost`` is the flop count
of the cheaper order: ``2qn(m+r)`` for ``(L psi) R^T``, ``2mr(n+q)`` for
``L (psi R^T)`` (``order`` = 1 only when strictly cheaper); an identity side
drops its product (``2mnr`` or ``2qmn``; ``2mn`` when both are identity).
The table is sorted stably by output sector, keeping (term, input sector)
order inside each output sector.
"""

import numpy as np

from .blocks import MONO, SITE_Q, mono_action

TASK_DTYPE = np.dtype([("out", "<i4"), ("in", "<i4"), ("term", "<i4"), ("lblk", "<i4"),
                       ("rblk", "<i4"), ("order", "<i4"), ("alpha", "<f8"), ("cost", "<i8")])
assert TASK_DTYPE.itemsize == 40


def _parity_op(P, op):
    return int(abs(int(P.op_dN[op])) % 2) if op >= 0 else 0


def _mono_parity(m):
    # monomials change N by the number of ladder factors
    nz = np.nonzero(MONO[m])
    if len(nz[0]) == 0:
        return 0
    o, i = nz[0][0], nz[1][0]
    return int(abs(int(SITE_Q[o][0] - SITE_Q[i][0])) % 2)


def task_cost(q, m, n, r, has_L, has_R):
    """Flop count and order flag of one task (see module docstring)."""
    if has_L and has_R:
        c0 = 2 * q * n * (m + r)
        c1 = 2 * m * r * (n + q)
        return (c1, 1) if c1 < c0 else (c0, 0)
    if has_L:
        return 2 * q * m * n, 0
    if has_R:
        return 2 * m * n * r, 0
    return 2 * m * n, 0


def _op_in_map(P):
    """``{op: {in_sector: block}}``."""
    out = {}
    for b in range(P.nBlk):
        out.setdefault(int(P.blk_op[b]), {})[int(P.blk_in[b])] = b
    return out


def enumerate_tasks(P, out_filter=None):
    """Levels 1 and 2: every (term, input sector) pair that produces a
    contribution, in (term, input sector) order, as a list of tuples
    ``(out, in, term, lblk, rblk, order, alpha, cost)``.

    A task exists when the left block of ``op_L`` on the input left sector
    exists (or ``op_L`` is the identity), both site monomials have a non-zero
    element on the input site states, the right block exists (or identity),
    and the resulting output sector is in the wavefunction sector table."""
    inmap = _op_in_map(P)
    sec_index = {(int(a), int(b), int(c)): s for s, (a, b, c, _) in enumerate(P.psi_sec)}
    act = [[mono_action(m, s) for s in range(4)] for m in range(16)]
    mpar = [_mono_parity(m) for m in range(16)]
    NL = P.qL[:, 0]
    tasks = []
    for k in range(P.nTerms):
        oL, ma, mb, oR = int(P.term_L[k]), int(P.term_ma[k]), int(P.term_mb[k]), int(P.term_R[k])
        c = float(P.term_coef[k])
        mL = inmap.get(oL, {}) if oL >= 0 else None
        mR = inmap.get(oR, {}) if oR >= 0 else None
        pa, pb, pR = mpar[ma], mpar[mb], _parity_op(P, oR)
        for s in range(P.nS):
            iL, sa, sb, iR = (int(v) for v in P.psi_sec[s])
            if oL >= 0:
                lb = mL.get(iL)
                if lb is None:
                    continue
                iL2 = int(P.blk_out[lb])
            else:
                lb, iL2 = -1, iL
            sa2, va = act[ma][sa]
            if sa2 is None:
                continue
            sb2, vb = act[mb][sb]
            if sb2 is None:
                continue
            if oR >= 0:
                rb = mR.get(iR)
                if rb is None:
                    continue
                iR2 = int(P.blk_out[rb])
            else:
                rb, iR2 = -1, iR
            s2 = sec_index.get((iL2, sa2, sb2))
            if s2 is None or int(P.psi_sec[s2][3]) != iR2:
                continue
            if out_filter is not None and s2 not in out_filter:
                continue
            Nl, Na, Nb = int(NL[iL]), int(SITE_Q[sa][0]), int(SITE_Q[sb][0])
            e = pa * Nl + pb * (Nl + Na) + pR * (Nl + Na + Nb)
            sgn = -1.0 if e % 2 else 1.0
            alpha = ((c * va) * vb) * sgn
            q, m = int(P.dimL[iL2]), int(P.dimL[iL])
            n, r = int(P.dimR[iR]), int(P.dimR[iR2])
            cost, order = task_cost(q, m, n, r, oL >= 0, oR >= 0)
            tasks.append((s2, s, k, lb, rb, order, alpha, cost))
    return tasks


def task_table(P):
    """Canonical task table (numpy structured array, 40-byte records):
    :func:`enumerate_tasks` stably sorted by output sector, and the CSR
    pointer ``out_ptr[nS+1]``."""
    t = enumerate_tasks(P)
    arr = np.array(t, dtype=TASK_DTYPE) if t else np.zeros(0, dtype=TASK_DTYPE)
    order = np.argsort(arr["out"], kind="stable")
    arr = arr[order]
    counts = np.bincount(arr["out"], minlength=P.nS) if len(arr) else np.zeros(P.nS, dtype=np.int64)
    ptr = np.zeros(P.nS + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(counts)
    return arr, ptr


def task_product(P, psi, t):
    """``alpha * L psi_in R^T`` of one task, in the task's order."""
    s2, s, k, lb, rb, order, alpha, _ = t
    X = P.psi_sector_view(psi, s)
    if lb >= 0 and rb >= 0:
        Lm, Rm = P.block(lb), P.block(rb)
        Y = (Lm @ (X @ Rm.T)) if order == 1 else ((Lm @ X) @ Rm.T)
    elif lb >= 0:
        Y = P.block(lb) @ X
    elif rb >= 0:
        Y = X @ P.block(rb).T
    else:
        Y = X.copy()
    return alpha * Y


def sigma(P, psi, tasks=None):
    """Eq. (2) summed over the whole task table:
    ``sigma_out = sum_tasks alpha L psi_in R^T`` (FP64)."""
    if tasks is None:
        tasks = enumerate_tasks(P)
    out = np.zeros(P.psi_dim)
    for t in tasks:
        s2 = t[0]
        out[P.psi_off[s2]:P.psi_off[s2 + 1]] += task_product(P, psi, t).reshape(-1)
    return out


def sigma_sectors(P, psi, sectors, tasks=None):
    """Only the listed output sectors of :func:`sigma` (for sampled checks)."""
    sel = set(int(s) for s in sectors)
    if tasks is None:
        tasks = enumerate_tasks(P, out_filter=sel)
    res = {s: np.zeros((int(P.dimL[P.psi_sec[s][0]]), int(P.dimR[P.psi_sec[s][3]]))) for s in sel}
    for t in tasks:
        if t[0] in sel:
            res[t[0]] += task_product(P, psi, t)
    return res


def sigma_threaded(P, psi, tasks=None, threads=None, sectors=None):
    """:func:`sigma` (Eq. (2)) with the output sectors shared out over a pool
    of ``threads`` Python threads (default: the cores this process may run
    on), BLAS at one thread per call.  Each output sector is summed by one
    thread in task-table order, as :func:`sigma` sums it; the two differ
    only by the rounding inside the BLAS calls.  ``sectors``: only these output
    sectors (the rest of the result stays zero).  Returns ``(sigma, threads)``."""
    from concurrent.futures import ThreadPoolExecutor
    import os
    from threadpoolctl import threadpool_limits
    if tasks is None:
        tasks = enumerate_tasks(P)
    by_out = {}
    for t in tasks:
        by_out.setdefault(int(t[0]), []).append(t)
    outs = sorted(by_out) if sectors is None else sorted(set(int(x) for x in sectors) & set(by_out))
    # largest sectors first so that the pool ends evenly
    outs.sort(key=lambda s2: -sum(int(t[7]) for t in by_out[s2]))
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    out = np.zeros(P.psi_dim)

    def one(s2):
        acc = None
        for t in by_out[s2]:
            y = task_product(P, psi, t)
            acc = y if acc is None else acc + y
        out[P.psi_off[s2]:P.psi_off[s2 + 1]] += acc.reshape(-1)

    with threadpool_limits(limits=1, user_api="blas"):
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, outs))
    return out, threads


def diagonal(P, tasks):
    """diag(H_eff) from the definition of Eq. (2): only tasks whose output
    sector is their input sector reach the diagonal, each adding
    ``alpha * diag(L) (x) diag(R)`` (a ones vector for an identity side)."""
    d = np.zeros(P.psi_dim)
    for (s2, s, k, lb, rb, order, alpha, _) in tasks:
        if s2 != s:
            continue
        m = int(P.dimL[P.psi_sec[s][0]])
        n = int(P.dimR[P.psi_sec[s][3]])
        dl = np.diag(P.block(lb)) if lb >= 0 else np.ones(m)
        dr = np.diag(P.block(rb)) if rb >= 0 else np.ones(n)
        d[P.psi_off[s]:P.psi_off[s + 1]] += alpha * np.outer(dl, dr).reshape(-1)
    return d


def total_flops(tasks):
    return int(sum(int(t[7]) for t in tasks))


# ---------------------------------------------------------------------------
# Level 4: full-form representation
# ---------------------------------------------------------------------------


def _full_op(P, op, side):
    """Full matrix of a block operator over all states of its block."""
    dims = P.dimL if side == 0 else P.dimR
    off = np.zeros(len(dims) + 1, dtype=np.int64)
    off[1:] = np.cumsum(dims)
    n = int(off[-1])
    if op < 0:
        return np.eye(n), off
    M = np.zeros((n, n))
    for b in np.nonzero(P.blk_op == op)[0]:
        i, j = int(P.blk_in[b]), int(P.blk_out[b])
        M[off[j]:off[j + 1], off[i]:off[i + 1]] = P.block(b)
    return M, off


def dense_heff(P):
    """Full-form H_eff on the packed wavefunction basis.

    Every term is written as ``c * (L (x) a (x) b (x) R) * diag(sign)`` over
    the full (all-sector) spaces of the four subsystems, with the sign of the
    module docstring as a diagonal on the input product basis, and evaluated
    only on the rows and columns of the wavefunction sectors.  This is the
    level-4 full-form self-check: no task table, no block lookup, no
    per-sector products; it shares only the sign formula with :func:`sigma`.
    Cost is (psi_dim)^2 per term, so it is meant for tiny instances."""
    offL = np.concatenate([[0], np.cumsum(P.dimL)])
    offR = np.concatenate([[0], np.cumsum(P.dimR)])
    ls, sas, sbs, rs = [], [], [], []
    for s in range(P.nS):
        iL, sa, sb, iR = (int(v) for v in P.psi_sec[s])
        li = np.arange(offL[iL], offL[iL + 1])
        ri = np.arange(offR[iR], offR[iR + 1])
        g = np.meshgrid(li, ri, indexing="ij")
        ls.append(g[0].reshape(-1))
        rs.append(g[1].reshape(-1))
        sas.append(np.full(g[0].size, sa))
        sbs.append(np.full(g[0].size, sb))
    l_, a_, b_, r_ = (np.concatenate(x) for x in (ls, sas, sbs, rs))
    NLfull = np.repeat(P.qL[:, 0], P.dimL)
    Nl = NLfull[l_]
    Na = SITE_Q[a_, 0]
    Nb = SITE_Q[b_, 0]
    n = len(l_)
    H = np.zeros((n, n))
    mpar = [_mono_parity(m) for m in range(16)]
    for k in range(P.nTerms):
        oL, ma, mb, oR = int(P.term_L[k]), int(P.term_ma[k]), int(P.term_mb[k]), int(P.term_R[k])
        Lf, _ = _full_op(P, oL, 0)
        Rf, _ = _full_op(P, oR, 1)
        pa, pb, pR = mpar[ma], mpar[mb], _parity_op(P, oR)
        e = pa * Nl + pb * (Nl + Na) + pR * (Nl + Na + Nb)
        sg = np.where(e % 2 == 1, -1.0, 1.0)
        H += float(P.term_coef[k]) * (Lf[np.ix_(l_, l_)] * MONO[ma][np.ix_(a_, a_)] * MONO[mb][np.ix_(b_, b_)]
                                      * Rf[np.ix_(r_, r_)]) * sg[None, :]
    return H
