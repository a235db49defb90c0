"""Seeded inputs of a renormalisation (blocking) step: a block with its
block-sparse operators, the isometries of the enlarged block, and the terms
of the new operators.  Inputs only: the renormalised operators themselves are
computed by the oracle and by the GPU library.

* Block sectors: :func:`synth.problem.block_profile` (Gaussian profile of
  sector sizes around half filling).
* Operators: ``n_ops`` random shifts from :data:`synth.problem.SHIFTS`; every
  block that the shift allows is filled with ``N(0, 1/cols)`` entries from a
  counter-based stream keyed by ``(seed, operator)``; rows are padded to a
  multiple of 8 elements (the library's operator layout).
* Enlarged sectors: every ``q(i) + q(s)``; ``keep(Q)`` = the full dimension
  times ``keep_frac`` (at least 1), and ``U_Q`` the first ``keep(Q)``
  columns of the orthogonal factor of a Gaussian matrix (orthonormal columns).
* New operators: ``n_new``, each with one term ``O (x) m`` (random operator
  and monomial), a second term of the same shift with probability one half
  (another operator whose shift a monomial can complete), and every
  ``identity_every``-th one is the site monomial alone (``1 (x) m``).
"""

from dataclasses import dataclass

import numpy as np

from .problem import SHIFTS, MONO_SHIFT, block_profile, site_q, _round_up, ALIGN


@dataclass
class RenormInstance:
    qL: np.ndarray
    dimL: np.ndarray
    op_dN: np.ndarray
    op_d2Sz: np.ndarray
    blk_op: np.ndarray
    blk_in: np.ndarray
    blk_out: np.ndarray
    blk_rows: np.ndarray
    blk_cols: np.ndarray
    blk_ld: np.ndarray
    blk_off: np.ndarray
    op_vals: np.ndarray
    qQ: np.ndarray
    keep: np.ndarray
    u_off: np.ndarray
    u_vals: np.ndarray
    term_new: np.ndarray
    term_op: np.ndarray
    term_mono: np.ndarray
    term_coef: np.ndarray
    n_new: int
    full: np.ndarray  # full dimension of each enlarged sector

    @property
    def nL(self):
        return len(self.dimL)

    def block(self, b):
        o, r, c, ld = int(self.blk_off[b]), int(self.blk_rows[b]), int(self.blk_cols[b]), int(self.blk_ld[b])
        return self.op_vals[o:o + r * ld].reshape(r, ld)[:, :c]

    def op_blocks(self, op):
        """``{in_sector: (out_sector, block)}`` of an operator."""
        return {int(self.blk_in[b]): (int(self.blk_out[b]), self.block(b))
                for b in np.nonzero(self.blk_op == op)[0]}

    def isometries(self):
        """``U_Q`` matrices (full x keep) in enlarged-sector order."""
        out = []
        for Q in range(len(self.keep)):
            full = int(self.full[Q])
            o = int(self.u_off[Q])
            out.append(self.u_vals[o:o + full * int(self.keep[Q])].reshape(full, int(self.keep[Q])))
        return out

    def terms_of(self, nu):
        sel = np.nonzero(self.term_new == nu)[0]
        return [(int(self.term_op[t]), int(self.term_mono[t]), float(self.term_coef[t])) for t in sel]


def _enlarged(qL, dimL):
    comps = {}
    for i in range(len(dimL)):
        for s in range(4):
            sq = site_q(s)
            q = (int(qL[i][0]) + sq[0], int(qL[i][1]) + sq[1])
            comps[q] = comps.get(q, 0) + int(dimL[i])
    qQ = sorted(comps)
    return np.array(qQ, dtype=np.int32).reshape(-1, 2), np.array([comps[q] for q in qQ], dtype=np.int64)


def renorm_instance(n_sites, D, mean, dmax, n_ops, n_new, seed, keep_frac=0.25, identity_every=8):
    qL, dimL = block_profile(n_sites, D, mean, dmax, seed)
    qidx = {(int(a), int(b)): i for i, (a, b) in enumerate(qL)}
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    ops = []
    while len(ops) < n_ops:
        sh = SHIFTS[rng.integers(len(SHIFTS))]
        shape = []
        for i in range(len(qL)):
            j = qidx.get((int(qL[i][0]) + sh[0], int(qL[i][1]) + sh[1]))
            if j is not None:
                shape.append((i, j))
        if shape:
            ops.append((sh, shape))
    layout, off = [], 0
    for o, (sh, shape) in enumerate(ops):
        for (i, j) in shape:
            r, c = int(dimL[j]), int(dimL[i])
            ld = _round_up(c, ALIGN)
            layout.append((o, i, j, r, c, ld, off))
            off += _round_up(r * ld, ALIGN)
    vals = np.zeros(max(off, ALIGN))
    for (o, i, j, r, c, ld, bo) in layout:
        g = np.random.Generator(np.random.Philox(key=[seed, 1 + o]))
        vals[bo:bo + r * ld].reshape(r, ld)[:, :c] = g.standard_normal((r, c)) / np.sqrt(c)
    lay = np.array(layout, dtype=np.int64).reshape(-1, 7)
    qQ, full = _enlarged(qL, dimL)
    keep = np.maximum(1, np.rint(keep_frac * full)).astype(np.int32)
    u_off = np.zeros(len(qQ), dtype=np.int64)
    parts, o = [], 0
    for Q in range(len(qQ)):
        g = np.random.Generator(np.random.Philox(key=[seed, 1000003 + Q]))
        Qm, _ = np.linalg.qr(g.standard_normal((int(full[Q]), int(full[Q]))))
        Um = np.ascontiguousarray(Qm[:, :int(keep[Q])])
        u_off[Q] = o
        parts.append(Um.reshape(-1))
        o += Um.size
    u_vals = np.concatenate(parts)
    # terms of the new operators
    op_sh = [sh for sh, _ in ops]
    t_new, t_op, t_mono, t_coef = [], [], [], []
    for nu in range(n_new):
        if identity_every and nu % identity_every == identity_every - 1:
            m = int(rng.integers(16))
            t_new.append(nu); t_op.append(-1); t_mono.append(m); t_coef.append(1.0)
            continue
        oa, ma = int(rng.integers(len(ops))), int(rng.integers(16))
        tot = (op_sh[oa][0] + MONO_SHIFT[ma][0], op_sh[oa][1] + MONO_SHIFT[ma][1])
        t_new.append(nu); t_op.append(oa); t_mono.append(ma); t_coef.append(1.0)
        if rng.random() < 0.5:
            ob = int(rng.integers(len(ops)))
            need = (tot[0] - op_sh[ob][0], tot[1] - op_sh[ob][1])
            mb = [m for m in range(16) if MONO_SHIFT[m] == need]
            if mb:
                t_new.append(nu); t_op.append(ob); t_mono.append(mb[int(rng.integers(len(mb)))])
                t_coef.append(float(rng.standard_normal()))
    return RenormInstance(
        qL=qL, dimL=dimL,
        op_dN=np.array([sh[0] for sh in op_sh], dtype=np.int32),
        op_d2Sz=np.array([sh[1] for sh in op_sh], dtype=np.int32),
        blk_op=lay[:, 0].astype(np.int32), blk_in=lay[:, 1].astype(np.int32), blk_out=lay[:, 2].astype(np.int32),
        blk_rows=lay[:, 3].astype(np.int32), blk_cols=lay[:, 4].astype(np.int32), blk_ld=lay[:, 5].astype(np.int32),
        blk_off=lay[:, 6].astype(np.int64), op_vals=vals, qQ=qQ, keep=keep, u_off=u_off, u_vals=u_vals,
        term_new=np.array(t_new, dtype=np.int32), term_op=np.array(t_op, dtype=np.int32),
        term_mono=np.array(t_mono, dtype=np.int32), term_coef=np.array(t_coef, dtype=np.float64), n_new=n_new,
        full=full)
