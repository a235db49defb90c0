"""Problem container and the seeded synthetic block-sparse instance generator.

The synthetic instances stand in for the molecular F2 / FeMoco active spaces
of the paper's results section, whose integrals are not available: they take
their shapes (orbital count, half filling, bond dimension split over (N, 2Sz)
sectors, O(L^2)-like numbers of operator terms) and nothing else.
"""

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

# Allowed (dN, d2Sz) shifts of a block operator in the synthetic instances.
SHIFTS = ((0, 0), (0, 2), (0, -2), (1, 1), (1, -1), (-1, 1), (-1, -1),
          (2, 0), (-2, 0), (2, 2), (2, -2), (-2, 2), (-2, -2))

# Site-state quantum numbers (N, 2Sz) for states 0 (empty), 1 (up), 2 (down), 3 (up-down).
_SITE_Q = ((0, 0), (1, 1), (1, -1), (2, 0))

# dN of a single-spin factor: 0 -> identity, 1 -> n, 2 -> creator, 3 -> annihilator.
_FACTOR_DN = (0, 0, 1, -1)


def site_q(state):
    return _SITE_Q[state]


def mono_id(u, d):
    return 4 * u + d


def _mono_shift(m):
    u, d = divmod(m, 4)
    du, dd = _FACTOR_DN[u], _FACTOR_DN[d]
    return (du + dd, du - dd)


MONO_SHIFT = tuple(_mono_shift(m) for m in range(16))


def mono_parity(m):
    u, d = divmod(m, 4)
    return (abs(_FACTOR_DN[u]) + abs(_FACTOR_DN[d])) % 2


_ADJ_FACTOR = (0, 1, 3, 2)


def mono_adjoint(m):
    """Id of the monomial whose factors are the adjoints of ``m``'s, and the
    sign picked up when the reversed product is put back in up-left order."""
    u, d = divmod(m, 4)
    pu, pd = abs(_FACTOR_DN[u]) % 2, abs(_FACTOR_DN[d]) % 2
    return mono_id(_ADJ_FACTOR[u], _ADJ_FACTOR[d]), (-1.0 if (pu and pd) else 1.0)


def _round_up(x, a):
    return (x + a - 1) // a * a


ALIGN = 8  # block offsets and leading dimensions are multiples of 8 elements


@dataclass
class Problem:
    """One two-site effective Hamiltonian in packed array form.

    Operators are listed with their side (0 = left block, 1 = right block) and
    quantum-number shift; their dense blocks live in ``op_vals``.  Terms are
    ``(op_L, mono_a, mono_b, op_R, coef)`` with op id -1 meaning identity.
    """
    target: tuple
    qL: np.ndarray
    dimL: np.ndarray
    qR: np.ndarray
    dimR: np.ndarray
    psi_sec: np.ndarray
    psi_off: np.ndarray
    op_side: np.ndarray
    op_dN: np.ndarray
    op_d2Sz: np.ndarray
    blk_op: np.ndarray
    blk_in: np.ndarray
    blk_out: np.ndarray
    blk_rows: np.ndarray
    blk_cols: np.ndarray
    blk_ld: np.ndarray
    blk_off: np.ndarray
    term_L: np.ndarray
    term_ma: np.ndarray
    term_mb: np.ndarray
    term_R: np.ndarray
    term_coef: np.ndarray
    op_vals: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nL(self):
        return len(self.dimL)

    @property
    def nR(self):
        return len(self.dimR)

    @property
    def nS(self):
        return len(self.psi_sec)

    @property
    def nOps(self):
        return len(self.op_side)

    @property
    def nBlk(self):
        return len(self.blk_op)

    @property
    def nTerms(self):
        return len(self.term_L)

    @property
    def psi_dim(self):
        return int(self.psi_off[-1])

    def block(self, b):
        """Dense view of block ``b`` (rows x cols)."""
        o, r, c, ld = int(self.blk_off[b]), int(self.blk_rows[b]), int(self.blk_cols[b]), int(self.blk_ld[b])
        if r == 0 or c == 0:
            return np.zeros((r, c))
        return self.op_vals[o:o + r * ld].reshape(r, ld)[:, :c]

    def op_blocks(self, op):
        """``{in_sector: block_id}`` of operator ``op``."""
        ids = np.nonzero(self.blk_op == op)[0]
        return {int(self.blk_in[b]): int(b) for b in ids}

    def psi_sector_view(self, x, s):
        iL, _, _, iR = self.psi_sec[s]
        return x[self.psi_off[s]:self.psi_off[s + 1]].reshape(int(self.dimL[iL]), int(self.dimR[iR]))

    def check_format(self):
        """Structural checks of the packed format (shapes and ranges only)."""
        assert self.qL.shape == (self.nL, 2) and self.qR.shape == (self.nR, 2)
        assert self.psi_sec.shape == (self.nS, 4)
        assert self.psi_off.shape == (self.nS + 1,) and self.psi_off[0] == 0
        for s in range(self.nS):
            iL, sa, sb, iR = (int(v) for v in self.psi_sec[s])
            assert self.psi_off[s + 1] - self.psi_off[s] == self.dimL[iL] * self.dimR[iR]
        for b in range(self.nBlk):
            assert self.blk_ld[b] >= self.blk_cols[b]
            assert self.blk_off[b] + (self.blk_rows[b] - 1) * self.blk_ld[b] + self.blk_cols[b] <= len(self.op_vals)
        return True


def pack_problem(target, qL, dimL, qR, dimR, ops, terms, meta=None):
    """Pack sector tables, operators and terms into a :class:`Problem`.

    ``ops`` is a list of ``(side, (dN, d2Sz), {in_sector: dense block})``;
    ``terms`` a list of ``(op_L, mono_a, mono_b, op_R, coef)``.  The
    wavefunction sector table is the full list of ``(iL, sa, sb, iR)`` whose
    quantum numbers add up to ``target``.
    """
    qL = np.asarray(qL, dtype=np.int32).reshape(-1, 2)
    qR = np.asarray(qR, dtype=np.int32).reshape(-1, 2)
    dimL = np.asarray(dimL, dtype=np.int32)
    dimR = np.asarray(dimR, dtype=np.int32)
    psi_sec, psi_off = psi_sector_table(target, qL, dimL, qR, dimR)

    layout = []  # (op, in, out, rows, cols, ld, off)
    off = 0
    for o, (side, shift, blocks) in enumerate(ops):
        q = qL if side == 0 else qR
        qidx = {tuple(int(v) for v in q[i]): i for i in range(len(q))}
        for i_in in sorted(blocks):
            mat = blocks[i_in]
            qo = (int(q[i_in][0]) + shift[0], int(q[i_in][1]) + shift[1])
            i_out = qidx[qo]
            r, c = mat.shape
            ld = _round_up(max(c, 1), ALIGN)
            layout.append((o, i_in, i_out, r, c, ld, off))
            off += _round_up(r * ld, ALIGN)
    vals = np.zeros(max(off, ALIGN), dtype=np.float64)
    k = 0
    for o, (side, shift, blocks) in enumerate(ops):
        for i_in in sorted(blocks):
            _, _, _, r, c, ld, bo = layout[k]
            k += 1
            vals[bo:bo + r * ld].reshape(r, ld)[:, :c] = blocks[i_in]
    return _assemble(target, qL, dimL, qR, dimR, psi_sec, psi_off, ops_meta=[(s, sh) for s, sh, _ in ops],
                     layout=layout, terms=terms, vals=vals, meta=meta)


def _assemble(target, qL, dimL, qR, dimR, psi_sec, psi_off, ops_meta, layout, terms, vals, meta):
    lay = np.array(layout, dtype=np.int64).reshape(-1, 7)
    t = list(terms)
    return Problem(
        target=(int(target[0]), int(target[1])),
        qL=qL, dimL=dimL, qR=qR, dimR=dimR, psi_sec=psi_sec, psi_off=psi_off,
        op_side=np.array([s for s, _ in ops_meta], dtype=np.int32),
        op_dN=np.array([sh[0] for _, sh in ops_meta], dtype=np.int32),
        op_d2Sz=np.array([sh[1] for _, sh in ops_meta], dtype=np.int32),
        blk_op=lay[:, 0].astype(np.int32), blk_in=lay[:, 1].astype(np.int32),
        blk_out=lay[:, 2].astype(np.int32), blk_rows=lay[:, 3].astype(np.int32),
        blk_cols=lay[:, 4].astype(np.int32), blk_ld=lay[:, 5].astype(np.int32),
        blk_off=lay[:, 6].astype(np.int64),
        term_L=np.array([x[0] for x in t], dtype=np.int32),
        term_ma=np.array([x[1] for x in t], dtype=np.int32),
        term_mb=np.array([x[2] for x in t], dtype=np.int32),
        term_R=np.array([x[3] for x in t], dtype=np.int32),
        term_coef=np.array([x[4] for x in t], dtype=np.float64),
        op_vals=vals, meta=dict(meta or {}))


def psi_sector_table(target, qL, dimL, qR, dimR):
    """All ``(iL, sa, sb, iR)`` with ``qL + q(sa) + q(sb) + qR = target``,
    sorted by ``(iL, sa, sb)``, and the packed offsets."""
    ridx = {tuple(int(v) for v in qR[i]): i for i in range(len(qR))}
    sec = []
    for iL in range(len(qL)):
        for sa in range(4):
            for sb in range(4):
                need = (target[0] - int(qL[iL][0]) - _SITE_Q[sa][0] - _SITE_Q[sb][0],
                        target[1] - int(qL[iL][1]) - _SITE_Q[sa][1] - _SITE_Q[sb][1])
                iR = ridx.get(need)
                if iR is not None:
                    sec.append((iL, sa, sb, iR))
    psi_sec = np.array(sec, dtype=np.int32).reshape(-1, 4)
    sizes = np.array([int(dimL[s[0]]) * int(dimR[s[3]]) for s in sec], dtype=np.int64)
    psi_off = np.zeros(len(sec) + 1, dtype=np.int64)
    psi_off[1:] = np.cumsum(sizes)
    return psi_sec, psi_off


def gaussian_psi(prob, seed):
    """Gaussian entries on every wavefunction sector, global 2-norm one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(prob.psi_dim)
    return x / np.linalg.norm(x)


def gapped_guess(prob, seed, noise=1e-2):
    """Starting vector for the gapped variant: the unit vector on the element
    whose designed diagonal energy (block ladders plus site energies) is
    lowest, plus ``noise`` times a Gaussian vector, normalised.  A DMRG
    iteration starts from the previous wavefunction; this stands in for it."""
    nl, nr = prob.meta["nl"], prob.meta["nr"]
    best, where = None, None
    site_e = np.zeros((4, 4))
    for (ma, mb, e) in SITE_ENERGIES:
        for sa in range(4):
            for sb in range(4):
                ua, da = divmod(ma, 4)
                ub, db = divmod(mb, 4)
                occ_a = (1 if ua == 0 else (sa & 1)) * (1 if da == 0 else (sa >> 1) & 1)
                occ_b = (1 if ub == 0 else (sb & 1)) * (1 if db == 0 else (sb >> 1) & 1)
                site_e[sa, sb] += e * occ_a * occ_b
    for s in range(prob.nS):
        iL, sa, sb, iR = (int(v) for v in prob.psi_sec[s])
        rl = (int(prob.qL[iL][0]) - nl) ** 2 + (int(prob.qL[iL][1]) - nl % 2) ** 2
        rr = (int(prob.qR[iR][0]) - nr) ** 2 + (int(prob.qR[iR][1]) - nr % 2) ** 2
        e = 2.0 + 0.5 * (rl + rr) + site_e[sa, sb]
        if best is None or e < best:
            best, where = e, int(prob.psi_off[s])
    x = noise * gaussian_psi(prob, seed)
    x[where] += 1.0
    return x / np.linalg.norm(x)


# ----------------------------------------------------------------------------
# Synthetic block profile
# ----------------------------------------------------------------------------

def _grid(n_sites):
    pts = []
    for N in range(0, 2 * n_sites + 1):
        m = min(N, 2 * n_sites - N)
        for s2 in range(-m, m + 1, 2):
            pts.append((N, s2))
    return pts


def block_profile(n_sites, D, mean, dmax, seed):
    """Sector quantum numbers and sizes of one block.

    The ``round(D/mean)`` grid points closest to half filling get sizes from a
    Gaussian profile of peak ``dmax`` with a 10% log-normal jitter; the width
    is bisected so that the sizes sum to ``D`` after a cyclic +-1 fix-up.
    Returns ``(q[n,2], dims[n])`` sorted by (N, 2Sz).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Nc, Sc = n_sites, n_sites % 2
    pts = sorted(_grid(n_sites), key=lambda p: ((p[0] - Nc) ** 2 + (p[1] - Sc) ** 2, p[0], p[1]))
    nsec = max(1, min(len(pts), int(round(D / mean))))
    pts = pts[:nsec]
    r2 = np.array([(p[0] - Nc) ** 2 + (p[1] - Sc) ** 2 for p in pts], dtype=np.float64)
    xi = np.concatenate([[0.0], rng.standard_normal(nsec - 1)])
    jit = np.exp(0.1 * xi)

    def sizes(s):
        d = np.rint(dmax * np.exp(-r2 / (2.0 * s * s)) * jit)
        return np.clip(d, 1, dmax).astype(np.int64)

    lo, hi = 1e-3, 1e3
    if sizes(hi).sum() <= D:
        d = sizes(hi)
    else:
        for _ in range(200):
            mid = np.sqrt(lo * hi)
            if sizes(mid).sum() <= D:
                lo = mid
            else:
                hi = mid
        d = sizes(lo)
    order = sorted(range(nsec), key=lambda j: pts[j])
    q = np.array([pts[j] for j in order], dtype=np.int32)
    d = d[order]
    # cyclic fix-up in canonical order
    j = 0
    guard = 0
    while d.sum() != D and guard < 10 * D + 100:
        if d.sum() < D and d[j] < dmax:
            d[j] += 1
        elif d.sum() > D and d[j] > 1:
            d[j] -= 1
        j = (j + 1) % nsec
        guard += 1
    return q, d.astype(np.int32)


def _op_blocks_shape(q, dims, shift):
    """``[(in, out, rows, cols)]`` of a block operator with the given shift."""
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(q)}
    out = []
    for i in range(len(q)):
        j = idx.get((int(q[i][0]) + shift[0], int(q[i][1]) + shift[1]))
        if j is not None:
            out.append((i, j, int(dims[j]), int(dims[i])))
    return out


# (mono_a, mono_b, energy) of the gapped variant: n_up and n_down on each site
SITE_ENERGIES = ((mono_id(1, 0), 0, 0.25), (mono_id(0, 1), 0, 0.5),
                 (0, mono_id(1, 0), 0.35), (0, mono_id(0, 1), 0.15))


def synthetic_problem(L, N, twoSz, D, mean, dmax, K, seed, gapped=False, lam=0.05,
                      threads=None, with_values=True, share=1):
    """Seeded synthetic block-sparse two-site problem.

    * Left block = ``L//2 - 1`` orbitals, right block the rest minus the two
      sites, both with the Gaussian sector profile of :func:`block_profile`
      (right block seeded with ``seed + 1``).
    * ``K/2`` random terms (shift of the left operator from :data:`SHIFTS`,
      random site monomials, right shift fixed by conservation and rejected if
      not in :data:`SHIFTS`), each with its adjoint, so that H is symmetric.
      Every block entry is ``N(0, 1/cols)``; each operator has its own
      counter-based stream keyed by ``(seed, operator index)``.
    * ``gapped``: two diagonal block Hamiltonians ``H_L x 1 x 1 x 1`` and
      ``1 x 1 x 1 x H_R`` (entries ``1 + i/d + 0.5 r^2`` inside a sector of
      size ``d`` whose distance from half filling is ``r``), spin-dependent
      site energies (:data:`SITE_ENERGIES`) and the random terms scaled by
      ``lam``, which isolates the lowest eigenvalue.
    * ``share`` > 1: each random operator pair serves up to ``share`` terms
      (the first monomial pair and further distinct ones of the same total
      shift), as the normal and complementary operators of a block serve
      several site monomials; the term count stays ``K``.
    """
    nl = L // 2 - 1
    nr = L - nl - 2
    qL, dimL = block_profile(nl, D, mean, dmax, seed)
    qR, dimR = block_profile(nr, D, mean, dmax, seed + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    shifts = set(SHIFTS)
    ops_meta = []   # (side, shift)
    ops_shape = []  # list of [(in, out, rows, cols)]
    ops_src = []    # None for random ops, ("adj", k) for transposes, ("diag", side) for gapped
    terms = []
    coef = lam if gapped else 1.0
    npairs = K // 2
    while len(terms) < 2 * npairs:
        dL = SHIFTS[rng.integers(len(SHIFTS))]
        ma = int(rng.integers(16))
        mb = int(rng.integers(16))
        sa, sb = MONO_SHIFT[ma], MONO_SHIFT[mb]
        dR = (-(dL[0] + sa[0] + sb[0]), -(dL[1] + sa[1] + sb[1]))
        if dR not in shifts:
            continue
        shL = _op_blocks_shape(qL, dimL, dL)
        shR = _op_blocks_shape(qR, dimR, dR)
        if not shL or not shR:
            continue
        oL = len(ops_meta)
        ops_meta += [(0, dL), (1, dR)]
        ops_shape += [shL, shR]
        ops_src += [None, None]
        oR = oL + 1
        # adjoint operators: transposed blocks, opposite shifts
        ops_meta += [(0, (-dL[0], -dL[1])), (1, (-dR[0], -dR[1]))]
        ops_shape += [[(o, i, c, r) for (i, o, r, c) in shL], [(o, i, c, r) for (i, o, r, c) in shR]]
        ops_src += [("adj", oL), ("adj", oR)]
        pL, pR = abs(dL[0]) % 2, abs(dR[0]) % 2
        def pair_terms(ma, mb):
            ma2, ga = mono_adjoint(ma)
            mb2, gb = mono_adjoint(mb)
            pa, pb = mono_parity(ma), mono_parity(mb)
            par = [pL, pa, pb, pR]
            npair = sum(par[x] * par[y] for x in range(4) for y in range(x + 1, 4))
            g = (-1.0 if npair % 2 else 1.0) * ga * gb
            return [(oL, ma, mb, oR, coef), (oL + 2, ma2, mb2, oR + 2, coef * g)]

        terms += pair_terms(ma, mb)
        if share > 1:
            tot = (sa[0] + sb[0], sa[1] + sb[1])
            alt = [(x, y) for x in range(16) for y in range(16) if (x, y) != (ma, mb)
                   and (MONO_SHIFT[x][0] + MONO_SHIFT[y][0], MONO_SHIFT[x][1] + MONO_SHIFT[y][1]) == tot]
            for k in rng.permutation(len(alt))[:share - 1]:
                if len(terms) >= 2 * npairs:
                    break
                terms += pair_terms(*alt[int(k)])
    if gapped:
        for side, (q, dims) in enumerate(((qL, dimL), (qR, dimR))):
            ops_meta.append((side, (0, 0)))
            ops_shape.append([(i, i, int(dims[i]), int(dims[i])) for i in range(len(q))])
            ops_src.append(("diag", side))
        nb = len(ops_meta)
        terms.append((nb - 2, 0, 0, -1, 1.0))
        terms.append((-1, 0, 0, nb - 1, 1.0))
        # spin-dependent site energies lift the degeneracy of the site states
        for (ma, mb, e) in SITE_ENERGIES:
            terms.append((-1, ma, mb, -1, e))

    # layout
    layout = []
    off = 0
    op_first_blk = []
    for o, shp in enumerate(ops_shape):
        op_first_blk.append(len(layout))
        for (i, j, r, c) in sorted(shp):
            ld = _round_up(max(c, 1), ALIGN)
            layout.append((o, i, j, r, c, ld, off))
            off += _round_up(r * ld, ALIGN)
    op_first_blk.append(len(layout))
    psi_sec, psi_off = psi_sector_table((N, twoSz), qL, dimL, qR, dimR)
    meta = dict(kind="synthetic", L=L, N=N, twoSz=twoSz, D=D, mean=mean, dmax=dmax, K=K, seed=seed,
                gapped=gapped, lam=lam if gapped else None, nl=nl, nr=nr)
    if not with_values:
        vals = np.zeros(ALIGN)
        meta["n_vals"] = off
    else:
        vals = np.empty(max(off, ALIGN), dtype=np.float64)
        _fill_values(vals, layout, op_first_blk, ops_src, (qL, dimL, qR, dimR, nl, nr), seed, threads)
    return _assemble((N, twoSz), qL, dimL, qR, dimR, psi_sec, psi_off, ops_meta, layout, terms, vals, meta)


def _fill_values(vals, layout, op_first_blk, ops_src, tables, seed, threads):
    qL, dimL, qR, dimR, nl, nr = tables
    nops = len(ops_src)

    def fill_random(o):
        # one counter-based stream per operator, keyed by (seed, operator)
        g = np.random.Generator(np.random.Philox(key=[seed & 0xFFFFFFFFFFFFFFFF, o]))
        for b in range(op_first_blk[o], op_first_blk[o + 1]):
            _, i, j, r, c, ld, bo = layout[b]
            v = vals[bo:bo + r * ld]
            g.standard_normal(out=v)
            v *= 1.0 / np.sqrt(c)
            if ld > c:
                v.reshape(r, ld)[:, c:] = 0.0

    def fill_derived(o):
        src = ops_src[o]
        if src[0] == "adj":
            so = src[1]
            sblk = {(layout[b][1], layout[b][2]): b for b in range(op_first_blk[so], op_first_blk[so + 1])}
            for b in range(op_first_blk[o], op_first_blk[o + 1]):
                _, i, j, r, c, ld, bo = layout[b]
                sb = sblk[(j, i)]
                _, _, _, sr, sc, sld, sbo = layout[sb]
                dst = vals[bo:bo + r * ld].reshape(r, ld)
                dst[:, :c] = vals[sbo:sbo + sr * sld].reshape(sr, sld)[:, :sc].T
                dst[:, c:] = 0.0
        else:
            side = src[1]
            q, dims, nsite = (qL, dimL, nl) if side == 0 else (qR, dimR, nr)
            Nc, Sc = nsite, nsite % 2
            for b in range(op_first_blk[o], op_first_blk[o + 1]):
                _, i, j, r, c, ld, bo = layout[b]
                r2 = (int(q[i][0]) - Nc) ** 2 + (int(q[i][1]) - Sc) ** 2
                d = int(dims[i])
                v = vals[bo:bo + r * ld].reshape(r, ld)
                v[:] = 0.0
                v[np.arange(d), np.arange(d)] = 1.0 + np.arange(d) / d + 0.5 * r2

    prim = [o for o in range(nops) if ops_src[o] is None]
    der = [o for o in range(nops) if ops_src[o] is not None]
    nthr = threads or min(16, os.cpu_count() or 1)
    if nthr > 1 and len(prim) > 8:
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(fill_random, prim))
            list(ex.map(fill_derived, der))
    else:
        for o in prim:
            fill_random(o)
        for o in der:
            fill_derived(o)
