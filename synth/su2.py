"""Seeded inputs of the spin-adapted (SU(2)) two-block product (Section IV.E):
blocks whose sectors are spin multiplets (N, S), reduced operator blocks of
tensor operators, and terms that couple a left and a right tensor operator of
the same rank to a spin scalar.  Inputs only: the product itself (and its
recoupling scalars) is computed by the oracle and by the GPU library.

Conventions (readings; the paper names the variant without its formulas):

* A block of ``l`` orbitals has modes ``2 i + s`` (``s`` = 0 up, 1 down);
  its Fock states are bit strings, ``c+_p`` carries the Jordan-Wigner sign of
  the occupied modes below ``p``.
* Sector (N, S) holds the highest-weight states (M = S) of the spin-S
  multiplets with N electrons: an orthonormal basis of the kernel of S+ in
  the (N, 2Sz = 2S) Fock sector, turned by a seeded random rotation and cut
  to its first ``keep_frac`` part (at least one multiplet).
* Tensor operators (rank k, component q):  ``cd_i`` (k = 1/2):
  c+_{i up}, c+_{i dn};  ``ct_i`` (k = 1/2): c_{i dn}, -c_{i up};  ``S_i``
  (k = 1): -S+_i / sqrt 2, Sz_i, S-_i / sqrt 2;  ``n_i`` and the block
  Hamiltonian ``H`` (k = 0).
* Reduced matrix elements in the Clebsch-Gordan convention
  <j' m'| T_q |j m> = <j m; k q | j' m'> <j'||T||j>, read off the
  highest-weight states.
* A term ``(O_L, O_R, coef)`` is coef [O_L x O_R]^0 = coef sum_q <k q; k -q|0 0>
  O_L,q O_R,-q (left factor first); identity = -1 (rank 0).
* The physical two-block Hamiltonian: H_L + H_R + sum t_ij sum_s (c+_is c_js
  + h.c.) + sum J_ij S_i.S_j + sum V_ij n_i n_j over i in L, j in R, i.e. the
  terms -sqrt2 t [cd_i x ct_j]^0, -sqrt2 t [ct_i x cd_j]^0, -sqrt3 J [S_i x S_j]^0
  and V [n_i x n_j]^0.
* Layout for the library: sectors ascending by (N, 2S); block rows padded to a
  multiple of 8 elements, offsets multiples of 8.
"""

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import scipy.linalg

ALIGN = 8


@lru_cache(maxsize=None)
def cg2(j1, m1, j2, m2, j, m):
    """Clebsch-Gordan coefficient <j1 m1; j2 m2 | j m> with every argument
    doubled (sympy's exact value as a float)."""
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan
    return float(clebsch_gordan(Rational(j1, 2), Rational(j2, 2), Rational(j, 2), Rational(m1, 2), Rational(m2, 2),
                                Rational(m, 2)))


# --- block Fock space ------------------------------------------------------------

def ladder(l, p, create):
    """Matrix of c+_p (create) or c_p on the 4^l Fock states of l orbitals."""
    n = 4 ** l
    M = np.zeros((n, n))
    for st in range(n):
        occ = (st >> p) & 1
        if occ == create:
            continue
        sg = -1.0 if bin(st & ((1 << p) - 1)).count("1") & 1 else 1.0
        M[st ^ (1 << p), st] = sg
    return M


class BlockSpace:
    """Fock-space matrices of one block of ``l`` orbitals."""

    def __init__(self, l):
        self.l = l
        self.n = 4 ** l
        self.cd = [ladder(l, p, 1) for p in range(2 * l)]
        self.c = [ladder(l, p, 0) for p in range(2 * l)]
        occ = np.array([[(st >> p) & 1 for p in range(2 * l)] for st in range(self.n)])
        self.N = occ.sum(axis=1)
        self.twoSz = occ[:, 0::2].sum(axis=1) - occ[:, 1::2].sum(axis=1)

    def num(self, i):
        return self.cd[2 * i] @ self.c[2 * i] + self.cd[2 * i + 1] @ self.c[2 * i + 1]

    def splus(self, i):
        return self.cd[2 * i] @ self.c[2 * i + 1]

    def sminus(self, i):
        return self.cd[2 * i + 1] @ self.c[2 * i]

    def sz(self, i):
        return 0.5 * (self.cd[2 * i] @ self.c[2 * i] - self.cd[2 * i + 1] @ self.c[2 * i + 1])

    def total(self, f):
        return sum(f(i) for i in range(self.l))

    def hamiltonian(self, hop, U, eps):
        """Spin-scalar block Hamiltonian: sum_{i<j} hop[i,j] sum_s (c+_is c_js +
        h.c.) + sum_i U[i] n_i,up n_i,dn + sum_i eps[i] n_i."""
        H = np.zeros((self.n, self.n))
        for i in range(self.l):
            for j in range(i + 1, self.l):
                for s in range(2):
                    h = self.cd[2 * i + s] @ self.c[2 * j + s]
                    H += hop[i, j] * (h + h.T)
            H += U[i] * (self.cd[2 * i] @ self.c[2 * i]) @ (self.cd[2 * i + 1] @ self.c[2 * i + 1])
            H += eps[i] * self.num(i)
        return H

    def tensor(self, kind, i, blockH=None):
        """(2k, dN, {2q: matrix}) of a tensor operator of the block."""
        if kind == "cd":
            return 1, 1, {1: self.cd[2 * i], -1: self.cd[2 * i + 1]}
        if kind == "ct":
            return 1, -1, {1: self.c[2 * i + 1], -1: -self.c[2 * i]}
        if kind == "S":
            r = 1 / np.sqrt(2)
            return 2, 0, {2: -r * self.splus(i), 0: self.sz(i), -2: r * self.sminus(i)}
        if kind == "n":
            return 0, 0, {0: self.num(i)}
        if kind == "H":
            return 0, 0, {0: blockH}
        raise ValueError(kind)


def check_tensor(space, twok, comps):
    """Assert the commutation relations of a rank-k tensor operator with the
    block's total spin: [Sz, T_q] = q T_q, [S+-, T_q] = sqrt(k(k+1) - q(q+-1)) T_q+-1."""
    Sp, Sm, Sz = space.total(space.splus), space.total(space.sminus), space.total(space.sz)
    k = twok / 2
    for q2, T in comps.items():
        q = q2 / 2
        assert np.allclose(Sz @ T - T @ Sz, q * T)
        up = comps.get(q2 + 2, np.zeros_like(T))
        dn = comps.get(q2 - 2, np.zeros_like(T))
        assert np.allclose(Sp @ T - T @ Sp, np.sqrt(max(k * (k + 1) - q * (q + 1), 0)) * up)
        assert np.allclose(Sm @ T - T @ Sm, np.sqrt(max(k * (k + 1) - q * (q - 1), 0)) * dn)


def multiplets(space, keep_frac, rng):
    """Sectors [(N, 2S)] ascending and the highest-weight vectors of each
    (columns, Fock coordinates of the block), rotated and truncated."""
    Sp = space.total(space.splus)
    out_q, out_v = [], []
    for N in range(2 * space.l + 1):
        for twoS in range(0, 2 * space.l + 1):
            cols = np.nonzero((space.N == N) & (space.twoSz == twoS))[0]
            if len(cols) == 0:
                continue
            rows = np.nonzero((space.N == N) & (space.twoSz == twoS + 2))[0]
            if len(rows):
                K = scipy.linalg.null_space(Sp[np.ix_(rows, cols)])
            else:
                K = np.eye(len(cols))
            d = K.shape[1]
            if d == 0:
                continue
            Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
            keep = max(1, int(round(keep_frac * d)))
            V = np.zeros((space.n, keep))
            V[cols] = (K @ Q)[:, :keep]
            out_q.append((N, twoS))
            out_v.append(V)
    return out_q, out_v


def reduced_blocks(q, V, twok, dN, comps):
    """{(in, out): reduced block} of a tensor operator between the sectors
    (q, V) of one block (zero blocks left out)."""
    idx = {qq: i for i, qq in enumerate(q)}
    out = {}
    for i, (N, s2) in enumerate(q):
        for s2o in range(abs(s2 - twok), s2 + twok + 1, 2):
            j = idx.get((N + dN, s2o))
            if j is None:
                continue
            q2 = s2o - s2
            B = V[j].T @ comps[q2] @ V[i] / cg2(s2, s2, twok, q2, s2o, s2o)
            if np.max(np.abs(B)) > 1e-13:
                out[(i, j)] = B
    return out


@dataclass
class Su2Instance:
    """Packed two-block SU(2) problem plus what the oracle needs to rebuild
    the Fock-space operators (orbital counts, operator definitions, block
    Hamiltonian parameters, highest-weight vectors)."""
    target: tuple            # (N, 2S)
    lL: int
    lR: int
    qL: np.ndarray           # [nL, 2] (N, 2S)
    dimL: np.ndarray
    qR: np.ndarray
    dimR: np.ndarray
    op_side: np.ndarray
    op_2k: np.ndarray
    op_dN: np.ndarray
    op_def: list             # (side, kind, orbital)
    blk_op: np.ndarray
    blk_in: np.ndarray
    blk_out: np.ndarray
    blk_rows: np.ndarray
    blk_cols: np.ndarray
    blk_ld: np.ndarray
    blk_off: np.ndarray
    op_vals: np.ndarray
    term_L: np.ndarray
    term_R: np.ndarray
    term_coef: np.ndarray
    hw_L: list               # highest-weight vectors per left sector (4^lL x dim)
    hw_R: list
    hblk: dict               # side -> (hop, U, eps)
    params: dict             # t, J, V between the blocks

    @property
    def nOps(self):
        return len(self.op_side)

    def psi_sectors(self):
        """[(iL, iR)] in canonical order (iL major) with N_L + N_R = N and
        |S_L - S_R| <= S <= S_L + S_R."""
        N, s2 = self.target
        out = []
        for a in range(len(self.dimL)):
            for b in range(len(self.dimR)):
                nl, sl = self.qL[a]
                nr, sr = self.qR[b]
                if nl + nr == N and abs(sl - sr) <= s2 <= sl + sr and (sl + sr + s2) % 2 == 0:
                    out.append((a, b))
        return out

    @property
    def nS(self):
        return len(self.psi_sectors())

    def psi_off(self):
        secs = self.psi_sectors()
        off = [0]
        for a, b in secs:
            off.append(off[-1] + int(self.dimL[a]) * int(self.dimR[b]))
        return np.array(off, dtype=np.int64)

    @property
    def psi_dim(self):
        return int(self.psi_off()[-1])

    def block(self, b):
        o, r, c, ld = int(self.blk_off[b]), int(self.blk_rows[b]), int(self.blk_cols[b]), int(self.blk_ld[b])
        return self.op_vals[o:o + r * ld].reshape(r, ld)[:, :c]


def _pack(blocks_of_op):
    """Lay out [(op, in, out, B)] with rows padded to multiples of 8."""
    lay, off = [], 0
    for (o, i, j, B) in blocks_of_op:
        r, c = B.shape
        ld = (c + ALIGN - 1) // ALIGN * ALIGN
        lay.append((o, i, j, r, c, ld, off, B))
        off += (r * ld + ALIGN - 1) // ALIGN * ALIGN
    vals = np.zeros(max(off, ALIGN))
    for (o, i, j, r, c, ld, bo, B) in lay:
        vals[bo:bo + r * ld].reshape(r, ld)[:, :c] = B
    return lay, vals


def su2_instance(lL, lR, target, seed, keep_frac=1.0, hops=True, heis=True, dens=True):
    """Two-block spin-adapted instance from Fock-space tensor operators (exact
    reduced blocks; keep_frac < 1 truncates the multiplet bases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spaces = (BlockSpace(lL), BlockSpace(lR))
    qs, hws, hblk, Hs = [], [], {}, []
    for side, sp in enumerate(spaces):
        q, V = multiplets(sp, keep_frac, rng)
        qs.append(q)
        hws.append(V)
        hop = np.triu(rng.standard_normal((sp.l, sp.l)), 1)
        U = rng.uniform(0.5, 2.0, sp.l)
        eps = rng.uniform(-1.0, 0.0, sp.l)
        hblk[side] = (hop, U, eps)
        Hs.append(sp.hamiltonian(hop, U, eps))
    defs = []
    for side, sp in enumerate(spaces):
        defs.append((side, "H", -1))
        for i in range(sp.l):
            defs += [(side, "cd", i), (side, "ct", i), (side, "S", i), (side, "n", i)]
    op_id = {d: k for k, d in enumerate(defs)}
    op_side, op_2k, op_dN, blocks = [], [], [], []
    for k, (side, kind, i) in enumerate(defs):
        sp = spaces[side]
        twok, dN, comps = sp.tensor(kind, i, Hs[side])
        check_tensor(sp, twok, comps)
        op_side.append(side)
        op_2k.append(twok)
        op_dN.append(dN)
        for (a, b), B in sorted(reduced_blocks(qs[side], hws[side], twok, dN, comps).items()):
            blocks.append((k, a, b, B))
    t = rng.standard_normal((lL, lR)) * 0.5
    J = rng.standard_normal((lL, lR)) * 0.3
    Vd = rng.standard_normal((lL, lR)) * 0.2
    terms = [(op_id[(0, "H", -1)], -1, 1.0), (-1, op_id[(1, "H", -1)], 1.0)]
    for i in range(lL):
        for j in range(lR):
            if hops:
                terms.append((op_id[(0, "cd", i)], op_id[(1, "ct", j)], -np.sqrt(2) * t[i, j]))
                terms.append((op_id[(0, "ct", i)], op_id[(1, "cd", j)], -np.sqrt(2) * t[i, j]))
            if heis:
                terms.append((op_id[(0, "S", i)], op_id[(1, "S", j)], -np.sqrt(3) * J[i, j]))
            if dens:
                terms.append((op_id[(0, "n", i)], op_id[(1, "n", j)], Vd[i, j]))
    lay, vals = _pack(blocks)
    col = lambda k, dt: np.array([x[k] for x in lay], dtype=dt)
    return Su2Instance(
        target=tuple(target), lL=lL, lR=lR,
        qL=np.array(qs[0], dtype=np.int32).reshape(-1, 2), dimL=np.array([v.shape[1] for v in hws[0]], dtype=np.int32),
        qR=np.array(qs[1], dtype=np.int32).reshape(-1, 2), dimR=np.array([v.shape[1] for v in hws[1]], dtype=np.int32),
        op_side=np.array(op_side, dtype=np.int32), op_2k=np.array(op_2k, dtype=np.int32),
        op_dN=np.array(op_dN, dtype=np.int32), op_def=defs,
        blk_op=col(0, np.int32), blk_in=col(1, np.int32), blk_out=col(2, np.int32), blk_rows=col(3, np.int32),
        blk_cols=col(4, np.int32), blk_ld=col(5, np.int32), blk_off=col(6, np.int64), op_vals=vals,
        term_L=np.array([x[0] for x in terms], dtype=np.int32), term_R=np.array([x[1] for x in terms], dtype=np.int32),
        term_coef=np.array([x[2] for x in terms], dtype=np.float64),
        hw_L=hws[0], hw_R=hws[1], hblk=hblk, params={"t": t, "J": J, "V": Vd})


def su2_synthetic(nsec_N, D, dmax, n_ops, n_terms, target, seed, max_2S=6):
    """Synthetic spin-adapted instance at scale (random reduced blocks, no
    Fock space): each block has sectors (N, 2S) for N in a window of
    ``nsec_N`` particle numbers around the target's half and 2S <= max_2S
    with matching parity, multiplet counts from a Gaussian profile summing to
    about D (at most dmax); ``n_ops`` operators per side with rank 0, 1/2 or 1
    (spinors change N by one, the others by 0), blocks N(0, 1/cols) on every
    sector pair the rank allows; ``n_terms`` terms pairing a left and a right
    operator of equal rank and opposite dN."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N, s2t = target
    half = N // 2
    sides = []
    for side in range(2):
        q, d = [], []
        for n in range(half - nsec_N // 2, half - nsec_N // 2 + nsec_N):
            for s2 in range(n % 2, max_2S + 1, 2):
                q.append((n, s2))
        w = np.array([np.exp(-((qq[0] - half) ** 2) / 4.0 - (qq[1] / 2) ** 2 / 6.0) for qq in q])
        dims = np.maximum(1, np.minimum(dmax, np.rint(D * w / w.sum()))).astype(np.int32)
        sides.append((q, dims))
    ranks = [(0, 0), (1, 1), (1, -1), (2, 0)]
    ops, blocks = [], []
    for side in range(2):
        q, dims = sides[side]
        idx = {qq: i for i, qq in enumerate(q)}
        for _ in range(n_ops):
            twok, dN = ranks[rng.integers(len(ranks))]
            o = len(ops)
            ops.append((side, twok, dN))
            for i, (n, s2) in enumerate(q):
                for s2o in range(abs(s2 - twok), s2 + twok + 1, 2):
                    j = idx.get((n + dN, s2o))
                    if j is None:
                        continue
                    g = np.random.Generator(np.random.Philox(key=[seed, ((1 + o) << 32) | (i << 16) | j]))
                    blocks.append((o, i, j, g.standard_normal((int(dims[j]), int(dims[i]))) / np.sqrt(dims[i])))
    left = [k for k, o in enumerate(ops) if o[0] == 0]
    right = [k for k, o in enumerate(ops) if o[0] == 1]
    terms = []
    while len(terms) < n_terms:
        a = left[rng.integers(len(left))]
        match = [b for b in right if ops[b][1] == ops[a][1] and ops[b][2] == -ops[a][2]]
        if match:
            terms.append((a, match[rng.integers(len(match))], float(rng.standard_normal())))
    lay, vals = _pack(blocks)
    col = lambda k, dt: np.array([x[k] for x in lay], dtype=dt)
    return Su2Instance(
        target=tuple(target), lL=0, lR=0,
        qL=np.array(sides[0][0], dtype=np.int32).reshape(-1, 2), dimL=sides[0][1],
        qR=np.array(sides[1][0], dtype=np.int32).reshape(-1, 2), dimR=sides[1][1],
        op_side=np.array([o[0] for o in ops], dtype=np.int32), op_2k=np.array([o[1] for o in ops], dtype=np.int32),
        op_dN=np.array([o[2] for o in ops], dtype=np.int32), op_def=[],
        blk_op=col(0, np.int32), blk_in=col(1, np.int32), blk_out=col(2, np.int32), blk_rows=col(3, np.int32),
        blk_cols=col(4, np.int32), blk_ld=col(5, np.int32), blk_off=col(6, np.int64), op_vals=vals,
        term_L=np.array([x[0] for x in terms], dtype=np.int32), term_R=np.array([x[1] for x in terms], dtype=np.int32),
        term_coef=np.array([x[2] for x in terms], dtype=np.float64),
        hw_L=[], hw_R=[], hblk={}, params={})
