"""Oracle of the spin-adapted (SU(2)) two-block product (Section IV.E).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it; the library never does.

The spin-adapted product is sigma = V^T H V psi by definition, in the
reading of the conventions documented with the instance generator:

* H is the two-block Hamiltonian on the Fock space of all lL + lR orbitals
  (left orbitals first, so a determinant is the left bit string in the low
  bits), the sum over terms of coef [O_L x O_R]^0 = coef sum_q
  <k q; k -q | 0 0> O_L,q O_R,-q (left factor first), every tensor-operator
  component built here from ladder operators on that space;
* the columns of V are the coupled states
  |(aL SL)(aR SR); S, M = S> = sum_mL <SL mL; SR S-mL | S S> |aL SL mL> |aR SR S-mL>
  of every wavefunction sector (canonical order, row-major inside a sector),
  the block states |a S m> obtained from the given highest-weight vectors by
  repeated lowering with the block's S- and normalisation.

In :func:`sigma` no recoupling coefficient enters: the Clebsch-Gordan
coefficients (sympy's exact values) only build the coupled states and the
scalar products, and the block Hamiltonians are rebuilt from their
parameters.  :func:`sigma_reduced` is the Wigner-Eckart route on the reduced
blocks (each sector pair's coefficient by expanding the coupled states),
for instances that have no Fock space; it is pinned to :func:`sigma`.
"""

from functools import lru_cache

import numpy as np
import scipy.sparse as sp


@lru_cache(maxsize=None)
def _cg(j1, m1, j2, m2, j, m):
    """<j1 m1; j2 m2 | j m>, arguments doubled (sympy, exact)."""
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan
    return float(clebsch_gordan(Rational(j1, 2), Rational(j2, 2), Rational(j, 2), Rational(m1, 2), Rational(m2, 2),
                                Rational(m, 2)))


class FullSpace:
    """Sparse ladder operators on the Fock space of ``n`` orbitals (mode
    2 i + s, Jordan-Wigner sign of the occupied modes below)."""

    def __init__(self, n):
        self.n = n
        self.dim = 4 ** n
        st = np.arange(self.dim)
        self.cd, self.c = [], []
        for p in range(2 * n):
            empty = ((st >> p) & 1) == 0
            below = st & ((1 << p) - 1)
            par = np.array([bin(int(x)).count("1") & 1 for x in below])
            sign = np.where(par, -1.0, 1.0)
            src = st[empty]
            M = sp.csr_matrix((sign[empty], (src | (1 << p), src)), shape=(self.dim, self.dim))
            self.cd.append(M)
            self.c.append(M.T.tocsr())

    def n_op(self, i):
        return self.cd[2 * i] @ self.c[2 * i] + self.cd[2 * i + 1] @ self.c[2 * i + 1]

    def s_plus(self, i):
        return self.cd[2 * i] @ self.c[2 * i + 1]

    def s_minus(self, i):
        return self.cd[2 * i + 1] @ self.c[2 * i]

    def s_z(self, i):
        return 0.5 * (self.cd[2 * i] @ self.c[2 * i] - self.cd[2 * i + 1] @ self.c[2 * i + 1])

    def block_h(self, orbs, hop, U, eps):
        H = sp.csr_matrix((self.dim, self.dim))
        for a, i in enumerate(orbs):
            for b in range(a + 1, len(orbs)):
                j = orbs[b]
                for s in range(2):
                    h = self.cd[2 * i + s] @ self.c[2 * j + s]
                    H = H + hop[a, b] * (h + h.T)
            H = H + U[a] * (self.cd[2 * i] @ self.c[2 * i]) @ (self.cd[2 * i + 1] @ self.c[2 * i + 1])
            H = H + eps[a] * self.n_op(i)
        return H.tocsr()


def components(F, inst, op):
    """(2k, {2q: component}) of operator ``op`` on the full space."""
    side, kind, i = inst.op_def[op]
    orb = i + (inst.lL if side else 0)
    if kind == "cd":
        return 1, {1: F.cd[2 * orb], -1: F.cd[2 * orb + 1]}
    if kind == "ct":
        return 1, {1: F.c[2 * orb + 1], -1: -F.c[2 * orb]}
    if kind == "S":
        r = 1 / np.sqrt(2)
        return 2, {2: -r * F.s_plus(orb), 0: F.s_z(orb), -2: r * F.s_minus(orb)}
    if kind == "n":
        return 0, {0: F.n_op(orb)}
    if kind == "H":
        orbs = list(range(inst.lL, inst.lL + inst.lR)) if side else list(range(inst.lL))
        return 0, {0: F.block_h(orbs, *inst.hblk[side])}
    raise ValueError(kind)


def hamiltonian(inst, F=None):
    """H = sum over terms of coef [O_L x O_R]^0 on the full space."""
    F = F or FullSpace(inst.lL + inst.lR)
    eye = sp.identity(F.dim, format="csr")
    H = sp.csr_matrix((F.dim, F.dim))
    for oL, oR, coef in zip(inst.term_L, inst.term_R, inst.term_coef):
        kL, cL = components(F, inst, int(oL)) if oL >= 0 else (0, {0: eye})
        kR, cR = components(F, inst, int(oR)) if oR >= 0 else (0, {0: eye})
        assert kL == kR
        for q, A in cL.items():
            if -q in cR:
                H = H + (float(coef) * _cg(kL, q, kR, -q, 0, 0)) * (A @ cR[-q])
    return H.tocsr()


def _lowered(hw, twoS, l):
    """Block states |a S m> for m = S, S-1, ..., -S (doubled: twoS .. -twoS)
    of the highest-weight columns ``hw`` (4^l Fock coordinates)."""
    Fb = _block_space(l)
    Sm = Fb[1]
    out = {twoS: hw}
    cur = hw
    for m2 in range(twoS, -twoS, -2):
        cur = Sm @ cur
        nrm = np.sqrt((twoS + m2) * (twoS - m2 + 2) / 4.0)  # |S- |S m>| = sqrt((S+m)(S-m+1))
        cur = cur / nrm
        out[m2 - 2] = cur
    return out


@lru_cache(maxsize=None)
def _block_space(l):
    F = FullSpace(l)
    Sm = sum((F.s_minus(i) for i in range(l)), sp.csr_matrix((F.dim, F.dim))).tocsr()
    return F, Sm


def coupled_basis(inst):
    """V: one column per wavefunction element (sector order of
    ``inst.psi_sectors()``, row-major inside a sector)."""
    N, twoS = inst.target
    cols = []
    dL, dR = 4 ** inst.lL, 4 ** inst.lR
    low = {}
    for side, q, hws, l in ((0, inst.qL, inst.hw_L, inst.lL), (1, inst.qR, inst.hw_R, inst.lR)):
        for k, V in enumerate(hws):
            low[(side, k)] = _lowered(V, int(q[k][1]), l)
    for a, b in inst.psi_sectors():
        sl, sr = int(inst.qL[a][1]), int(inst.qR[b][1])
        A, B = low[(0, a)], low[(1, b)]
        blk = np.zeros((dL * dR, A[sl].shape[1], B[sr].shape[1]))
        for ml in range(-sl, sl + 1, 2):
            mr = twoS - ml
            if abs(mr) > sr:
                continue
            c = _cg(sl, ml, sr, mr, twoS, twoS)
            if c == 0.0:
                continue
            # determinant index = left bits + 4^lL * right bits
            blk += c * np.einsum("ri,lj->rlij", B[mr], A[ml]).reshape(dR * dL, B[mr].shape[1], A[ml].shape[1]) \
                .transpose(0, 2, 1)
        cols.append(blk.reshape(dL * dR, -1))
    return np.concatenate(cols, axis=1) if cols else np.zeros((dL * dR, 0))


def sigma(inst, psi, H=None, V=None):
    """sigma = V^T H V psi."""
    H = hamiltonian(inst) if H is None else H
    V = coupled_basis(inst) if V is None else V
    return V.T @ (H @ (V @ np.asarray(psi, dtype=np.float64)))


def direct_hamiltonian(inst, F=None):
    """The same two-block Hamiltonian from spin-orbital strings:
    H_L + H_R + sum t_ij sum_s (c+_is c_js + h.c.) + J_ij S_i.S_j + V_ij n_i n_j."""
    F = F or FullSpace(inst.lL + inst.lR)
    H = F.block_h(list(range(inst.lL)), *inst.hblk[0]) + F.block_h(list(range(inst.lL, inst.lL + inst.lR)),
                                                                   *inst.hblk[1])
    t, J, V = inst.params["t"], inst.params["J"], inst.params["V"]
    for i in range(inst.lL):
        for jj in range(inst.lR):
            j = inst.lL + jj
            for s in range(2):
                h = F.cd[2 * i + s] @ F.c[2 * j + s]
                H = H + t[i, jj] * (h + h.T)
            SS = F.s_z(i) @ F.s_z(j) + 0.5 * (F.s_plus(i) @ F.s_minus(j) + F.s_minus(i) @ F.s_plus(j))
            H = H + J[i, jj] * SS + V[i, jj] * (F.n_op(i) @ F.n_op(j))
    return H.tocsr()


def total_spin(F, n):
    """(S^2, Sz) of all n orbitals on the full space."""
    Sp = sum((F.s_plus(i) for i in range(n)), sp.csr_matrix((F.dim, F.dim)))
    Sm = sum((F.s_minus(i) for i in range(n)), sp.csr_matrix((F.dim, F.dim)))
    Sz = sum((F.s_z(i) for i in range(n)), sp.csr_matrix((F.dim, F.dim)))
    return (Sm @ Sp + Sz @ Sz + Sz).tocsr(), Sz.tocsr()


def recoupling(slp, srp, s, sl, sr, k):
    """<(SL' SR') S S| [T^k x U^k]^0 |(SL SR) S S> per unit reduced elements
    (Clebsch-Gordan convention), spins doubled: the coupled states expanded
    and the components applied by the Wigner-Eckart theorem."""
    w = 0.0
    for ml in range(-sl, sl + 1, 2):
        c_in = _cg(sl, ml, sr, s - ml, s, s)
        if c_in == 0.0:
            continue
        for q in range(-k, k + 1, 2):
            w += (c_in * _cg(k, q, k, -q, 0, 0) * _cg(sl, ml, k, q, slp, ml + q)
                  * _cg(sr, s - ml, k, -q, srp, s - ml - q) * _cg(slp, ml + q, srp, s - ml - q, s, s))
    return w


def sigma_reduced(inst, psi):
    """The same product on reduced blocks, sector by sector: for every term,
    input sector (iL, iR) and reduced blocks L: iL -> iL', R: iR -> iR' with
    (iL', iR') a wavefunction sector, sigma_(iL',iR') += coef
    (-1)^(p_R N_L) recoupling(...) L psi_(iL,iR) R^T (identity = -1).  Valid for
    instances without a Fock space (synthetic reduced blocks); pinned against
    :func:`sigma` where both apply."""
    secs = inst.psi_sectors()
    off = inst.psi_off()
    idx = {sec: n for n, sec in enumerate(secs)}
    N, s2 = inst.target
    out = np.zeros(int(off[-1]))
    blocks = {}
    for b in range(len(inst.blk_op)):
        blocks.setdefault((int(inst.blk_op[b]), int(inst.blk_in[b])), []).append(b)
    for oL, oR, coef in zip(inst.term_L, inst.term_R, inst.term_coef):
        oL, oR = int(oL), int(oR)
        k = int(inst.op_2k[oL]) if oL >= 0 else 0
        pR = abs(int(inst.op_dN[oR])) % 2 if oR >= 0 else 0
        for n, (a, b) in enumerate(secs):
            x = psi[off[n]:off[n + 1]].reshape(int(inst.dimL[a]), int(inst.dimR[b]))
            Ls = [(int(inst.blk_out[lb]), inst.block(lb)) for lb in blocks.get((oL, a), [])] if oL >= 0 \
                else [(a, None)]
            Rs = [(int(inst.blk_out[rb]), inst.block(rb)) for rb in blocks.get((oR, b), [])] if oR >= 0 \
                else [(b, None)]
            for a2, Lb in Ls:
                for b2, Rb in Rs:
                    m = idx.get((a2, b2))
                    if m is None:
                        continue
                    w = recoupling(int(inst.qL[a2][1]), int(inst.qR[b2][1]), s2, int(inst.qL[a][1]),
                                   int(inst.qR[b][1]), k)
                    sign = -1.0 if (pR * int(inst.qL[a][0])) % 2 else 1.0
                    y = x if Lb is None else Lb @ x
                    y = y if Rb is None else y @ Rb.T
                    out[off[m]:off[m + 1]] += float(coef) * w * sign * y.reshape(-1)
    return out
