"""Exact block bases, site monomials and term tables of the two-site topology.

Section III.A.1: operators are stored as dense matrices per (row, column)
quantum-number sector pair.  Section III.A.2: in the two-site topology the
modes split into four subsystems (left block, two single sites, right block);
the site factors of each operator product are one-dimensional per sector, so
they reduce to scalars; partial summation turns the O(N^4) operator strings
into O(N^2) products of normal and complementary operators.

Conventions (readings, the paper leaves them open):

* Left block = orbitals ``0..l-1``, site a = orbital ``l``, site b = orbital
  ``l+1``, right block = the rest.
* A block state is the bit string of its own modes (local mode ``m`` is
  global mode ``2*orb0 + m``); sectors (N, 2Sz) ascending; inside a sector,
  states ascending by bit string.
* The product state ``|l, sa, sb, r>`` is ``C_l C_a C_b C_r |0>`` with each
  ``C`` the block's creators in ascending mode order, i.e. the determinant
  ``bl | sa << 2l | sb << (2l+2) | br << (2l+4)`` with no extra sign.
* Site monomials are ``x_up * x_down`` with ``x`` in {1, n, c+, c}, id
  ``4*u + d`` (u, d the index of x in that list).
"""

import itertools
from collections import OrderedDict

import numpy as np

from synth.problem import pack_problem
from .fock import apply_string, hamiltonian_strings

SUB_L, SUB_A, SUB_B, SUB_R = 0, 1, 2, 3

# ---------------------------------------------------------------------------
# Site monomials (4 x 4 matrices on the site basis 0, up, down, up-down)
# ---------------------------------------------------------------------------


def _site_string_matrix(string):
    """4x4 matrix of a string of site-local ladder operators (mode 0 = up,
    mode 1 = down) in the basis |0>, |up>, |down>, |up down> = bit strings 0..3."""
    M = np.zeros((4, 4))
    for st in range(4):
        sg, out = apply_string(string, st)
        if sg:
            M[out, st] += sg
    return M


def _factor(x, spin):
    if x == 0:
        return []
    if x == 1:
        return [(spin, 1), (spin, 0)]
    if x == 2:
        return [(spin, 1)]
    return [(spin, 0)]


MONO = np.array([_site_string_matrix(_factor(u, 0) + _factor(d, 1))
                 for u in range(4) for d in range(4)])
SITE_Q = np.array([[0, 0], [1, 1], [1, -1], [2, 0]])


def identify_monomial(site_string):
    """Write a site-local string as ``sign * MONO[m]``; ``None`` if it vanishes."""
    M = _site_string_matrix(site_string)
    if not M.any():
        return None
    for m in range(16):
        for g in (1.0, -1.0):
            if np.array_equal(M, g * MONO[m]):
                return m, g
    raise ValueError("site string is not a monomial: %r" % (site_string,))


def mono_action(m, s):
    """Output state and value of monomial ``m`` on site state ``s``
    (each monomial has at most one non-zero per column)."""
    col = MONO[m][:, s]
    nz = np.nonzero(col)[0]
    if len(nz) == 0:
        return None, 0.0
    return int(nz[0]), float(col[nz[0]])


# ---------------------------------------------------------------------------
# Exact block bases
# ---------------------------------------------------------------------------


class BlockBasis:
    """All Fock states of ``norb`` consecutive orbitals, sorted into sectors."""

    def __init__(self, orb0, norb):
        self.orb0, self.norb = orb0, norb
        nm = 2 * norb
        qs = {}
        for st in range(1 << nm):
            n = bin(st).count("1")
            up = sum((st >> (2 * i)) & 1 for i in range(norb))
            qs.setdefault((n, up - (n - up)), []).append(st)
        self.q = np.array(sorted(qs), dtype=np.int32).reshape(-1, 2)
        self.states = [np.array(sorted(qs[tuple(q)]), dtype=np.int64) for q in self.q]
        self.dims = np.array([len(s) for s in self.states], dtype=np.int32)
        self.where = {}
        for i, sts in enumerate(self.states):
            for j, st in enumerate(sts):
                self.where[int(st)] = (i, j)

    def local(self, string):
        return tuple((p - 2 * self.orb0, d) for p, d in string)

    def blocks(self, local_string):
        """``(shift, {in_sector: dense block})`` of a local string; all-zero
        blocks are dropped."""
        dN = sum(1 if d else -1 for _, d in local_string)
        d2 = sum((1 if d else -1) * (1 if p % 2 == 0 else -1) for p, d in local_string)
        qidx = {(int(a), int(b)): i for i, (a, b) in enumerate(self.q)}
        out = {}
        for i, sts in enumerate(self.states):
            j = qidx.get((int(self.q[i][0]) + dN, int(self.q[i][1]) + d2))
            if j is None:
                continue
            B = np.zeros((int(self.dims[j]), int(self.dims[i])))
            for c, st in enumerate(sts):
                sg, o = apply_string(local_string, int(st))
                if sg:
                    B[self.where[o][1], c] += sg
            if B.any():
                out[i] = B
        return (dN, d2), out


# ---------------------------------------------------------------------------
# String splitting over the four subsystems
# ---------------------------------------------------------------------------


def subsystem(orb, l):
    if orb < l:
        return SUB_L
    if orb == l:
        return SUB_A
    if orb == l + 1:
        return SUB_B
    return SUB_R


def split_string(string, l):
    """Stable reordering of a string by subsystem (L, a, b, R).

    Returns ``(eps, parts)``: ``eps`` = (-1)^(number of exchanged pairs of
    factors from different subsystems), ``parts[k]`` the factors of
    subsystem ``k`` in their original relative order."""
    subs = [subsystem(p // 2, l) for p, _ in string]
    inv = sum(1 for x in range(len(subs)) for y in range(x + 1, len(subs)) if subs[x] > subs[y])
    parts = [[f for f, s in zip(string, subs) if s == k] for k in range(4)]
    return (-1.0 if inv % 2 else 1.0), parts


class Construction:
    """Block operators and term table of Eq. (2) built from integrals.

    ``grouping='naive'`` keeps one term per Hamiltonian string;
    ``grouping='complementary'`` applies the partial summation: strings with
    an empty side are summed into one operator per site-monomial pair, the
    others are grouped by the explicit string on the side with fewer factors
    (ties: the left block) and summed into a complementary operator on the
    other side.  ``provenance`` records, for each string, where its weight
    went (used for integral gradients).
    """

    def __init__(self, h, eri, N, twoSz, l=None, grouping="complementary", strings=None):
        L = h.shape[0]
        self.L = L
        self.l = l if l is not None else (3 if L == 8 else L // 2 - 1)
        l = self.l
        self.Lb = BlockBasis(0, l)
        self.Rb = BlockBasis(l + 2, L - l - 2)
        self.N, self.twoSz = N, twoSz
        self.ops = []           # (side, shift, blocks)
        self._op_cache = {}
        self.terms = []
        self.provenance = []    # (weight index, term, side or None, op, factor, blocks)
        strs = strings if strings is not None else hamiltonian_strings(h, eri, labels=True)
        self.labels = [x[2] if len(x) > 2 else None for x in strs]
        items = []
        for wi, x in enumerate(strs):
            w, s = x[0], x[1]
            eps, parts = split_string(s, l)
            a = identify_monomial(tuple((p - 2 * l, d) for p, d in parts[SUB_A]))
            b = identify_monomial(tuple((p - 2 * (l + 1), d) for p, d in parts[SUB_B]))
            if a is None or b is None:
                continue
            Ls = self.Lb.local(parts[SUB_L])
            Rs = self.Rb.local(parts[SUB_R])
            items.append((wi, w, eps * a[1] * b[1], Ls, a[0], b[0], Rs))
        if grouping == "naive":
            self._naive(items)
        else:
            self._complementary(items)

    def _op(self, side, local_string):
        key = (side, local_string)
        if key not in self._op_cache:
            basis = self.Lb if side == 0 else self.Rb
            shift, blocks = basis.blocks(local_string)
            self.ops.append((side, shift, blocks))
            self._op_cache[key] = len(self.ops) - 1
        return self._op_cache[key]

    def _naive(self, items):
        for wi, w, f, Ls, ma, mb, Rs in items:
            oL = self._op(0, Ls) if Ls else -1
            oR = self._op(1, Rs) if Rs else -1
            self.terms.append((oL, ma, mb, oR, w * f))
            self.provenance.append((wi, len(self.terms) - 1, None, -1, f, None))

    def _complementary(self, items):
        groups = OrderedDict()
        nr = self.L - self.l - 2
        for it in items:
            wi, w, f, Ls, ma, mb, Rs = it
            if not Ls and not Rs:
                key = ("scalar", ma, mb)
            elif not Rs:
                key = ("sumL", ma, mb)
            elif not Ls:
                key = ("sumR", ma, mb)
            elif len(Ls) < len(Rs) or (len(Ls) == len(Rs) and self.l <= nr):
                key = ("L", Ls, ma, mb)
            else:
                key = ("R", Rs, ma, mb)
            groups.setdefault(key, []).append(it)
        for key, its in groups.items():
            kind = key[0]
            ma, mb = its[0][4], its[0][5]
            if kind == "scalar":
                c = sum(w * f for _, w, f, _, _, _, _ in its)
                self.terms.append((-1, ma, mb, -1, c))
                for wi, w, f, *_ in its:
                    self.provenance.append((wi, len(self.terms) - 1, None, -1, f, None))
                continue
            sum_side = 0 if kind in ("sumL", "R") else 1
            basis = self.Lb if sum_side == 0 else self.Rb
            acc = {}
            shift = None
            parts = []
            for wi, w, f, Ls, _, _, Rs in its:
                sstr = Ls if sum_side == 0 else Rs
                sh, bl = basis.blocks(sstr)
                shift = sh
                parts.append((wi, f, bl))
                for i, B in bl.items():
                    acc[i] = acc.get(i, 0.0) + (w * f) * B
            acc = {i: B for i, B in acc.items() if np.any(B)}
            self.ops.append((sum_side, shift, acc))
            osum = len(self.ops) - 1
            if kind == "sumL":
                term = (osum, ma, mb, -1, 1.0)
            elif kind == "sumR":
                term = (-1, ma, mb, osum, 1.0)
            elif kind == "L":
                term = (self._op(0, key[1]), ma, mb, osum, 1.0)
            else:
                term = (osum, ma, mb, self._op(1, key[1]), 1.0)
            self.terms.append(term)
            for wi, f, bl in parts:
                self.provenance.append((wi, len(self.terms) - 1, sum_side, osum, f, bl))

    def problem(self):
        """Pack into the shared array format (see :mod:`synth`)."""
        P = pack_problem((self.N, self.twoSz), self.Lb.q, self.Lb.dims, self.Rb.q, self.Rb.dims,
                         self.ops, self.terms, meta=dict(kind="exact", L=self.L, l=self.l))
        return P

    def fci_map(self, P, dets):
        """Index of each packed wavefunction element in the FCI determinant list."""
        l = self.l
        idx = np.empty(P.psi_dim, dtype=np.int64)
        for s in range(P.nS):
            iL, sa, sb, iR = (int(v) for v in P.psi_sec[s])
            bl = self.Lb.states[iL]
            br = self.Rb.states[iR]
            d = (bl[:, None] | (sa << (2 * l)) | (sb << (2 * l + 2)) | (br[None, :] << (2 * l + 4))).reshape(-1)
            pos = np.searchsorted(dets, d)
            assert np.all(dets[pos] == d)
            idx[P.psi_off[s]:P.psi_off[s + 1]] = pos
        return idx


def free_strings(h):
    """One-body strings only (used by the free-fermion pin)."""
    return hamiltonian_strings(h, np.zeros((h.shape[0],) * 4))


def all_pairs(L):
    return list(itertools.product(range(L), repeat=2))
