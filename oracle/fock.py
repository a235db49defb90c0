"""Fock space, Jordan-Wigner strings and the brute-force FCI Hamiltonian.

Section III, Eq. (1): the long-range Hamiltonian with one-particle hopping and
two-particle scattering terms over modes with an internal (spin) label.  Read
here in the spin-free chemists' form with real orbitals

    H = sum_{ij,s} h_ij c+_is c_js + 1/2 sum_{ijkl,s,t} (ij|kl) c+_is c+_kt c_lt c_js

Modes are ``p = 2 i + s`` (orbital ``i``, spin ``s`` = 0 up, 1 down).  A
determinant is a bit string with bit ``p`` set when mode ``p`` is occupied,
and ``c+_p |n>`` carries the sign ``(-1)^(number of occupied modes q < p)``.

FCI (the exact limit for small active spaces, results section) is the
Hamiltonian matrix over all determinants with the target (N, 2Sz).
"""

import itertools

import numpy as np
import scipy.sparse as sp


def mode(i, s):
    return 2 * i + s


def apply_string(string, det):
    """Apply a product of ladder operators to one determinant.

    ``string`` lists ``(mode, is_creator)`` from left to right; the rightmost
    factor acts first.  Returns ``(sign, new_det)`` or ``(0, None)``.
    """
    sign = 1
    for p, dag in reversed(string):
        occ = (det >> p) & 1
        if occ == dag:
            return 0, None
        if bin(det & ((1 << p) - 1)).count("1") & 1:
            sign = -sign
        det ^= (1 << p)
    return sign, det


def apply_string_vec(string, dets):
    """Vectorised :func:`apply_string` over an int64 array of determinants.
    Returns ``(sign[int64], new_dets, valid[bool])``."""
    d = dets.copy()
    sign = np.ones(len(d), dtype=np.int64)
    valid = np.ones(len(d), dtype=bool)
    for p, dag in reversed(string):
        occ = (d >> p) & 1
        valid &= (occ != dag)
        par = np.bitwise_count(d & ((1 << p) - 1)) & 1
        sign = np.where(par == 1, -sign, sign)
        d = d ^ (1 << p)
    return sign, d, valid


def determinants(L, N, twoSz):
    """All 2L-mode determinants with N electrons and 2Sz = N_up - N_down,
    ascending by bit-string value."""
    nup = (N + twoSz) // 2
    ndn = (N - twoSz) // 2
    if nup < 0 or ndn < 0 or nup > L or ndn > L or nup + ndn != N:
        return np.zeros(0, dtype=np.int64)
    out = []
    for ups in itertools.combinations(range(L), nup):
        u = sum(1 << (2 * i) for i in ups)
        for dns in itertools.combinations(range(L), ndn):
            out.append(u | sum(1 << (2 * i + 1) for i in dns))
    return np.array(sorted(out), dtype=np.int64)


def hamiltonian_strings(h, eri, tol=0.0, labels=False):
    """Every string of Eq. (1) (spin-free reading) with its weight:
    ``(weight, [(mode, is_creator), ...])``.  One-body strings carry ``h_ij``,
    two-body strings ``(ij|kl)/2``.  Strings with zero weight are dropped.
    With ``labels`` each entry also carries ``("h", i, j)`` or
    ``("v", i, j, k, l)``."""
    L = h.shape[0]
    out = []
    for i in range(L):
        for j in range(L):
            if abs(h[i, j]) > tol:
                for s in (0, 1):
                    e = (h[i, j], [(mode(i, s), 1), (mode(j, s), 0)])
                    out.append(e + (("h", i, j),) if labels else e)
    for i, j, k, l in itertools.product(range(L), repeat=4):
        v = eri[i, j, k, l]
        if abs(v) > tol:
            for s in (0, 1):
                for t in (0, 1):
                    e = (0.5 * v, [(mode(i, s), 1), (mode(k, t), 1), (mode(l, t), 0), (mode(j, s), 0)])
                    out.append(e + (("v", i, j, k, l),) if labels else e)
    return out


def string_matrix(strings, dets):
    """Sparse matrix of ``sum_S w_S S`` over the determinant list ``dets``."""
    n = len(dets)
    rows, cols, vals = [], [], []
    for w, s in strings:
        sign, nd, valid = apply_string_vec(s, dets)
        if not valid.any():
            continue
        src = np.nonzero(valid)[0]
        tgt = np.searchsorted(dets, nd[src])
        ok = (tgt < n)
        ok[ok] &= dets[tgt[ok]] == nd[src[ok]]
        rows.append(tgt[ok])
        cols.append(src[ok])
        vals.append(w * sign[src[ok]].astype(np.float64))
    if not rows:
        return sp.csr_matrix((n, n))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def fci_hamiltonian(h, eri, N, twoSz):
    """Brute-force FCI matrix of Eq. (1) in the (N, 2Sz) sector.
    Returns ``(H (scipy CSR), dets)``."""
    L = h.shape[0]
    dets = determinants(L, N, twoSz)
    return string_matrix(hamiltonian_strings(h, eri), dets), dets


def number_strings(L):
    return [(1.0, [(mode(i, s), 1), (mode(i, s), 0)]) for i in range(L) for s in (0, 1)]


def s2_strings(L, normal_ordered=False):
    """Total spin squared, S^2 = Sz^2 + (S+S- + S-S+)/2, written as strings.

    With ``normal_ordered`` every string has its creators to the left (the
    anticommutator terms are written out), as the site-monomial reduction of
    the two-site split requires."""
    out = []
    for i in range(L):
        for j in range(L):
            for s in (0, 1):
                for t in (0, 1):
                    sg = 0.25 * (1 if s == t else -1)
                    if not normal_ordered:
                        out.append((sg, [(mode(i, s), 1), (mode(i, s), 0), (mode(j, t), 1), (mode(j, t), 0)]))
                    else:
                        if i == j and s == t:
                            out.append((sg, [(mode(i, s), 1), (mode(j, t), 0)]))
                        out.append((-sg, [(mode(i, s), 1), (mode(j, t), 1), (mode(i, s), 0), (mode(j, t), 0)]))
            for (a, b) in ((0, 1), (1, 0)):
                # S+_i S-_j (a=up) and S-_i S+_j (a=down): c+_ia c_ib c+_jb c_ja
                if not normal_ordered:
                    out.append((0.5, [(mode(i, a), 1), (mode(i, b), 0), (mode(j, b), 1), (mode(j, a), 0)]))
                else:
                    if i == j:
                        out.append((0.5, [(mode(i, a), 1), (mode(j, a), 0)]))
                    out.append((-0.5, [(mode(i, a), 1), (mode(j, b), 1), (mode(i, b), 0), (mode(j, a), 0)]))
    return out


def rdms(vec, dets, L):
    """Spin-summed reduced density matrices of a normalised FCI vector:
    ``gamma_ij = sum_s <c+_is c_js>`` and
    ``Gamma_ijkl = sum_st <c+_is c+_kt c_lt c_js>`` (chemists' index order)."""
    gamma = np.zeros((L, L))
    Gamma = np.zeros((L, L, L, L))
    for i in range(L):
        for j in range(L):
            M = string_matrix([(1.0, [(mode(i, s), 1), (mode(j, s), 0)]) for s in (0, 1)], dets)
            gamma[i, j] = vec @ (M @ vec)
    for i, j, k, l in itertools.product(range(L), repeat=4):
        M = string_matrix([(1.0, [(mode(i, s), 1), (mode(k, t), 1), (mode(l, t), 0), (mode(j, s), 0)])
                           for s in (0, 1) for t in (0, 1)], dets)
        Gamma[i, j, k, l] = vec @ (M @ vec)
    return gamma, Gamma
