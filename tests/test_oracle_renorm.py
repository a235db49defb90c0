"""Pins of the oracle's renormalisation (blocking) step.

* Without truncation and with U the permutation from the product basis
  |l, s> onto the canonical basis of the enlarged block, the renormalised
  operator of every ladder, number and pair string equals that string's
  matrix built directly on the enlarged block (brute force over its Fock
  states): signs, sector bookkeeping and component offsets all enter.
* With random orthogonal U (no truncation) renormalisation commutes with
  products: (c+_p c_p)~ = c+_p~ c_p~.
* With truncated random isometries the total particle number renormalises
  to N_Q times the identity in every sector.
"""
import itertools

import numpy as np

from oracle.blocks import BlockBasis, identify_monomial, split_string, SUB_L, SUB_A
from oracle.renorm import enlarged_sectors, full_basis_offsets, renormalize


def _terms_of(string, l, old):
    """One renormalisation term (op, monomial, coef) of an enlarged-block
    string: the old-block factors as an old-block operator, the site factors
    as a monomial, the reordering sign and the monomial's sign in coef."""
    eps, parts = split_string(string, l)
    a = identify_monomial(tuple((p - 2 * l, d) for p, d in parts[SUB_A]))
    if a is None:
        return None, None
    m, g = a
    ops = {}
    if parts[SUB_L]:
        shift, bl = old.blocks(old.local(parts[SUB_L]))
        qidx = {(int(x), int(y)): i for i, (x, y) in enumerate(old.q)}
        blocks = {}
        for i, B in bl.items():
            j = qidx[(int(old.q[i][0]) + shift[0], int(old.q[i][1]) + shift[1])]
            blocks[i] = (j, B)
        ops[0] = blocks
        return [(0, m, eps * g)], ops
    return [(-1, m, eps * g)], ops


def _permutation_isometries(old, new, l):
    qQ, comps = enlarged_sectors(old.q, old.dims)
    U = []
    for Q, cs in zip(qQ, comps):
        k = [i for i, q in enumerate(new.q) if tuple(q) == tuple(Q)][0]
        canon = {int(st): c for c, st in enumerate(new.states[k])}
        rows = []
        for (i, s, d) in cs:
            rows += [int(st) | (s << (2 * l)) for st in old.states[i]]
        M = np.zeros((len(rows), len(canon)))
        for r, st in enumerate(rows):
            M[r, canon[st]] = 1.0
        U.append(M)
    return qQ, U


def test_renormalized_strings_equal_enlarged_block_matrices():
    l = 2
    old, new = BlockBasis(0, l), BlockBasis(0, l + 1)
    qQ, U = _permutation_isometries(old, new, l)
    modes = range(2 * (l + 1))
    strings = [[(p, 1)] for p in modes] + [[(p, 0)] for p in modes] + [[(p, 1), (p, 0)] for p in modes]
    strings += [[(p, 1), (q, 0)] for p, q in itertools.product(modes, modes) if p != q]
    strings += [[(p, 1), (q, 1), (r, 0), (t, 0)] for (p, q, r, t) in [(0, 5, 4, 1), (4, 2, 5, 3), (5, 4, 1, 0)]]
    checked = 0
    for S in strings:
        terms, ops = _terms_of(S, l, old)
        want_shift, want = new.blocks(new.local(S))
        if terms is None:
            assert not want
            continue
        got = renormalize(old.q, old.dims, terms, ops, U)
        qidx = {(int(x), int(y)): i for i, (x, y) in enumerate(new.q)}
        want_map = {}
        for i, B in want.items():
            j = qidx[(int(new.q[i][0]) + want_shift[0], int(new.q[i][1]) + want_shift[1])]
            want_map[(i, j)] = B
        assert set(k for k, B in got.items() if np.any(B)) == set(want_map), S
        for k, B in want_map.items():
            assert np.array_equal(got[k], B), (S, k)
        checked += 1
    assert checked == len(strings)


def _random_isometries(old, keep_frac, seed):
    rng = np.random.default_rng(seed)
    qQ, comps = enlarged_sectors(old.q, old.dims)
    U = []
    for cs in comps:
        full = sum(d for _, _, d in cs)
        k = max(1, int(round(keep_frac * full)))
        Q, _ = np.linalg.qr(rng.standard_normal((full, full)))
        U.append(Q[:, :k])
    return qQ, comps, U


def test_rotation_commutes_with_products():
    l = 2
    old = BlockBasis(0, l)
    qQ, comps, U = _random_isometries(old, 1.0, 3)
    for p in range(2 * (l + 1)):
        t_cd, o_cd = _terms_of([(p, 1)], l, old)
        t_c, o_c = _terms_of([(p, 0)], l, old)
        t_n, o_n = _terms_of([(p, 1), (p, 0)], l, old)
        A = renormalize(old.q, old.dims, t_cd, o_cd, U)
        B = renormalize(old.q, old.dims, t_c, o_c, U)
        Nn = renormalize(old.q, old.dims, t_n, o_n, U)
        prod = {}
        for (a, b), Y in B.items():
            for (c, d), X in A.items():
                if c == b:
                    prod[(a, d)] = prod.get((a, d), 0) + X @ Y
        for k in set(prod) | set(Nn):
            assert np.allclose(prod.get(k, 0), Nn.get(k, 0), atol=1e-12), (p, k)


def test_truncated_number_operator():
    l = 2
    old = BlockBasis(0, l)
    qQ, comps, U = _random_isometries(old, 0.5, 5)
    terms, ops = [], {}
    for p in range(2 * (l + 1)):
        t, o = _terms_of([(p, 1), (p, 0)], l, old)
        k = len(ops)
        for (op, m, c) in t:
            if op >= 0:
                ops[k] = o[op]
                terms.append((k, m, c))
            else:
                terms.append((-1, m, c))
    got = renormalize(old.q, old.dims, terms, ops, U)
    for (a, b), B in got.items():
        assert a == b
        assert np.allclose(B, qQ[a][0] * np.eye(U[a].shape[1]), atol=1e-12)
    assert len(got) == sum(1 for q in qQ if q[0] > 0)
