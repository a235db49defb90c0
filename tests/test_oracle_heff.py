"""Pins of the oracle's sigma = H_eff psi (Eq. 2), task table and full form."""
import numpy as np
import pytest

from synth import molecular_integrals, synthetic_problem, gaussian_psi, hubbard_integrals
from synth.problem import MONO_SHIFT
from oracle.blocks import Construction, MONO, SITE_Q
from oracle.fock import fci_hamiltonian, number_strings, s2_strings, string_matrix
from oracle import heff


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_cfg1_heff_equals_fci(cfg1):
    P, H, idx = cfg1["P"], cfg1["H"], cfg1["idx"]
    psi = gaussian_psi(P, 1)
    x = np.zeros(H.shape[0])
    x[idx] = psi
    assert P.psi_dim == 4900 and len(np.unique(idx)) == 4900
    assert rel(heff.sigma(P, psi), (H @ x)[idx]) < 1e-13


def test_naive_and_complementary_agree():
    h, eri = molecular_integrals(6, 7)
    Pn = Construction(h, eri, 6, 0, l=2, grouping="naive").problem()
    Pc = Construction(h, eri, 6, 0, l=2, grouping="complementary").problem()
    assert Pc.nTerms < Pn.nTerms
    psi = gaussian_psi(Pc, 2)
    assert rel(heff.sigma(Pn, psi), heff.sigma(Pc, psi)) < 1e-13


@pytest.mark.parametrize("l", [1, 2, 3])
def test_heff_fci_other_cuts_and_odd_sector(l):
    h, eri = molecular_integrals(6, 13)
    C = Construction(h, eri, 5, 1, l=l)
    P = C.problem()
    H, dets = fci_hamiltonian(h, eri, 5, 1)
    idx = C.fci_map(P, dets)
    psi = gaussian_psi(P, 4)
    x = np.zeros(len(dets))
    x[idx] = psi
    assert rel(heff.sigma(P, psi), (H @ x)[idx]) < 1e-13


def test_free_fermion_through_heff():
    h, _ = molecular_integrals(6, 21)
    C = Construction(h, np.zeros((6,) * 4), 6, 0, l=2)
    P = C.problem()
    D = heff.dense_heff(P)
    eps = np.linalg.eigvalsh(h)
    assert abs(np.linalg.eigvalsh(D)[0] - 2 * eps[:3].sum()) < 1e-12


def test_number_and_spin_as_terms():
    L, l = 6, 2
    Cn = Construction(np.zeros((L, L)), np.zeros((L,) * 4), 6, 0, l=l, strings=number_strings(L))
    P = Cn.problem()
    psi = gaussian_psi(P, 5)
    assert rel(heff.sigma(P, psi), 6 * psi) < 1e-14
    # S^2 of the Hubbard ground state is S(S+1) with S = 0 at half filling
    h, eri = hubbard_integrals(L, 1.0, 4.0)
    C = Construction(h, eri, 6, 0, l=l)
    Ph = C.problem()
    e, v = np.linalg.eigh(heff.dense_heff(Ph))
    Cs = Construction(np.zeros((L, L)), np.zeros((L,) * 4), 6, 0, l=l, strings=s2_strings(L, normal_ordered=True))
    Ps = Cs.problem()
    g = v[:, 0]
    assert abs(g @ heff.sigma(Ps, g) - 0.0) < 1e-10
    # the normal-ordered S^2 table equals the direct one on the FCI space
    from oracle.fock import determinants
    dets = determinants(L, 6, 0)
    assert abs(string_matrix(s2_strings(L), dets) - string_matrix(s2_strings(L, True), dets)).max() < 1e-13


def test_dense_full_form_matches_sigma():
    P = synthetic_problem(10, 10, 0, 24, 4, 8, 20, seed=31)
    x = gaussian_psi(P, 1)
    D = heff.dense_heff(P)
    assert rel(D @ x, heff.sigma(P, x)) < 1e-13


@pytest.mark.parametrize("seed", [41, 42])
def test_synthetic_hermitian(seed):
    P = synthetic_problem(12, 12, 0, 40, 5, 12, 30, seed=seed)
    x, y = gaussian_psi(P, 1), gaussian_psi(P, 2)
    Hx, Hy = heff.sigma(P, x), heff.sigma(P, y)
    assert abs(x @ Hy - Hx @ y) < 1e-13 * np.linalg.norm(x) * np.linalg.norm(Hy)


def test_gapped_variant_hermitian():
    P = synthetic_problem(12, 12, 0, 40, 5, 12, 30, seed=5, gapped=True)
    x, y = gaussian_psi(P, 1), gaussian_psi(P, 2)
    assert abs(x @ heff.sigma(P, y) - heff.sigma(P, x) @ y) < 1e-13


def test_quantum_numbers_conserved(cfg1):
    for P in (cfg1["P"], synthetic_problem(12, 12, 0, 40, 5, 12, 30, seed=3)):
        tasks, ptr = heff.task_table(P)
        for t in tasks:
            iL, sa, sb, iR = P.psi_sec[t["in"]]
            jL, ta, tb, jR = P.psi_sec[t["out"]]
            k = t["term"]
            dq = np.zeros(2, dtype=int)
            for op in (P.term_L[k], P.term_R[k]):
                if op >= 0:
                    dq += (P.op_dN[op], P.op_d2Sz[op])
            dq += MONO_SHIFT[P.term_ma[k]]
            dq += MONO_SHIFT[P.term_mb[k]]
            qin = P.qL[iL] + SITE_Q[sa] + SITE_Q[sb] + P.qR[iR]
            qout = P.qL[jL] + SITE_Q[ta] + SITE_Q[tb] + P.qR[jR]
            assert tuple(qin + dq) == tuple(qout) == tuple(P.target)
            if t["lblk"] >= 0:
                assert P.blk_in[t["lblk"]] == iL and P.blk_out[t["lblk"]] == jL
            if t["rblk"] >= 0:
                assert P.blk_in[t["rblk"]] == iR and P.blk_out[t["rblk"]] == jR
        # every block sits at its operator's shift
        for b in range(P.nBlk):
            o = P.blk_op[b]
            q = P.qL if P.op_side[o] == 0 else P.qR
            assert tuple(q[P.blk_out[b]] - q[P.blk_in[b]]) == (P.op_dN[o], P.op_d2Sz[o])


def test_task_table_brute_force():
    """Second enumeration: loop over (output, input) sector pairs and terms,
    test the block table directly, and compare records byte for byte."""
    P = synthetic_problem(10, 10, 0, 24, 3, 8, 40, seed=77)
    tasks, ptr = heff.task_table(P)
    rec = []
    for s2 in range(P.nS):
        jL, ta, tb, jR = (int(v) for v in P.psi_sec[s2])
        for k in range(P.nTerms):
            for s in range(P.nS):
                iL, sa, sb, iR = (int(v) for v in P.psi_sec[s])
                oL, oR = int(P.term_L[k]), int(P.term_R[k])
                lb = rb = -1
                if oL >= 0:
                    hit = [b for b in range(P.nBlk) if P.blk_op[b] == oL and P.blk_in[b] == iL and P.blk_out[b] == jL]
                    if not hit:
                        continue
                    lb = hit[0]
                elif iL != jL:
                    continue
                if oR >= 0:
                    hit = [b for b in range(P.nBlk) if P.blk_op[b] == oR and P.blk_in[b] == iR and P.blk_out[b] == jR]
                    if not hit:
                        continue
                    rb = hit[0]
                elif iR != jR:
                    continue
                va = MONO[P.term_ma[k]][ta, sa]
                vb = MONO[P.term_mb[k]][tb, sb]
                if va == 0 or vb == 0:
                    continue
                # sign: count ladder factors moved across occupied input modes
                pa = abs(MONO_SHIFT[P.term_ma[k]][0]) % 2
                pb = abs(MONO_SHIFT[P.term_mb[k]][0]) % 2
                pR = abs(int(P.op_dN[oR])) % 2 if oR >= 0 else 0
                Nl = int(P.qL[iL][0])
                Na, Nb = int(SITE_Q[sa][0]), int(SITE_Q[sb][0])
                sgn = (-1.0) ** (pa * Nl + pb * (Nl + Na) + pR * (Nl + Na + Nb))
                alpha = ((float(P.term_coef[k]) * va) * vb) * sgn
                q, m, n, r = int(P.dimL[jL]), int(P.dimL[iL]), int(P.dimR[iR]), int(P.dimR[jR])
                cost, order = heff.task_cost(q, m, n, r, oL >= 0, oR >= 0)
                rec.append((s2, s, k, lb, rb, order, alpha, cost))
    brute = np.array(rec, dtype=heff.TASK_DTYPE)
    assert len(brute) == len(tasks) > 100
    assert brute.tobytes() == tasks.tobytes()
    assert ptr[-1] == len(tasks) and np.all(np.diff(ptr) >= 0)


def test_task_cost_rule():
    # square sectors tie -> order 0; a small left input makes L (psi R^T) cheaper
    assert heff.task_cost(8, 8, 8, 8, True, True) == (2 * 8 * 8 * 16, 0)
    c, o = heff.task_cost(64, 8, 64, 64, True, True)
    assert o == 1 and c == 2 * 8 * 64 * (64 + 64)
    c, o = heff.task_cost(64, 64, 8, 64, True, True)
    assert o == 0 and c == 2 * 64 * 8 * (64 + 64)
    assert heff.task_cost(5, 5, 7, 3, False, True) == (2 * 5 * 7 * 3, 0)
    assert heff.task_cost(5, 4, 7, 7, True, False) == (2 * 5 * 4 * 7, 0)
    assert heff.task_cost(5, 5, 7, 7, False, False) == (2 * 5 * 7, 0)


def test_order_flag_does_not_change_sigma():
    P = synthetic_problem(12, 12, 0, 40, 5, 12, 30, seed=9)
    x = gaussian_psi(P, 1)
    tasks = heff.enumerate_tasks(P)
    flipped = [t[:5] + (1 - t[5],) + t[6:] if (t[3] >= 0 and t[4] >= 0) else t for t in tasks]
    assert rel(heff.sigma(P, x, tasks), heff.sigma(P, x, flipped)) < 1e-13


def _sectors_instances(cfg1):
    h, eri = molecular_integrals(6, 13)
    return [("exact cfg1", cfg1["P"]),
            ("exact odd 2Sz", Construction(h, eri, 5, 1, l=2).problem()),
            ("ragged synthetic", synthetic_problem(14, 14, 0, 70, 6, 23, 40, seed=17)),
            ("gapped synthetic", synthetic_problem(12, 12, 0, 40, 5, 12, 30, seed=5, gapped=True))]


def test_sigma_sectors_equals_sigma(cfg1):
    """Eq. (2) restricted to a subset of output sectors: ``sigma_sectors``
    (the reference of the sampled and whole-product checks) returns exactly
    the corresponding slices of the pinned ``sigma`` on every sector, through
    both of its routes (its own filtered enumeration, and a caller's task
    list that holds other sectors too).  The instances cover identity-side
    and both-identity terms (cfg1), an odd 2Sz target, ragged sector sizes
    and the gapped diagonal terms."""
    for name, P in _sectors_instances(cfg1):
        psi = gaussian_psi(P, 9)
        full = heff.sigma(P, psi)
        every = heff.sigma_sectors(P, psi, range(P.nS))
        assert sorted(every) == list(range(P.nS)), name
        for s in range(P.nS):
            got = every[s].reshape(-1)
            want = full[P.psi_off[s]:P.psi_off[s + 1]]
            assert got.shape == want.shape and np.array_equal(got, want), (name, s)
        rng = np.random.default_rng(3)
        pick = sorted(int(s) for s in rng.choice(P.nS, min(5, P.nS), replace=False))
        all_tasks = heff.enumerate_tasks(P)
        for sub in (heff.sigma_sectors(P, psi, pick), heff.sigma_sectors(P, psi, pick, tasks=all_tasks)):
            assert sorted(sub) == pick, name
            for s in pick:
                assert np.array_equal(sub[s].reshape(-1), full[P.psi_off[s]:P.psi_off[s + 1]]), (name, s)
        # the filtered enumeration holds exactly the tasks of the picked sectors
        filt = heff.enumerate_tasks(P, out_filter=set(pick))
        assert filt == [t for t in all_tasks if t[0] in set(pick)], name
        # identity-side and both-identity tasks are present where the instance has them
        if name == "exact cfg1":
            assert any(t[3] < 0 <= t[4] for t in all_tasks) and any(t[4] < 0 <= t[3] for t in all_tasks)
            assert any(t[3] < 0 and t[4] < 0 for t in all_tasks)


def test_sigma_threaded_equals_sigma():
    """The thread-pool driver of the oracle's sigma (output sectors over
    threads, BLAS at one thread) against the pinned sequential sum of Eq. (2),
    on a ragged synthetic instance, an exact-block instance and a subset of
    output sectors."""
    from synth import molecular_integrals
    from oracle.blocks import Construction
    for P in (synthetic_problem(22, 22, 0, 700, 23, 187, 120, seed=12),
              Construction(*molecular_integrals(8, 1), 8, 0).problem()):
        psi = gaussian_psi(P, 4)
        t = heff.enumerate_tasks(P)
        ref = heff.sigma(P, psi, t)
        got, n = heff.sigma_threaded(P, psi, t, threads=3)
        assert n == 3
        assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
        part, _ = heff.sigma_threaded(P, psi, t, threads=2, sectors=[0, P.nS - 1])
        for s in range(P.nS):
            a, b = P.psi_off[s], P.psi_off[s + 1]
            if s in (0, P.nS - 1):
                assert np.allclose(part[a:b], ref[a:b], rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))
            else:
                assert not part[a:b].any()
