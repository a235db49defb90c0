"""Host-side validation of a problem by the library (no GPU needed): every
malformed table is rejected before anything is copied to the device, and
well-formed degenerate problems are accepted."""
import dataclasses
import os

import numpy as np
import pytest

from synth import synthetic_problem


@pytest.fixture(scope="module")
def lib_ok():
    from paper_2305_05581_amd.tns import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libtns.so not built (run __graft_entry__.build())")
    return True


@pytest.fixture(scope="module")
def base():
    return synthetic_problem(10, 10, 0, 24, 3, 8, 10, seed=7)


def _bytes(P):
    from paper_2305_05581_amd.tns import tasklist_workspace_bytes
    return tasklist_workspace_bytes(P)


def _with(P, **arrays):
    return dataclasses.replace(P, **{k: np.array(v) for k, v in arrays.items()})


def test_valid_and_degenerate_problems_accepted(lib_ok, base):
    assert _bytes(base) > 0
    empty = _with(base, term_L=np.zeros(0, np.int32), term_ma=np.zeros(0, np.int32),
                  term_mb=np.zeros(0, np.int32), term_R=np.zeros(0, np.int32), term_coef=np.zeros(0))
    assert _bytes(empty) > 0


def test_malformed_tables_rejected(lib_ok, base):
    P = base
    cases = {}
    d = P.dimL.copy(); d[0] = 40000
    cases["sector dimension above the limit"] = _with(P, dimL=d)
    d = P.dimR.copy(); d[0] = 0
    cases["empty sector dimension"] = _with(P, dimR=d)
    r = P.blk_rows.copy(); r[0] += 1
    cases["block rows differ from the output sector"] = _with(P, blk_rows=r)
    ld = P.blk_ld.copy(); ld[0] += 1
    cases["leading dimension not a multiple of 8"] = _with(P, blk_ld=ld)
    off = P.blk_off.copy(); off[-1] = len(P.op_vals)
    cases["block beyond the value array"] = _with(P, blk_off=off)
    dn = P.op_dN.copy(); dn[0] += 2
    cases["block not at its operator's shift"] = _with(P, op_dN=dn)
    po = P.psi_off.copy(); po[1] += 1
    cases["sector offsets inconsistent with the dimensions"] = _with(P, psi_off=po)
    ma = P.term_ma.copy(); ma[0] = 16
    cases["site monomial out of range"] = _with(P, term_ma=ma)
    tl = P.term_L.copy(); tl[0] = P.nOps
    cases["term operator out of range"] = _with(P, term_L=tl)
    for name, Q in cases.items():
        assert _bytes(Q) == 0, name


def _rn_bytes(R):
    from paper_2305_05581_amd.tns import renorm_workspace_bytes
    return renorm_workspace_bytes(R)


def test_renorm_validation(lib_ok):
    """Renormalisation steps: a well-formed step is accepted; a missing
    enlarged sector, a new operator whose terms change the quantum numbers
    differently, a block of the wrong shape and kept dimensions beyond the
    full ones are rejected on the host."""
    from synth.renorm import renorm_instance
    R = renorm_instance(6, 64, 8, 24, 20, 30, seed=3)
    assert _rn_bytes(R) > 0
    assert _rn_bytes(dataclasses.replace(R, qQ=R.qQ[1:], keep=R.keep[1:], u_off=R.u_off[1:], full=R.full[1:])) == 0
    # second term of new operator 0: its operator with a monomial of another shift
    from synth.problem import MONO_SHIFT
    m2 = next(m for m in range(16) if MONO_SHIFT[m] != MONO_SHIFT[int(R.term_mono[0])])
    bad = dataclasses.replace(R, term_new=np.concatenate([R.term_new, [0]]),
                              term_op=np.concatenate([R.term_op, [R.term_op[0]]]),
                              term_mono=np.concatenate([R.term_mono, [m2]]),
                              term_coef=np.concatenate([R.term_coef, [1.0]]))
    assert _rn_bytes(bad) == 0
    rows = R.blk_rows.copy()
    rows[0] += 1
    assert _rn_bytes(dataclasses.replace(R, blk_rows=rows)) == 0
    keep = R.keep.copy()
    keep[0] = R.full[0] + 1
    assert _rn_bytes(dataclasses.replace(R, keep=keep)) == 0


def test_ttcache_plan_sizes(lib_ok, base):
    """Tree-traversal cache plans (host only): a cache holding everything runs
    one product, the smallest one holding the two operators of any term runs
    several, and a cache below that size, an empty cache or a malformed
    problem are rejected."""
    from paper_2305_05581_amd.tns import ttcache_sizes, TnsError
    P = synthetic_problem(16, 16, 0, 96, 8, 24, 60, seed=5)
    lo = np.full(P.nOps, np.iinfo(np.int64).max)
    hi = np.full(P.nOps, -1)
    for b in range(P.nBlk):
        o = int(P.blk_op[b])
        lo[o] = min(lo[o], int(P.blk_off[b]))
        hi[o] = max(hi[o], int(P.blk_off[b]) + int(P.blk_rows[b]) * int(P.blk_ld[b]))
    fp = np.where(hi >= 0, (hi - lo + 7) // 8 * 8, 0)
    pair = max((int(fp[a]) if a >= 0 else 0) + (int(fp[b]) if b >= 0 else 0) for a, b in zip(P.term_L, P.term_R))
    hb, db, e_all = ttcache_sizes(P, int(fp.sum()))
    assert hb > 0 and db > 0 and e_all == 1  # everything fits: one product
    _, _, e_pair = ttcache_sizes(P, pair)
    # the smallest cache holds one term's operators: at least the copies of the
    # largest operators' terms run apart
    assert e_pair > 1
    for cap in (pair - 8, 0):
        with pytest.raises(TnsError):
            ttcache_sizes(P, cap)
    # buffering: a cache of a quarter of the operators double-buffered splits
    # into at least as many epochs as single-buffered; everything-fits stays one
    # product either way; an unknown mode is rejected
    quarter = max(pair, int(fp.sum()) // 4)
    _, _, e1 = ttcache_sizes(P, quarter, "single")
    _, _, e2 = ttcache_sizes(P, quarter, "double")
    assert e1 > 1 and e2 >= e1
    assert ttcache_sizes(P, int(fp.sum()), "double")[2] == 1
    import paper_2305_05581_amd.tns as T
    T.TT_MODES["bad"] = 7
    try:
        with pytest.raises(TnsError):
            ttcache_sizes(P, quarter, "bad")
    finally:
        del T.TT_MODES["bad"]
    tl = P.term_L.copy()
    tl[0] = P.nOps
    with pytest.raises(TnsError):
        ttcache_sizes(_with(P, term_L=tl), int(fp.sum()))


@pytest.mark.parametrize("seed,gapped", [(7, False), (11, True), (23, False)])
def test_host_task_count_matches_oracle(lib_ok, seed, gapped):
    """The library's host task count (which sizes the build workspace and
    which the device enumeration must reproduce) equals the length of the
    oracle's task table of Eq. (2)."""
    from paper_2305_05581_amd.tns import count_tasks
    from oracle import heff as oheff
    P = synthetic_problem(12, 12, 0, 48, 4, 12, 40, seed=seed, gapped=gapped)
    tasks, _ = oheff.task_table(P)
    assert len(tasks) > 0
    assert count_tasks(P) == len(tasks)


def test_host_task_count_degenerate_and_rejected(lib_ok, base):
    from paper_2305_05581_amd.tns import TnsError, count_tasks
    empty = _with(base, term_L=np.zeros(0, np.int32), term_ma=np.zeros(0, np.int32),
                  term_mb=np.zeros(0, np.int32), term_R=np.zeros(0, np.int32), term_coef=np.zeros(0))
    assert count_tasks(empty) == 0
    bad = _with(base, term_ma=np.full_like(np.asarray(base.term_ma), 16))
    with pytest.raises(TnsError):
        count_tasks(bad)
