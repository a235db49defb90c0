"""Host logic of the spin-adapted product (no GPU): the library's sector and
task tables, contracted here task by task as Eq. (2) prescribes, against the
oracle (V^T H V psi on Fock-space instances, the reduced route on synthetic
ones with larger spins); validation of malformed problems."""
import dataclasses
import os

import numpy as np
import pytest

from synth.su2 import su2_instance, su2_synthetic
from oracle import su2 as osu


@pytest.fixture(scope="module")
def lib_ok():
    from paper_2305_05581_amd.tns import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libtns.so not built (run __graft_entry__.build())")
    return True


def _contract(I, tasks, off, secL, secR, psi):
    """sigma from a task table: sigma_out += alpha L psi_in R^T."""
    out = np.zeros(int(off[-1]))
    for t in tasks:
        a, b = int(secL[t["in"]]), int(secR[t["in"]])
        x = psi[off[t["in"]]:off[t["in"] + 1]].reshape(int(I.dimL[a]), int(I.dimR[b]))
        y = x if t["lblk"] < 0 else I.block(int(t["lblk"])) @ x
        y = y if t["rblk"] < 0 else y @ I.block(int(t["rblk"])).T
        out[off[t["out"]]:off[t["out"] + 1]] += t["alpha"] * y.reshape(-1)
    return out


FOCK = {"2x2 N=4 S=0": (2, 2, (4, 0), 1.0), "3x2 N=5 S=1/2 cut": (3, 2, (5, 1), 0.6),
        "3x2 N=4 S=1": (3, 2, (4, 2), 1.0), "2x2 N=3 S=3/2": (2, 2, (3, 3), 1.0)}


@pytest.mark.parametrize("case", list(FOCK))
def test_tables_against_oracle(lib_ok, case):
    from paper_2305_05581_amd.tns import su2_tables
    lL, lR, target, keep = FOCK[case]
    I = su2_instance(lL, lR, target, seed=21, keep_frac=keep)
    secL, secR, off, tasks, ptr = su2_tables(I)
    assert list(zip(secL.tolist(), secR.tolist())) == I.psi_sectors()
    assert np.array_equal(off, I.psi_off())
    assert np.all(np.diff(tasks["out"]) >= 0) and ptr[-1] == len(tasks)
    psi = np.random.default_rng(2).standard_normal(I.psi_dim)
    want = osu.sigma(I, psi)
    got = _contract(I, tasks, off, secL, secR, psi)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_tables_against_reduced_oracle_large_spins(lib_ok):
    from paper_2305_05581_amd.tns import su2_tables
    I = su2_synthetic(5, 120, 24, 10, 60, (10, 2), seed=4, max_2S=8)
    secL, secR, off, tasks, ptr = su2_tables(I)
    psi = np.random.default_rng(3).standard_normal(I.psi_dim)
    want = osu.sigma_reduced(I, psi)
    got = _contract(I, tasks, off, secL, secR, psi)
    assert int(I.qL[:, 1].max()) == 8
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_validation(lib_ok):
    from paper_2305_05581_amd.tns import su2_workspace_bytes
    I = su2_instance(2, 2, (4, 0), seed=22)
    assert su2_workspace_bytes(I) > 0
    rep = lambda **kw: dataclasses.replace(I, **kw)
    assert su2_workspace_bytes(rep(target=(4, 1))) == 0          # N and 2S of different parity
    assert su2_workspace_bytes(rep(target=(9, 0))) == 0          # no sector of the target
    k = I.op_2k.copy()
    k[int(I.term_L[2])] = 3                                      # rank mismatch in a term
    assert su2_workspace_bytes(rep(op_2k=k)) == 0
    b = I.blk_out.copy()
    b[0] = (b[0] + 1) % len(I.dimL)                              # block breaks N or the triangle rule
    assert su2_workspace_bytes(rep(blk_out=b)) == 0
    r = I.blk_rows.copy()
    r[0] += 1                                                    # block of the wrong shape
    assert su2_workspace_bytes(rep(blk_rows=r)) == 0
    t = I.term_R.copy()
    t[0] = 0                                                     # a left operator on the right
    assert su2_workspace_bytes(rep(term_R=t)) == 0
