"""Host-side checks run against a build of the library whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged): the
validation, layout and planning entry points on well-formed and malformed
problems.  Run by ``test_host_sanitized.py`` in a child process with the
sanitizer runtime preloaded; any sanitizer report aborts it.

    python tests/sanitized_host_checks.py <sanitized libtns.so>
"""
import dataclasses
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main(lib):
    from paper_2305_05581_amd import tns
    tns.library(lib)
    from synth import synthetic_problem
    from synth.renorm import renorm_instance
    from synth.su2 import su2_instance, su2_synthetic

    rep = lambda P, **kw: dataclasses.replace(P, **{k: np.array(v) for k, v in kw.items()})
    checks = 0
    for P in (synthetic_problem(10, 10, 0, 24, 3, 8, 10, seed=7),
              synthetic_problem(22, 22, 0, 700, 23, 187, 120, seed=12, share=6)):
        assert tns.tasklist_workspace_bytes(P) > 0
        # malformed tables: rejected without touching memory out of range
        bad = [rep(P, blk_in=np.where(np.arange(P.nBlk) == 0, P.nL + 5, P.blk_in)),
               rep(P, blk_off=np.where(np.arange(P.nBlk) == 0, len(P.op_vals), P.blk_off)),
               rep(P, term_L=np.where(np.arange(P.nTerms) == 0, P.nOps, P.term_L)),
               rep(P, psi_off=np.where(np.arange(P.nS + 1) == P.nS, P.psi_off[-1] + 1, P.psi_off)),
               rep(P, term_ma=np.where(np.arange(P.nTerms) == 0, 16, P.term_ma))]
        for Q in bad:
            assert tns.tasklist_workspace_bytes(Q) == 0
        n = len(P.op_vals)
        for cap in (n, n // 4):
            try:
                tns.ttcache_sizes(P, cap)
            except tns.TnsError as e:
                assert e.code == -4  # a term's two operators larger than the cache
        try:
            tns.ttcache_sizes(P, 0)
            raise AssertionError("empty cache accepted")
        except tns.TnsError:
            pass
        checks += 1
    R = renorm_instance(6, 64, 8, 24, 20, 30, seed=3)
    assert tns.renorm_workspace_bytes(R) > 0
    keep = R.keep.copy()
    keep[0] = R.full[0] + 1
    assert tns.renorm_workspace_bytes(dataclasses.replace(R, keep=keep)) == 0
    for I in (su2_instance(2, 2, (4, 0), seed=1), su2_synthetic(5, 120, 24, 10, 60, (10, 2), seed=4, max_2S=8)):
        sl, sr, off, tasks, ptr = tns.su2_tables(I)
        assert len(sl) == I.nS and ptr[-1] == len(tasks)
        k = I.op_2k.copy()
        k[int(I.term_L[2])] += 2
        assert tns.su2_workspace_bytes(dataclasses.replace(I, op_2k=k)) == 0
        checks += 1
    print("sanitized host checks passed:", checks)


if __name__ == "__main__":
    main(sys.argv[1])
