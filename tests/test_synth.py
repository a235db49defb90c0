"""The seeded input generator: determinism and the stated recipe."""
import numpy as np

from synth import synthetic_problem, block_profile, gaussian_psi, molecular_integrals


def test_profile_recipe():
    for (n, D, mean, dmax, seed) in ((14, 1024, 32, 256, 2), (26, 4096, 64, 512, 3), (10, 300, 17, 139, 4)):
        q, d = block_profile(n, D, mean, dmax, seed)
        assert d.sum() == D and d.max() <= dmax and d.min() >= 1
        assert len(d) == round(D / mean)
        assert [tuple(x) for x in q] == sorted(tuple(x) for x in q)
        assert np.all((q[:, 0] - q[:, 1]) % 2 == 0)


def test_deterministic_and_shapes():
    a = synthetic_problem(16, 16, 0, 96, 8, 24, 40, seed=5)
    b = synthetic_problem(16, 16, 0, 96, 8, 24, 40, seed=5)
    assert a.op_vals.tobytes() == b.op_vals.tobytes()
    assert a.check_format()
    assert a.nTerms == 40 and a.nOps == 80
    assert np.array_equal(gaussian_psi(a, 1), gaussian_psi(b, 1))
    assert abs(np.linalg.norm(gaussian_psi(a, 1)) - 1) < 1e-14
    # adjoint operators are transposes
    for o in range(0, a.nOps, 4):
        for b_ in np.nonzero(a.blk_op == o)[0]:
            i, j = a.blk_in[b_], a.blk_out[b_]
            adj = [x for x in np.nonzero(a.blk_op == o + 2)[0] if a.blk_in[x] == j and a.blk_out[x] == i]
            assert len(adj) == 1 and np.array_equal(a.block(adj[0]), a.block(b_).T)
    # alignment used by vector loads
    assert np.all(a.blk_off % 8 == 0) and np.all(a.blk_ld % 8 == 0)


def test_integrals_symmetry():
    h, eri = molecular_integrals(6, 1)
    assert np.array_equal(h, h.T)
    for p in ((1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)):
        assert np.allclose(eri, eri.transpose(p))
    M = eri.reshape(36, 36)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > -1e-12
