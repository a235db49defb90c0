"""Device Davidson against FCI, the oracle and ARPACK; mixed precision
energies against FP64."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla
import torch

from synth import synthetic_problem, gaussian_psi, gapped_guess
from oracle import heff as oheff

from gpu_common import say, to_dev

pytestmark = pytest.mark.gpu


def test_cfg1_davidson_fci(cfg1):
    from paper_2305_05581_amd.tns import HeffProblem
    P, Hf = cfg1["P"], cfg1["H"]
    e_fci = sla.eigsh(Hf, k=1, which="SA", tol=1e-14)[0][0]
    H = HeffProblem(P)
    for inner in ("f64", "f32", "bf16x3"):
        say("cfg1 davidson", inner)
        e, x, info = H.davidson(to_dev(gaussian_psi(P, 1)), inner=inner, tol_res=1e-6)
        say("  E %.12f  dE %.2e  %s" % (e, e - e_fci, info))
        assert abs(e - e_fci) < 1e-8
        assert info["res_norm"] < 1e-4
        # the returned vector is normalised and reproduces the energy
        xv = x.cpu().numpy()
        assert abs(np.linalg.norm(xv) - 1) < 1e-12
        assert abs(xv @ oheff.sigma(P, xv) - e) < 1e-10


def test_gapped_davidson_mixed_vs_f64():
    from paper_2305_05581_amd.tns import HeffProblem
    P = synthetic_problem(20, 20, 0, 256, 16, 128, 400, seed=3, gapped=True)
    tasks = oheff.enumerate_tasks(P)
    op = sla.LinearOperator((P.psi_dim, P.psi_dim), matvec=lambda v: oheff.sigma(P, v, tasks), dtype=np.float64)
    e_ref = sla.eigsh(op, k=1, which="SA", tol=1e-12, v0=gapped_guess(P, 2))[0][0]
    H = HeffProblem(P)
    x0 = to_dev(gapped_guess(P, 2))
    e64, _, i64 = H.davidson(x0, inner="f64", tol_res=1e-7)
    say("f64", e64, e64 - e_ref, i64)
    assert abs(e64 - e_ref) < 1e-10
    for inner in ("f32", "bf16x3"):
        e, _, info = H.davidson(x0, inner=inner, tol_res=1e-5)
        say(inner, e, e - e64, info)
        assert abs(e - e64) < 1e-8
        assert info["matvecs_f64"] >= 1


def test_davidson_restart_small_subspace():
    from paper_2305_05581_amd.tns import HeffProblem
    P = synthetic_problem(16, 16, 0, 96, 8, 24, 60, seed=5, gapped=True)
    H = HeffProblem(P)
    x0 = to_dev(gapped_guess(P, 1))
    a, _, ia = H.davidson(x0, tol_res=1e-8, max_sub=6, keep=2)
    b, _, ib = H.davidson(x0, tol_res=1e-8)
    say("restart", a, b, ia, ib)
    assert abs(a - b) < 1e-10


def test_small_gap_mixed_acceptance():
    """Random terms without the gapped diagonal: the mixed-precision
    iteration accepts on the FP64 residual alone, so whatever the inner
    precision, a converged result has |r64| <= tol_res, its energy obeys the
    quadratic residual bound with the true gap, and at tol_res = 1e-6 it lies
    within 1e-8 of the exact lowest eigenvalue."""
    from paper_2305_05581_amd.tns import HeffProblem
    P = synthetic_problem(14, 14, 0, 64, 6, 16, 40, seed=8)
    tasks = oheff.enumerate_tasks(P)
    op = sla.LinearOperator((P.psi_dim, P.psi_dim), matvec=lambda v: oheff.sigma(P, v, tasks), dtype=np.float64)
    e1, e2 = sorted(sla.eigsh(op, k=2, which="SA", tol=1e-13)[0])
    gap = e2 - e1
    say("exact lowest pair %.12f %.12f gap %.3e" % (e1, e2, gap))
    H = HeffProblem(P)
    x0 = to_dev(gaussian_psi(P, 2))
    for inner in ("f32", "bf16x3"):
        for tol_res in (1e-6, 1e-3):
            e, _, info = H.davidson(x0, inner=inner, tol_res=tol_res, tol_e=1e-10)
            err = abs(e - e1)
            say(inner, tol_res, "dE %.2e" % err, info)
            assert info["converged"]
            assert info["res_norm"] <= tol_res * 1.0001
            assert err <= info["res_norm"] ** 2 / gap * 1.01 + 1e-12
            if tol_res <= 1e-6:
                assert err <= 1e-8


def test_checkpoint_resume(tmp_path):
    """A solve cut short, written to a checkpoint and resumed from it reaches
    the uninterrupted solve's energy in fewer products."""
    from paper_2305_05581_amd.tns import HeffProblem, save_davidson_checkpoint, load_davidson_checkpoint
    P = synthetic_problem(16, 16, 0, 96, 8, 24, 60, seed=5, gapped=True)
    H = HeffProblem(P)
    x0 = to_dev(gapped_guess(P, 1))
    e_full, _, i_full = H.davidson(x0, tol_res=1e-8)
    e_cut, x_cut, i_cut = H.davidson(x0, tol_res=1e-8, max_iter=6)
    assert not i_cut["converged"]
    path = str(tmp_path / "davidson.npz")
    save_davidson_checkpoint(path, e_cut, x_cut, i_cut)
    e_ck, x_ck, info_ck = load_davidson_checkpoint(path)
    assert e_ck == e_cut and info_ck["iters"] == i_cut["iters"]
    e_res, _, i_res = H.davidson(x_ck.to("cuda"), tol_res=1e-8)
    say("checkpoint", e_full, e_res, i_full, i_cut, i_res)
    assert i_res["converged"] and abs(e_res - e_full) < 1e-10
    assert i_res["iters"] < i_full["iters"]


def test_non_finite_operator_reported():
    """A NaN in the operator values makes the device Davidson stop with
    TNS_ERR_NUMERIC after its first iteration (every kernel runs to its end)."""
    from paper_2305_05581_amd.tns import HeffProblem, TnsError
    P = synthetic_problem(10, 10, 0, 24, 3, 8, 40, seed=77)
    vals = torch.from_numpy(P.op_vals.copy()).to("cuda")
    vals[int(P.blk_off[0])] = float("nan")
    H = HeffProblem(P, vals64=vals)
    with pytest.raises(TnsError) as e:
        H.davidson(to_dev(gaussian_psi(P, 1)), tol_res=1e-8)
    assert e.value.code == -6
