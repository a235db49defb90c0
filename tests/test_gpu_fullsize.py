"""Parity at full size in the launch configuration bench.py times: the
benchmark workload (L=54, D=4096, 3000 terms + gapped terms, 36 GB of FP64
operators) and the L=30, D=1024 workload, whole task tables and whole sigma
against the oracle; the backward and the batched product at full size."""
import os
import time

import numpy as np
import pytest
import torch

from synth import synthetic_problem, gaussian_psi
from oracle import heff as oheff

from gpu_common import say, to_dev, SIGMA_TOL as TOL

pytestmark = pytest.mark.gpu


def _upload(P):
    vals = torch.empty(len(P.op_vals), dtype=torch.float64, device="cuda")
    for i in range(0, len(P.op_vals), 1 << 28):
        vals[i:i + (1 << 28)].copy_(torch.from_numpy(P.op_vals[i:i + (1 << 28)]))
    return vals


def _whole_parity(P, H, psi_seed, bars):
    """Whole task table byte for byte against the oracle's canonical table,
    then all of sigma in every precision against the oracle's FP64 sigma
    (relative Frobenius error over the whole vector and the largest
    per-sector relative error)."""
    say("oracle task table")
    ref_tab, ref_ptr = oheff.task_table(P)
    tasks, ptr = H.tasks()
    say("tasks device %d oracle %d" % (len(tasks), len(ref_tab)))
    assert len(tasks) == len(ref_tab) == H.ntasks
    assert tasks.tobytes() == ref_tab.tobytes()
    assert np.array_equal(ptr, ref_ptr)
    psi = gaussian_psi(P, psi_seed)
    t = time.time()
    ref, nthr = oheff.sigma_threaded(P, psi, [tuple(x) for x in ref_tab.tolist()])
    say("oracle sigma: %.1f s on %d threads" % (time.time() - t, nthr))
    nref = np.linalg.norm(ref)
    for prec in ("f64", "f32", "bf16x3"):
        dt = torch.float64 if prec == "f64" else torch.float32
        out = H.apply(to_dev(psi, dt), prec).double().cpu().numpy()
        err = float(np.linalg.norm(out - ref) / nref)
        worst = 0.0
        for s in range(P.nS):
            a, b = P.psi_off[s], P.psi_off[s + 1]
            nb = np.linalg.norm(ref[a:b])
            if nb > 0:
                worst = max(worst, float(np.linalg.norm(out[a:b] - ref[a:b]) / nb))
        say("  %s whole-sigma rel err %.3e, worst sector %.3e" % (prec, err, worst))
        assert err <= bars[prec], (prec, err)


@pytest.mark.timeout(900)
def test_cfg3_whole_parity():
    """The benchmark workload (L=54, D=4096, 3000 terms + gapped terms, seed
    3): all 356 k task records and all of sigma against the oracle."""
    from paper_2305_05581_amd.tns import HeffProblem
    import bench
    cfg = bench.CONFIGS["d4096"]
    say("generating the D=4096 instance")
    P = synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                          seed=cfg["seed"], gapped=cfg["gapped"], threads=min(16, os.cpu_count() or 1))
    say("uploading %.1f GB" % (P.op_vals.nbytes / 1e9))
    H = HeffProblem(P, vals64=_upload(P))
    say("tasks", H.ntasks, "flops", H.total_flops)
    _whole_parity(P, H, 3, TOL)


@pytest.mark.timeout(600)
def test_cfg2_whole_parity():
    """Plain FP64 workload at L=30, D=1024 (mean sector 32, max 256), 900
    random terms, seed 2, no gapped terms: all task records and all of sigma
    in every precision against the oracle."""
    from paper_2305_05581_amd.tns import HeffProblem
    import bench
    cfg = bench.CONFIGS["d1024"]
    say("generating the D=1024 instance, seed %d" % cfg["seed"])
    P = synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                          seed=cfg["seed"], gapped=cfg["gapped"], threads=min(16, os.cpu_count() or 1))
    H = HeffProblem(P)
    say("tasks", H.ntasks, "flops", H.total_flops)
    _whole_parity(P, H, 2, TOL)


def _block_view(P, vals, b):
    o, r, c, ld = int(P.blk_off[b]), int(P.blk_rows[b]), int(P.blk_cols[b]), int(P.blk_ld[b])
    return vals[o:o + r * ld].reshape(r, ld)[:, :c]


@pytest.mark.timeout(600)
def test_grad1024_sampled_backward():
    """Backward at the size of bench.py's grad1024 (L=30, D=1024, 900 terms,
    seed 5) in FP64 and FP32: d psi of sampled input sectors (the oracle runs
    every task with that input sector) and the gradients of sampled operator
    blocks (every task that uses the block)."""
    from paper_2305_05581_amd.tns import HeffProblem
    from oracle import grad as ograd
    import bench
    cfg = bench.CONFIGS["d1024"]
    say("generating the D=1024 instance")
    P = synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                          seed=5, threads=min(16, os.cpu_count() or 1))
    H = HeffProblem(P)
    dev_tab, _ = H.tasks()
    tasks, _ = oheff.task_table(P)
    say("tasks", H.ntasks)
    assert dev_tab.tobytes() == tasks.tobytes()  # the oracle's records drive the reference below
    rng = np.random.default_rng(7)
    cost_in = np.bincount(tasks["in"], weights=tasks["cost"].astype(np.float64), minlength=P.nS)
    pick_s = {int(np.argmax(cost_in))} | set(int(s) for s in rng.choice(np.nonzero(cost_in > 0)[0], 3, replace=False))
    pick_b = set()
    for side in ("lblk", "rblk"):
        used = tasks[side][tasks[side] >= 0]
        counts = np.bincount(used)
        pick_b |= {int(np.argmax(counts))} | set(int(b) for b in rng.choice(np.unique(used), 2, replace=False))
    sel = np.isin(tasks["in"], list(pick_s)) | np.isin(tasks["lblk"], list(pick_b)) | np.isin(tasks["rblk"], list(pick_b))
    sub = [tuple(t) for t in tasks[sel].tolist()]
    say("sampled sectors", sorted(pick_s), "blocks", sorted(pick_b), "oracle tasks", len(sub))
    psi, G = gaussian_psi(P, 5), gaussian_psi(P, 6)
    ref_dpsi, ref_dvals, _ = ograd.backward(P, psi, G, sub)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        dt = torch.float64 if prec == "f64" else torch.float32
        x, g = to_dev(psi, dt), to_dev(G, dt)
        gp, go = H.backward(x, g, prec)
        gp, go = gp.double().cpu().numpy(), go.double().cpu().numpy()
        a = np.concatenate([gp[P.psi_off[s]:P.psi_off[s + 1]] for s in sorted(pick_s)])
        b = np.concatenate([ref_dpsi[P.psi_off[s]:P.psi_off[s + 1]] for s in sorted(pick_s)])
        e1 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        a = np.concatenate([_block_view(P, go, k).reshape(-1) for k in sorted(pick_b)])
        b = np.concatenate([_block_view(P, ref_dvals, k).reshape(-1) for k in sorted(pick_b)])
        e2 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        say("  %s sampled rel err d psi %.3e, d blocks %.3e" % (prec, e1, e2))
        assert e1 <= tol and e2 <= tol


@pytest.mark.timeout(600)
def test_batch64_generator_sampled_parity():
    """The batched product (one launch per phase for all instances) on the
    first 12 instances of bench.py's batch64 generator (L 20..40, D 256..2048
    log-uniform, K = L^2): FP64 on two output sectors per instance (its
    largest and a seeded random one) against the oracle, FP32 and BF16x3 over
    all of sigma against that FP64 product."""
    from paper_2305_05581_amd.tns import HeffProblem, HeffBatch
    import bench
    rng = np.random.default_rng(11)
    Ps, Hs, picks = [], [], []
    for i, c in enumerate(bench.batch_specs(64)[:12]):
        P = synthetic_problem(c["L"], c["N"], c["twoSz"], c["D"], c["mean"], c["dmax"], c["K"], seed=c["seed"],
                              threads=min(16, os.cpu_count() or 1))
        H = HeffProblem(P)
        tasks, ptr = H.tasks()
        cost = np.array([tasks["cost"][ptr[s]:ptr[s + 1]].sum() for s in range(P.nS)])
        pick = sorted({int(np.argmax(cost)), int(rng.choice(np.nonzero(cost > 0)[0]))})
        say("instance %d: L=%d D=%d tasks %d, sectors %s" % (i, c["L"], c["D"], H.ntasks, pick))
        Ps.append(P)
        Hs.append(H)
        picks.append(pick)
    B = HeffBatch(Hs)
    xs = [gaussian_psi(P, 60 + i) for i, P in enumerate(Ps)]
    ref64 = B.apply([to_dev(x) for x in xs], "f64")
    for i, (P, x, y, pick) in enumerate(zip(Ps, xs, ref64, picks)):
        ref = oheff.sigma_sectors(P, x, pick)
        got = y.cpu().numpy()
        a = np.concatenate([got[P.psi_off[s]:P.psi_off[s + 1]] for s in pick])
        b = np.concatenate([ref[s].reshape(-1) for s in pick])
        err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        say("  f64 instance %d sampled rel err %.2e" % (i, err))
        assert err <= 1e-12
    # the FP64 product is pinned to the oracle above; the reduced precisions
    # are held to their bars over the whole of sigma against it
    for prec, tol in (("f32", TOL["f32"]), ("bf16x3", TOL["bf16x3"])):
        outs = B.apply([to_dev(x, torch.float32) for x in xs], prec)
        for i, (y, r) in enumerate(zip(outs, ref64)):
            err = float(torch.linalg.norm(y.double() - r) / torch.linalg.norm(r))
            say("  %s instance %d whole-sigma rel err against FP64 %.2e" % (prec, i, err))
            assert err <= tol, (prec, i, err)
