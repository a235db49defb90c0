"""Benchmark: H_eff psi TFLOP/s on one MI355X at D=4096 (synthetic, FeMoco-sized).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec bf16x3|f32|f64]

Workload (synthetic stand-in for the molecular CAS(54,54) active space of the
paper, whose integrals are not available): L=54 orbitals, N=54, 2Sz=0, two
blocks of 26 orbitals with bond dimension D=4096 each, split over 64 (N, 2Sz)
sectors by a seeded Gaussian profile (mean 64, max 512), 3000 random operator
terms in adjoint pairs plus the gapped diagonal terms, seed 3.

A timed step is one application sigma = H_eff psi (persistent MFMA kernel and
the slot-sum epilogue) in the headline precision, inputs resident in HBM.
Algorithmic flops per step = sum over tasks of min(2qn(m+r), 2mr(n+q)).
Besides the timed steps the run reports every precision (same steps and
warm-up each), the device Davidson energies (FP64 and mixed, each against
the oracle's stored energy), the task-table build time, and the CPU oracle
on the whole product (thread pool over output sectors on every core this
process may use), which also checks all of sigma in every precision.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6 / 3.0}  # TFLOP/s per algorithmic flop
PREC_ID = {"f64": 0, "f32": 1, "bf16x3": 2}
# the two MFMA kernels of a product: phase A (T_k = alpha X_k M_k), phase B (sum_k T_k Y_k^T)
KERNEL = {p: ("k_fwd<%d, 0>" % i, "k_fwd<%d, 1>" % i) for p, i in PREC_ID.items()}
# sources that decide the forward kernels' memory traffic: the kernels and the
# schedule that orders their work items
KERNEL_SOURCES = ["paper_2305_05581_amd/csrc/fwd.hip", "paper_2305_05581_amd/csrc/kern.hpp",
                  "paper_2305_05581_amd/csrc/tns_internal.hpp", "paper_2305_05581_amd/csrc/tasklist.hip"]
TRAFFIC_FILE = os.path.join("profiles", "traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config, prec, phase):
    """HBM bytes per launch of one phase's kernel (0: phase A, 1: phase B)
    from the committed counter runs, if they were taken on the current kernel
    sources (else None)."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get("entries", {}).get("%s/%s/%s" % (config, prec, "AB"[phase]))
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    per = {}
    for x in rows:
        k = (int(x["Dispatch_Id"]), x["Kernel_Name"])
        per[k] = per.get(k, 0.0) + float(x["Counter_Value"])
    return per


def ingest_counters(args):
    """Per-launch HBM bytes of each phase-A kernel in two counter runs of
    `bench.py --only P --calib-bytes N`: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled by what the same counter reads for the element-wise
    calibration kernel that reads and writes N bytes."""
    if args.calib_bytes <= 0:
        sys.exit("--ingest-counters needs --calib-bytes (the size used in the counter runs)")
    fetch, write = _counter_rows(args.ingest_counters[0]), _counter_rows(args.ingest_counters[1])
    cal = [(v, k) for k, v in fetch.items() if "elementwise" in k[1]]
    if not cal:
        sys.exit("no calibration kernel in the FETCH_SIZE run")
    fv, ck = max(cal)
    f_fetch = args.calib_bytes / (fv * 1024.0)
    f_write = args.calib_bytes / (write[ck] * 1024.0)
    path = os.path.join(ROOT, TRAFFIC_FILE)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        rec = {"entries": {}}
    rec["note"] = ("HBM bytes per launch of each forward GEMM phase (key config/precision/phase): "
                   "FETCH_SIZE x f_fetch + WRITE_SIZE x f_write, f = calibration bytes / counter reading of a "
                   "plain element-wise kernel of known size")
    for prec, kernels in KERNEL.items():
        for ph, kn in enumerate(kernels):
            name = kn.replace("k_fwd", "tns::k_fwd")
            fk = [v for k, v in fetch.items() if name in k[1]]
            wk = [v for k, v in write.items() if name in k[1]]
            if not fk or not wk:
                continue
            fb = float(np.mean(fk)) * 1024 * f_fetch
            wb = float(np.mean(wk)) * 1024 * f_write
            rec["entries"].pop("%s/%s" % (args.config, prec), None)  # older phase-A-only record
            rec["entries"]["%s/%s/%s" % (args.config, prec, "AB"[ph])] = {
                "kernel": kn, "source_hash": kernel_source_hash(), "bytes_per_launch": round(fb + wb),
                "fetch_bytes": round(fb), "write_bytes": round(wb), "dispatches": len(fk),
                "f_fetch": round(f_fetch, 4), "f_write": round(f_write, 4)}
            log("%s %s: fetch %.1f GB, write %.1f GB per launch (f_fetch %.3f, f_write %.3f)"
                % (prec, kn, fb / 1e9, wb / 1e9, f_fetch, f_write))
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)


def phase_flops(P, tasks):
    """Algorithmic flops of the two phases: phase A 2 R K1 K2 per task with a
    non-identity X, phase B 2 R K2 C per task with a non-identity Y."""
    out, inn = tasks["out"], tasks["in"]
    q = P.dimL[P.psi_sec[out, 0]].astype(np.int64)
    r = P.dimR[P.psi_sec[out, 3]].astype(np.int64)
    m = P.dimL[P.psi_sec[inn, 0]].astype(np.int64)
    n = P.dimR[P.psi_sec[inn, 3]].astype(np.int64)
    o1 = tasks["order"] == 1
    R = np.where(o1, r, q)
    C = np.where(o1, q, r)
    K1 = np.where(o1, n, m)
    K2 = np.where(o1, m, n)
    idX = np.where(o1, tasks["rblk"] < 0, tasks["lblk"] < 0)
    idY = np.where(o1, tasks["lblk"] < 0, tasks["rblk"] < 0)
    fa = int(np.sum(np.where(idX, 0, 2 * R * K1 * K2)))
    fb = int(np.sum(np.where(idY, 0, 2 * R * K2 * C)))
    return fa, fb


def compulsory_bytes(P, tasks, prec):
    """HBM bytes a product cannot avoid: every operator block some task uses,
    read once, in the precision's operand format (FP64 8 B, FP32 4 B, BF16x3
    hi + lo 4 B per element), psi read and sigma written once (8 B in FP64,
    4 B otherwise) and the task table (40 B per task)."""
    used = np.unique(np.concatenate([tasks["lblk"][tasks["lblk"] >= 0], tasks["rblk"][tasks["rblk"] >= 0]]))
    elems = int(np.sum(P.blk_rows[used].astype(np.int64) * P.blk_cols[used].astype(np.int64)))
    eb = 8 if prec == "f64" else 4
    return elems * eb + 2 * P.psi_dim * eb + 40 * len(tasks)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_energy(config):
    """The FP64 oracle's Davidson energy of the workload, written by
    tests/golden/make_cfg3_energy.py (None if absent)."""
    if config != "d4096":
        return None
    try:
        with open(os.path.join(ROOT, "tests", "golden", "cfg3_oracle_energy.json")) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return None


def backward_flops(P, tasks):
    """Algorithmic flops of the backward product (d psi and the operator-block
    gradients of every task): d psi = alpha L^T G R in the cheaper order of
    the transposed task, which costs what the task itself costs (the two
    orders of L A R^T and of L^T G R are the same pair of costs); d L = alpha
    G R psi^T as (G R) psi^T, d R = alpha G^T L psi as (G^T L) psi; an
    identity side drops its product (and d of an identity is not formed)."""
    out, inn = tasks["out"], tasks["in"]
    q = P.dimL[P.psi_sec[out, 0]].astype(np.int64)
    r = P.dimR[P.psi_sec[out, 3]].astype(np.int64)
    m = P.dimL[P.psi_sec[inn, 0]].astype(np.int64)
    n = P.dimR[P.psi_sec[inn, 3]].astype(np.int64)
    iL, iR = tasks["lblk"] < 0, tasks["rblk"] < 0
    dpsi = tasks["cost"]
    dL = np.where(iL, 0, np.where(iR, 2 * q * r * m, 2 * q * r * n + 2 * q * n * m))
    dR = np.where(iR, 0, np.where(iL, 2 * r * q * n, 2 * r * q * m + 2 * r * m * n))
    return int(dpsi.sum()), int(dL.sum() + dR.sum())


CONFIGS = {
    "d4096": dict(L=54, N=54, twoSz=0, D=4096, mean=64, dmax=512, K=3000, seed=3, gapped=True),
    "d1024": dict(L=30, N=30, twoSz=0, D=1024, mean=32, dmax=256, K=900, seed=2, gapped=False),
    # exact blocks built from seeded molecular integrals (L = 10, blocks of 4
    # orbitals with all 256 states), the identity-factor-heavy molecular case
    "exact10": dict(L=10, N=10, twoSz=0, D=256, seed=21, exact=True, gapped=False),
}


def make_problem(cfg):
    """The workload of a config: a seeded synthetic instance, or exact blocks
    from seeded molecular integrals (through the oracle's construction, the
    only route to exact operator blocks)."""
    from synth import synthetic_problem, molecular_integrals
    if cfg.get("exact"):
        from oracle.blocks import Construction
        h, eri = molecular_integrals(cfg["L"], cfg["seed"])
        return Construction(h, eri, cfg["N"], cfg["twoSz"]).problem()
    return synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                             seed=cfg["seed"], gapped=cfg["gapped"], threads=min(16, os.cpu_count() or 1),
                             share=cfg.get("share", 1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_specs(n, seed=4000):
    """Instances of the batched workload: L ~ U{20..40}, D log-uniform in
    [256, 2048], sector mean sqrt(D), max 8 sqrt(D), K = L^2 terms, seed 4000+i."""
    import math
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(rng.integers(20, 41))
        D = int(round(math.exp(rng.uniform(math.log(256), math.log(2048)))))
        mean = max(1, int(round(math.sqrt(D))))
        out.append(dict(L=L, N=L, twoSz=L % 2, D=D, mean=mean, dmax=min(D, 8 * mean), K=L * L, seed=seed + i))
    return out


def bench_batch(args):
    """Many uneven products: one at a time (two launches each) against the
    batched form (one launch per phase for all instances), eager and replayed
    from a hipGraph.  Prints one JSON line."""
    import torch
    from synth import synthetic_problem, gaussian_psi
    from paper_2305_05581_amd.tns import HeffProblem, HeffBatch
    prec = args.only or "f32"
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = batch_specs(args.instances)
    Hs, flops, t0 = [], 0, time.time()
    for i, c in enumerate(specs):
        P = synthetic_problem(c["L"], c["N"], c["twoSz"], c["D"], c["mean"], c["dmax"], c["K"], seed=c["seed"],
                              threads=min(16, os.cpu_count() or 1))
        vals = torch.from_numpy(P.op_vals).to(dev)
        H = HeffProblem(P, device=dev, vals64=vals)
        H.operands(prec)
        P.op_vals = None  # the device copy is the only one needed from here on
        Hs.append(H)
        flops += H.total_flops
        log("instance %2d: L=%d D=%d sectors %d tasks %d %.2f GFLOP  (%.0f s)"
            % (i, c["L"], c["D"], P.nS, H.ntasks, H.total_flops / 1e9, time.time() - t0))
    B = HeffBatch(Hs)
    psis = [torch.from_numpy(gaussian_psi(H.P, 100 + i)).to(dev, dt) for i, H in enumerate(Hs)]
    seq_out = [torch.empty_like(x) for x in psis]
    bat_out = [torch.empty_like(x) for x in psis]

    def one_at_a_time():
        for H, x, y in zip(Hs, psis, seq_out):
            H.apply(x, prec, out=y)

    def batched():
        B.apply(psis, prec, outs=bat_out)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    tiles = Hs[0].tiles
    if args.autotune:
        t = time.time()
        tiles = B.autotune(psis, prec)
        log("autotuned tile table %08x (%.1f s)" % (tiles, time.time() - t))
    t_seq = timed(one_at_a_time, args.steps)
    log("one at a time: %.2f ms  %.2f TFLOP/s" % (t_seq * 1e3, flops / t_seq / 1e12))
    t_bat = timed(batched, args.steps)
    log("batched:       %.2f ms  %.2f TFLOP/s" % (t_bat * 1e3, flops / t_bat / 1e12))
    same = all(torch.equal(a, b) for a, b in zip(seq_out, bat_out))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batched()
    t_graph = timed(g.replay, args.steps)
    same_graph = all(torch.equal(a, b) for a, b in zip(seq_out, bat_out))
    log("batched graph: %.2f ms  %.2f TFLOP/s  (equal to one-at-a-time: %s / %s)"
        % (t_graph * 1e3, flops / t_graph / 1e12, same, same_graph))
    line = {
        "metric": "batched H_eff*psi TFLOP/s, %d uneven instances in one launch per phase" % len(Hs),
        "value": round(flops / t_graph / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_graph * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "batch64: %d instances, L ~ U{20..40}, N = L, 2Sz = L mod 2, D log-uniform "
                               "[256, 2048], sector mean sqrt(D), max 8 sqrt(D), K = L^2, seeds 4000+i"
                               % len(Hs),
                   "flops_per_step": flops, "tasks": sum(H.ntasks for H in Hs),
                   "tile_table": "%08x" % tiles, "autotuned": bool(args.autotune)},
        "one_at_a_time": {"ms_per_step": round(t_seq * 1e3, 3), "tflops": round(flops / t_seq / 1e12, 3)},
        "batched_eager": {"ms_per_step": round(t_bat * 1e3, 3), "tflops": round(flops / t_bat / 1e12, 3)},
        "batched_graph": {"ms_per_step": round(t_graph * 1e3, 3), "tflops": round(flops / t_graph / 1e12, 3)},
        "speedup_vs_one_at_a_time": round(t_seq / t_graph, 3),
        "equal_to_one_at_a_time": bool(same and same_graph),
    }
    print(json.dumps(line), flush=True)


def bench_grad(args):
    """Forward and hand-written backward (d psi and every operator-block
    gradient) of the L=30, D=1024 workload in FP32, checked against the FP64
    backward.  Prints one JSON line."""
    import torch
    from synth import synthetic_problem, gaussian_psi
    from paper_2305_05581_amd.tns import HeffProblem
    cfg = CONFIGS["d1024"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                          seed=5, threads=min(16, os.cpu_count() or 1))
    H = HeffProblem(P, device=dev)
    prec = args.only or "f32"
    psi64 = torch.from_numpy(gaussian_psi(P, 5)).to(dev)
    x = psi64.float() if prec != "f64" else psi64
    tasks, _ = H.tasks()
    fwd = H.total_flops
    f_dpsi, f_dops = backward_flops(P, tasks)
    log("grad1024: tasks %d, forward %.1f GFLOP, backward %.1f GFLOP (d psi %.1f, d operators %.1f)"
        % (H.ntasks, fwd / 1e9, (f_dpsi + f_dops) / 1e9, f_dpsi / 1e9, f_dops / 1e9))
    G = x  # loss <psi, sigma>: d loss / d sigma = psi

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    t_f = timed(lambda: H.apply(x, prec), args.steps)
    t_b = timed(lambda: H.backward(x, G, prec), args.steps)
    t_bpsi = timed(lambda: H.backward(x, G, prec, want_ops=False), args.steps)
    t_bops = timed(lambda: H.backward(x, G, prec, want_psi=False), args.steps)
    gp, go = H.backward(x, G, prec)
    gp64, go64 = H.backward(psi64, psi64, "f64")
    rel = lambda a, b: float(torch.linalg.norm(a.double() - b) / torch.linalg.norm(b))
    e_psi, e_ops = rel(gp, gp64), rel(go, go64)
    log("forward %.2f ms %.1f TFLOP/s; backward %.2f ms %.1f TFLOP/s; rel err vs FP64: d psi %.1e, d ops %.1e"
        % (t_f * 1e3, fwd / t_f / 1e12, t_b * 1e3, (f_dpsi + f_dops) / t_b / 1e12, e_psi, e_ops))
    log("one output at a time: d psi %.2f ms %.1f TFLOP/s; operator gradients %.2f ms %.1f TFLOP/s"
        % (t_bpsi * 1e3, f_dpsi / t_bpsi / 1e12, t_bops * 1e3, f_dops / t_bops / 1e12))
    bflops = f_dpsi + f_dops
    line = {
        "metric": "H_eff backward (d psi + d operator blocks) TFLOP/s", "value": round(bflops / t_b / 1e12, 3),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_b * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "grad1024: L=30 N=30 2Sz=0 D=1024 per block (mean sector 32, max 256), %d terms, "
                               "seed 5" % P.nTerms, "tasks": H.ntasks, "backward_flops": bflops,
                   "forward_flops": fwd},
        "forward": {"ms_per_step": round(t_f * 1e3, 3), "tflops": round(fwd / t_f / 1e12, 3)},
        "d_psi_only": {"ms_per_step": round(t_bpsi * 1e3, 3), "tflops": round(f_dpsi / t_bpsi / 1e12, 3)},
        "d_ops_only": {"ms_per_step": round(t_bops * 1e3, 3), "tflops": round(f_dops / t_bops / 1e12, 3)},
        "pct_mfma_peak": round(100 * bflops / t_b / 1e12 / PEAK[prec], 2),
        "rel_err_vs_f64": {"d_psi": e_psi, "d_ops": e_ops},
    }
    print(json.dumps(line), flush=True)


def bench_sbmm4s(args):
    """The paper's own execution scheme for the sum of Eq. (2), replicated
    with library GEMMs for comparison (Alg. 2, SBMM4S): per (output, input)
    sector pair with p terms, one strided batched GEMM writes A R_i^T for all
    i stacked (the interleaved output of the paper's column-major layout is
    plain stacking in row-major order), then one GEMM with the long inner
    dimension p m adds [a_1 L_1 ... a_p L_p] times that stack into the output
    sector.  The packed operands (coefficient folded into each L_i, identity
    sides materialised) are built untimed.  Timed against tns_apply_heff on
    the same workload; prints one JSON line.  Not a product path."""
    import torch
    from synth import synthetic_problem, gaussian_psi
    from paper_2305_05581_amd.tns import HeffProblem
    cfg = dict(CONFIGS["d1024"], share=8)
    prec = args.only or "f64"
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = synthetic_problem(cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"], cfg["dmax"], cfg["K"],
                          seed=cfg["seed"], gapped=cfg["gapped"], threads=min(16, os.cpu_count() or 1))
    H = HeffProblem(P, device=dev)
    tasks, _ = H.tasks()
    flops = H.total_flops
    vals = H.vals64.to(dt)
    t0 = time.time()

    def block(b, rows):
        if b < 0:
            return torch.eye(rows, dtype=dt, device=dev)
        o, r, c, ld = int(P.blk_off[b]), int(P.blk_rows[b]), int(P.blk_cols[b]), int(P.blk_ld[b])
        return vals[o:o + r * ld].view(r, ld)[:, :c]

    key = tasks["out"].astype(np.int64) * (P.nS + 1) + tasks["in"]
    order = np.argsort(key, kind="stable")
    bounds = np.flatnonzero(np.diff(key[order])) + 1
    groups = []
    for idx in np.split(order, bounds):
        s2, s = int(tasks["out"][idx[0]]), int(tasks["in"][idx[0]])
        q, m = int(P.dimL[P.psi_sec[s2, 0]]), int(P.dimL[P.psi_sec[s, 0]])
        n, r = int(P.dimR[P.psi_sec[s, 3]]), int(P.dimR[P.psi_sec[s2, 3]])
        Lp = torch.cat([float(tasks["alpha"][i]) * block(int(tasks["lblk"][i]), q) for i in idx], dim=1)
        RpT = torch.stack([block(int(tasks["rblk"][i]), r).t() for i in idx]).contiguous()  # p x n x r
        groups.append((s2, s, q, m, n, r, Lp.contiguous(), RpT))
    torch.cuda.synchronize()
    t_pack = time.time() - t0
    log("sbmm4s: %d tasks in %d (output, input) groups, packed in %.1f s" % (len(tasks), len(groups), t_pack))
    psi = torch.from_numpy(gaussian_psi(P, 3)).to(dev, dt)
    off = P.psi_off

    def sbmm4s(out):
        out.zero_()
        for (s2, s, q, m, n, r, Lp, RpT) in groups:
            A = psi[off[s]:off[s + 1]].view(m, n)
            temp = torch.matmul(A, RpT)  # strided batched: p x m x r, A shared (stride 0)
            B = out[off[s2]:off[s2 + 1]].view(q, r)
            B.addmm_(Lp, temp.view(-1, r))  # one GEMM over the stacked inner dimension p m

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    y_rep = torch.empty_like(psi)
    t_eager = timed(lambda: sbmm4s(y_rep), args.steps)
    # the replica's most favourable form: its whole call sequence replayed
    # from a HIP graph (no host launch cost); every replay checked against
    # the eager result
    y_ref = y_rep.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sbmm4s(y_rep)
    replays_equal = True

    t_rep = timed(g.replay, args.steps)
    torch.cuda.synchronize()
    replays_equal = bool(torch.equal(y_rep, y_ref))
    y_lib = torch.empty_like(psi)
    t_lib = timed(lambda: H.apply(psi, prec, out=y_lib), args.steps)
    err = float(torch.linalg.norm(y_rep - y_lib) / torch.linalg.norm(y_lib))
    log("SBMM4S replica: eager %.2f ms, graph replay %.2f ms (%.2f TFLOP/s, replays equal eager: %s); "
        "tns_apply_heff %.2f ms (%.2f TFLOP/s), %.1fx; rel diff %.2e"
        % (t_eager * 1e3, t_rep * 1e3, flops / t_rep / 1e12, replays_equal, t_lib * 1e3, flops / t_lib / 1e12,
           t_rep / t_lib, err))
    line = {
        "metric": "H_eff*psi TFLOP/s, SBMM4S library-GEMM replica vs the fused kernels", "unit": "TFLOP/s",
        "value": round(flops / t_lib / 1e12, 3), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_lib * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "d1024: L=30 N=30 2Sz=0 D=1024 per block (mean sector 32, max 256), %d terms, seed 2"
                               % P.nTerms, "tasks": int(len(tasks)), "groups": len(groups), "flops_per_step": flops},
        "sbmm4s": {"ms_per_step": round(t_rep * 1e3, 3), "tflops": round(flops / t_rep / 1e12, 3),
                   "eager_ms_per_step": round(t_eager * 1e3, 3), "graph_replays_equal_eager": replays_equal,
                   "library_calls_per_step": 2 * len(groups), "pack_seconds": round(t_pack, 1)},
        "fused_speedup": round(t_rep / t_lib, 2), "rel_diff": err,
    }
    print(json.dumps(line), flush=True)


def bench_renorm(args):
    """Renormalisation (blocking) step (tns_renormalize): a D = 1024 block
    (14 orbitals, mean sector 32, max 256) with 200 random block-sparse
    operators, its enlarged block (4096 states) truncated back to a quarter
    by random isometries, and 400 new operators (one or two terms each,
    every eighth a lifted site monomial).  Every precision timed over the same
    steps; FP64 checked against the oracle on sampled new operators.  Prints
    one JSON line."""
    import torch
    from synth.renorm import renorm_instance
    from oracle import renorm as orn
    from paper_2305_05581_amd.tns import RenormStep, KernelTimer
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    R = renorm_instance(14, 1024, 32, 256, 200, 400, seed=9, keep_frac=0.25)
    t_gen = time.time() - t0
    t0 = time.time()
    S = RenormStep(R, device=dev)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    flops = S.total_flops
    log("renorm: %d tasks, %d output blocks, %.1f GFLOP per step, build %.2f s (generate %.1f s)"
        % (S.ntasks, S.n_out_blk, flops / 1e9, t_build, t_gen))
    ops = torch.from_numpy(R.op_vals).to(dev)
    u = torch.from_numpy(R.u_vals).to(dev)
    res, outs = {}, {}
    order = [p for p in ("f64", "f32", "bf16x3") if p != args.prec] + [args.prec]
    for prec in order:
        out = S.apply(ops, u, prec)
        for _ in range(args.warmup):
            S.apply(ops, u, prec, out=out)
        kt = KernelTimer(args.steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            kt.arm()
            S.apply(ops, u, prec, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / args.steps
        ka, kb = np.array(kt.times_ms()).mean(axis=0)
        kt.close()
        outs[prec] = out.double()
        res[prec] = dict(ms_per_step=wall * 1e3, tflops=flops / wall / 1e12,
                         pct_peak=100 * flops / wall / 1e12 / PEAK[prec], phaseA_ms=float(ka), phaseB_ms=float(kb),
                         kernel_tflops=flops / ((ka + kb) / 1e3) / 1e12)
        log("%-6s %8.3f ms/step %7.2f TFLOP/s (%.1f%% of peak; phase A %.3f ms, phase B %.3f ms)"
            % (prec, wall * 1e3, res[prec]["tflops"], res[prec]["pct_peak"], ka, kb))
    ref = outs["f64"]
    for prec in ("f32", "bf16x3"):
        res[prec]["rel_err_vs_f64"] = float(torch.linalg.norm(outs[prec] - ref) / torch.linalg.norm(ref))
    # the oracle on sampled new operators (dense U^T O' U by definition)
    tab = S.out_table()
    got = ref.cpu().numpy()
    opb = {o: R.op_blocks(o) for o in range(len(R.op_dN))}
    U = R.isometries()
    rng = np.random.default_rng(1)
    pick = sorted(int(x) for x in rng.choice(R.n_new, 3, replace=False))
    num = den = 0.0
    t = time.perf_counter()
    for nu in pick:
        want = orn.renormalize(R.qL, R.dimL, R.terms_of(nu), opb, U)
        for k in np.nonzero(tab["new"] == nu)[0]:
            o, r, c, ld = int(tab["off"][k]), int(tab["rows"][k]), int(tab["cols"][k]), int(tab["ld"][k])
            B = got[o:o + r * ld].reshape(r, ld)[:, :c]
            W = want.get((int(tab["q_in"][k]), int(tab["q_out"][k])), np.zeros_like(B))
            num += float(np.sum((B - W) ** 2))
            den += float(np.sum(W ** 2))
    t_or = time.perf_counter() - t
    parity = float(np.sqrt(num / den)) if den > 0 else None
    log("oracle check on new operators %s: FP64 rel err %.2e (%.1f s)" % (pick, parity, t_or))
    head = res[args.prec]
    dom_ms = max(head["phaseA_ms"], head["phaseB_ms"])
    line = {
        "metric": "renormalisation step TFLOP/s (% MFMA peak)", "value": round(head["tflops"], 3),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "renorm: block of 14 orbitals, D=1024 (mean sector 32, max 256), 200 operators, "
                               "enlarged block 4096 states truncated to %d, 400 new operators, seed 9"
                               % int(R.keep.sum()),
                   "tasks": S.ntasks, "output_blocks": S.n_out_blk, "flops_per_step": flops},
        "precisions": {k: {kk: float("%.4g" % vv) for kk, vv in v.items()} for k, v in res.items()},
        "oracle_parity_f64": {"new_operators": pick, "rel_frobenius": parity},
        "roofline": {"bound": "mfma", "achieved_both_phases": round(head["kernel_tflops"], 3),
                     "peak": round(PEAK[args.prec], 1), "unit": "TFLOP/s",
                     "frac": round(head["kernel_tflops"] / PEAK[args.prec], 4), "dominant_phase_ms": round(dom_ms, 3)},
    }
    print(json.dumps(line), flush=True)


def bench_ttcache(args):
    """Out-of-HBM products (tree-traversal cache): the D = 1024 workload
    (L=30, 900 terms, seed 2; each operator pair serving up to 8 terms with
    different site monomials) with its operator values in pinned host memory,
    streamed through device caches of 1/8 and 1/2 of their size and of all of
    it, against the in-HBM product, each single- and double-buffered (epochs
    alternating between the cache's halves, each epoch's copies overlapping
    the previous epoch's product); the top-level figures of a cache are those
    of the plan's own choice (auto).  Reports the elements copied per product
    against a per-term load of both operators, the copy rate against a plain
    pinned host-to-device copy, and sigma against the in-HBM product and the
    oracle (FP64).  Prints one JSON line."""
    import torch
    from synth import gaussian_psi
    from oracle import heff as oheff
    from paper_2305_05581_amd.tns import HeffProblem, StreamedHeff
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = dict(CONFIGS["d1024"], share=8)
    prec = args.only or "f64"
    dt = torch.float64 if prec == "f64" else torch.float32
    es = 8 if prec == "f64" else 4
    P = make_problem(cfg)
    H = HeffProblem(P, device=dev)
    psi = gaussian_psi(P, 3)
    x = torch.from_numpy(psi).to(dev, dtype=dt)
    flops = H.total_flops

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    ref = H.apply(x, prec)
    t_hbm = timed(lambda: H.apply(x, prec, out=ref), args.steps)
    host = torch.from_numpy(np.ascontiguousarray(P.op_vals)).to(dt).pin_memory()
    # plain pinned copy of all operator values: the link's rate
    dst = torch.empty(host.numel(), dtype=dt, device=dev)
    t_copy = timed(lambda: dst.copy_(host, non_blocking=True), 3)
    link = host.numel() * es / t_copy / 1e9
    del dst
    log("ttcache: %d tasks, %.1f GFLOP, operators %.2f GB (%s); in-HBM product %.2f ms; pinned copy %.1f GB/s"
        % (H.ntasks, flops / 1e9, host.numel() * es / 1e9, prec, t_hbm * 1e3, link))
    t0 = time.perf_counter()
    want, thr = oheff.sigma_threaded(P, psi)
    t_or = time.perf_counter() - t0
    ref64 = ref.double().cpu().numpy()
    caches = {}
    for name, frac in (("eighth", 8), ("half", 2), ("all", 1)):
        n = (host.numel() + frac - 1) // frac
        rec = {}
        for mode in ("single", "double", "auto"):
            S = StreamedHeff(P, n, prec, device=dev, host_vals=host, buffering=mode)
            if mode == "auto":  # the plan's own choice: one of the two timed above
                rec["auto"] = "double" if S.halves else "single"
                del S
                continue
            y = S.apply(x)
            t_s = timed(lambda: S.apply(x, out=y), max(2, args.steps // 4))
            got = y.double().cpu().numpy()
            rec[mode] = {
                "cache_elems": S.cache_elems, "epochs": S.n_epochs, "loads": S.n_loads,
                "double_buffered": bool(S.halves),
                "loaded_GB": round(S.loaded_elems * es / 1e9, 3), "naive_GB": round(S.naive_elems * es / 1e9, 3),
                "copy_saved": round(1 - S.loaded_elems / max(S.naive_elems, 1), 4),
                "ms_per_product": round(t_s * 1e3, 2), "tflops": round(flops / t_s / 1e12, 3),
                "copy_GBps": round(S.loaded_elems * es / t_s / 1e9, 1),
                "frac_of_link": round(S.loaded_elems * es / t_s / 1e9 / link, 3),
                "rel_err_vs_in_hbm": float("%.3g" % (np.linalg.norm(got - ref64) / np.linalg.norm(ref64))),
                "rel_err_vs_oracle": float("%.3g" % (np.linalg.norm(got - want) / np.linalg.norm(want)))}
            del S
        caches[name] = dict(rec[rec["auto"]], auto=rec["auto"], single=rec["single"], double=rec["double"])
        log("cache %-6s auto=%s single %s double %s" % (name, rec["auto"], rec["single"], rec["double"]))
    head = caches["eighth"]
    line = {
        "metric": "out-of-HBM H_eff*psi (tree-traversal cache), copy bytes and rate", "value": head["tflops"],
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": head["ms_per_product"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "d1024: L=30 N=30 2Sz=0 D=1024 per block (mean sector 32, max 256), 900 terms "
                               "(operator pairs shared by up to 8 terms), seed 2; operator values in pinned host "
                               "memory, cache 1/8 of them",
                   "tasks": H.ntasks, "flops_per_step": flops, "operator_GB": round(host.numel() * es / 1e9, 3)},
        "in_hbm_ms": round(t_hbm * 1e3, 3), "pinned_copy_GBps": round(link, 1), "caches": caches,
        "roofline": {"bound": "pcie", "achieved": head["copy_GBps"], "peak": round(link, 1), "unit": "GB/s",
                     "frac": head["frac_of_link"], "peak_note": "plain pinned host-to-device copy of the same values"},
        "oracle_seconds": round(t_or, 1), "oracle_threads": thr,
    }
    print(json.dumps(line), flush=True)


def bench_su2(args):
    """Spin-adapted (SU(2)) products: a synthetic two-block instance of
    multiplet sectors (N within 4 of 15 per block, 2S <= 6, Gaussian profile
    of 1024 multiplets per block, at most 160 per sector; about 3230 states per
    block in U(1) terms), 150 tensor operators per side of rank 0, 1/2 or 1
    and 900 terms, seed 6, target N = 30, S = 0.  Every precision timed over
    the same steps; FP64 checked against the oracle's reduced route on the
    instance cut to its first 40 terms.  Prints one JSON line."""
    import torch
    from synth.su2 import su2_synthetic
    from paper_2305_05581_amd.tns import Su2Heff, KernelTimer
    from oracle import su2 as osu
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    I = su2_synthetic(9, 1024, 160, 150, 900, (30, 0), seed=6, max_2S=6)
    t_gen = time.time() - t0
    t0 = time.time()
    H = Su2Heff(I, device=dev)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    flops = H.total_flops
    states = int(sum(int(d) * (int(q[1]) + 1) for d, q in zip(I.dimL, I.qL)))
    log("su2: %d sectors, psi %d, %d tasks, %.1f GFLOP per product, build %.2f s (generate %.1f s)"
        % (H.n_sectors, H.psi_dim, H.ntasks, flops / 1e9, t_build, t_gen))
    psi = np.random.default_rng(3).standard_normal(H.psi_dim)
    res, outs = {}, {}
    order = [p for p in ("f64", "f32", "bf16x3") if p != args.prec] + [args.prec]
    for prec in order:
        dt = torch.float64 if prec == "f64" else torch.float32
        x = torch.from_numpy(psi).to(dev, dtype=dt)
        y = H.apply(x, prec)
        for _ in range(args.warmup):
            H.apply(x, prec, out=y)
        kt = KernelTimer(args.steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            kt.arm()
            H.apply(x, prec, out=y)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / args.steps
        ka, kb = np.array(kt.times_ms()).mean(axis=0)
        kt.close()
        outs[prec] = y.double()
        res[prec] = dict(ms_per_step=wall * 1e3, tflops=flops / wall / 1e12,
                         pct_peak=100 * flops / wall / 1e12 / PEAK[prec], phaseA_ms=float(ka), phaseB_ms=float(kb),
                         kernel_tflops=flops / ((ka + kb) / 1e3) / 1e12)
        log("%-6s %8.3f ms/step %7.2f TFLOP/s (%.1f%% of peak; phase A %.3f ms, phase B %.3f ms)"
            % (prec, wall * 1e3, res[prec]["tflops"], res[prec]["pct_peak"], ka, kb))
    ref = outs["f64"]
    for prec in ("f32", "bf16x3"):
        res[prec]["rel_err_vs_f64"] = float(torch.linalg.norm(outs[prec] - ref) / torch.linalg.norm(ref))
    # the oracle (reduced route) on the instance cut to its first 40 terms
    import dataclasses
    cut = dataclasses.replace(I, term_L=I.term_L[:40], term_R=I.term_R[:40], term_coef=I.term_coef[:40])
    Hc = Su2Heff(cut, device=dev)
    got = Hc.apply(torch.from_numpy(psi).to(dev), "f64").cpu().numpy()
    t = time.perf_counter()
    want = osu.sigma_reduced(cut, psi)
    t_or = time.perf_counter() - t
    parity = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    log("oracle check (first 40 terms): FP64 rel err %.2e (%.1f s)" % (parity, t_or))
    head = res[args.prec]
    line = {
        "metric": "spin-adapted H_eff*psi TFLOP/s (% MFMA peak)", "value": round(head["tflops"], 3),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "su2: synthetic SU(2) two-block instance, 1024 multiplets per block (%d states), "
                               "2S <= 6, 150 operators per side, 900 terms, N=30 S=0, seed 6" % states,
                   "sectors": H.n_sectors, "psi_dim": H.psi_dim, "tasks": H.ntasks, "flops_per_step": flops},
        "precisions": {k: {kk: float("%.4g" % vv) for kk, vv in v.items()} for k, v in res.items()},
        "oracle_parity_f64": {"terms": 40, "rel_frobenius": parity},
        "roofline": {"bound": "mfma", "achieved_both_phases": round(head["kernel_tflops"], 3),
                     "peak": round(PEAK[args.prec], 1), "unit": "TFLOP/s",
                     "frac": round(head["kernel_tflops"] / PEAK[args.prec], 4)},
        "setup_seconds": {"generate": round(t_gen, 2), "build": round(t_build, 2)},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="bf16x3", choices=["bf16x3", "f32", "f64"])
    ap.add_argument("--config", default="d4096",
                    choices=sorted(CONFIGS) + ["batch64", "grad1024", "sbmm4s", "renorm", "ttcache", "su2"],
                    help="batch64: many uneven instances, one launch per phase vs one product at a time; "
                         "grad1024: forward and backward at L=30, D=1024; sbmm4s: the paper's batched-GEMM "
                         "scheme with library GEMMs against the fused kernels at L=30, D=1024")
    ap.add_argument("--instances", type=int, default=64, help="batch64: number of instances")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's tile autotuner (per sector-size bucket) before timing")
    ap.add_argument("--no-davidson", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dav-iter", type=int, default=120, help="cap on Davidson products per solve")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes first (counter calibration under a profiler)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write the phase-A HBM traffic of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; "
                         "with --calib-bytes) into " + TRAFFIC_FILE + " and exit")
    ap.add_argument("--only", default=None, choices=["bf16x3", "f32", "f64"],
                    help="time only this precision (profiling runs)")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU's share only: the library runs the product on a single GPU "
              "(no collectives or sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.config == "batch64":
        bench_batch(args)
        return
    if args.config == "grad1024":
        bench_grad(args)
        return
    if args.config == "sbmm4s":
        bench_sbmm4s(args)
        return
    if args.config == "ttcache":
        bench_ttcache(args)
        return
    if args.config == "su2":
        bench_su2(args)
        return
    if args.config == "renorm":
        bench_renorm(args)
        return

    import torch
    from synth import synthetic_problem, gaussian_psi, gapped_guess
    from paper_2305_05581_amd.tns import HeffProblem, KernelTimer

    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    P = make_problem(cfg)
    t_gen = time.time() - t0
    log("generated: %d terms, %d blocks, %.1f GB operators, psi %d (%.1f s)"
        % (P.nTerms, P.nBlk, P.op_vals.nbytes / 1e9, P.psi_dim, t_gen))
    t0 = time.time()
    vals64 = torch.empty(len(P.op_vals), dtype=torch.float64, device=dev)
    chunk = 1 << 28
    for i in range(0, len(P.op_vals), chunk):
        vals64[i:i + chunk].copy_(torch.from_numpy(P.op_vals[i:i + chunk]))
    torch.cuda.synchronize()
    t_up = time.time() - t0
    # task table + schedules (levels 1-2), timed separately
    torch.cuda.synchronize()
    t0 = time.time()
    H = HeffProblem(P, device=dev, vals64=vals64)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    flops = H.total_flops
    log("tasks %d, %.3f TFLOP per product, build %.3f s, upload %.1f s" % (H.ntasks, flops / 1e12, t_build, t_up))
    for p in ("f32", "bf16x3"):
        H.operands(p)
    psi64 = torch.from_numpy(gaussian_psi(P, 3)).to(dev)
    psi32 = psi64.float()
    if args.calib_bytes > 0:
        src = torch.ones(args.calib_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)  # one element-wise kernel: reads and writes calib_bytes
        torch.cuda.synchronize()
        log("calibration copy: %d bytes" % (src.numel() * 4))
        del src, dst

    if args.autotune:
        t = time.time()
        tab = H.autotune(psi64 if args.prec == "f64" else psi32, args.prec)
        log("autotuned tile table %08x for %s (%.1f s)" % (tab, args.prec, time.time() - t))
    tasks_dev, ptr = H.tasks()
    flops_a, flops_b = phase_flops(P, tasks_dev)
    log("phase A %.3f TFLOP, phase B %.3f TFLOP (sum %.3f)" % (flops_a / 1e12, flops_b / 1e12,
                                                               (flops_a + flops_b) / 1e12))

    def run(prec, steps, warmup):
        x = psi64 if prec == "f64" else psi32
        out = torch.empty_like(x)
        for _ in range(warmup):
            H.apply(x, prec, out=out)
        kt = KernelTimer(steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            kt.arm()
            H.apply(x, prec, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        kms = np.array(kt.times_ms())
        kt.close()
        return out, wall, kms.mean(axis=0) / 1e3

    res = {}
    order = [p for p in ("f64", "f32", "bf16x3") if p != args.prec] + [args.prec]
    if args.only:
        order = [args.only]
    outs = {}
    for prec in order:
        out, wall, (ka, kb) = run(prec, args.steps, args.warmup)
        outs[prec] = out.double()
        res[prec] = dict(ms_per_step=wall * 1e3, kernel_ms=(ka + kb) * 1e3, tflops=flops / wall / 1e12,
                         kernel_tflops=flops / (ka + kb) / 1e12, pct_peak=100 * flops / wall / 1e12 / PEAK[prec],
                         phaseA_ms=ka * 1e3, phaseA_tflops=flops_a / ka / 1e12,
                         phaseB_ms=kb * 1e3, phaseB_tflops=flops_b / kb / 1e12)
        log("%-6s %8.2f ms/step  %7.2f TFLOP/s  (%.1f%% of %s peak; phase A %.2f ms %.1f TFLOP/s, "
            "phase B %.2f ms %.1f TFLOP/s)"
            % (prec, wall * 1e3, flops / wall / 1e12, res[prec]["pct_peak"], prec, ka * 1e3,
               flops_a / ka / 1e12, kb * 1e3, flops_b / kb / 1e12))
    if "f64" in outs:
        ref = outs["f64"]
        for prec in ("f32", "bf16x3"):
            if prec in outs:
                res[prec]["sigma_rel_err_vs_f64"] = float(torch.linalg.norm(outs[prec] - ref) / torch.linalg.norm(ref))
                log("%s sigma relative error against the FP64 product: %.3e" % (prec, res[prec]["sigma_rel_err_vs_f64"]))
    if args.only:
        print(json.dumps({"only": args.only, **res[args.only]}), flush=True)
        return

    # measured MFMA ceilings (per algorithmic flop: BF16x3 issues three BF16 products)
    mpeak = {}
    try:
        from paper_2305_05581_amd.tns import mfma_peak
        for prec in res:
            inst = mfma_peak(prec)
            mpeak[prec] = inst / 3.0 if prec == "bf16x3" else inst
            res[prec]["pct_measured_peak"] = 100 * res[prec]["tflops"] / mpeak[prec]
        log("measured MFMA peak (TFLOP/s per algorithmic flop): " +
            ", ".join("%s %.1f (%.1f%% of it)" % (p, mpeak[p], res[p]["pct_measured_peak"]) for p in mpeak))
    except Exception as e:  # reported, not fatal
        mpeak = {"error": str(e)[:200]}

    # hipGraph replay of the headline product
    graph = {}
    try:
        x = psi64 if args.prec == "f64" else psi32
        out = torch.empty_like(x)
        H.apply(x, args.prec, out=out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            H.apply(x, args.prec, out=out)
        g.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(out.double(), outs[args.prec]))
        t = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        gw = (time.perf_counter() - t) / args.steps
        graph = dict(ms_per_step=gw * 1e3, tflops=flops / gw / 1e12, equal_to_eager=same)
    except Exception as e:  # reported, not fatal
        graph = dict(error=str(e)[:200])

    dav = {}
    if not args.no_davidson and cfg["gapped"]:
        x0 = torch.from_numpy(gapped_guess(P, 2)).to(dev)
        for inner, tol in (("f64", 1e-6), (args.prec if args.prec != "f64" else "f32", 1e-5)):
            log("davidson %s ..." % inner)
            torch.cuda.synchronize()
            t = time.perf_counter()
            e, _, info = H.davidson(x0, inner=inner, tol_res=tol, max_iter=args.dav_iter)
            torch.cuda.synchronize()
            dav[inner] = dict(energy=e, seconds=time.perf_counter() - t, **info)
            log("davidson %-6s E=%.12f  %.2f s  %s" % (inner, e, dav[inner]["seconds"], info))
        keys = list(dav)
        if len(keys) == 2:
            dav["abs_energy_diff"] = abs(dav[keys[0]]["energy"] - dav[keys[1]]["energy"])
            dav["within_1e-8"] = dav["abs_energy_diff"] <= 1e-8
            dav["speedup"] = dav[keys[0]]["seconds"] / dav[keys[1]]["seconds"]

    cpu = None
    oracle_parity = {}
    if not args.no_cpu:
        from oracle import heff as oheff
        threads = len(os.sched_getaffinity(0))
        t = time.perf_counter()
        tl = oheff.enumerate_tasks(P)  # the oracle's own task list (levels 1-2), timed apart from sigma
        log("oracle task list: %d tasks, %.1f s" % (len(tl), time.perf_counter() - t))
        psi_np = psi64.cpu().numpy()
        t = time.perf_counter()
        ref, threads = oheff.sigma_threaded(P, psi_np, tl, threads=threads)
        el = time.perf_counter() - t
        cpu = dict(value=flops / el / 1e12, unit="TFLOP/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
                   sample="the whole product (%.2f TFLOP, %d output sectors), %.1f s; Python threads over output "
                          "sectors, BLAS one thread per call" % (flops / 1e12, P.nS, el))
        log("cpu oracle: %.4f TFLOP/s on %s" % (cpu["value"], cpu["sample"]))
        nref = np.linalg.norm(ref)
        for prec in outs:
            o = outs[prec].cpu().numpy()
            worst = 0.0
            for sct in range(P.nS):
                a, b = P.psi_off[sct], P.psi_off[sct + 1]
                nb = np.linalg.norm(ref[a:b])
                if nb > 0:
                    worst = max(worst, float(np.linalg.norm(o[a:b] - ref[a:b]) / nb))
            oracle_parity[prec] = {"rel_frobenius": float(np.linalg.norm(o - ref) / nref), "worst_sector": worst}
            log("%s sigma against the oracle: %.3e (worst sector %.3e)"
                % (prec, oracle_parity[prec]["rel_frobenius"], worst))
        del ref
    eo = oracle_energy(args.config)
    if eo is not None and dav:
        for k in list(dav):
            if isinstance(dav[k], dict):
                dav[k]["abs_energy_err_vs_oracle"] = abs(dav[k]["energy"] - eo["energy"])
        dav["oracle_energy"] = {k: eo[k] for k in ("energy", "res_norm", "iters", "tol_res", "davidson_seconds",
                                                   "threads", "cpu_model") if k in eo}

    head = res[args.prec]
    # dominant kernel of the headline precision: the longer of the two phases
    dom = 0 if head["phaseA_ms"] >= head["phaseB_ms"] else 1
    d_ms = head["phaseA_ms"] if dom == 0 else head["phaseB_ms"]
    d_fl = flops_a if dom == 0 else flops_b
    ach = d_fl / (d_ms / 1e3) / 1e12
    tA, tB = measured_traffic(args.config, args.prec, 0), measured_traffic(args.config, args.prec, 1)
    comp = compulsory_bytes(P, tasks_dev, args.prec)
    roofline = {"bound": "mfma", "kernel": KERNEL[args.prec][dom], "achieved": round(ach, 3),
                "peak": round(PEAK[args.prec], 1), "unit": "TFLOP/s", "frac": round(ach / PEAK[args.prec], 4),
                "traffic": (tA, tB)[dom],
                "traffic_per_product": (tA + tB) if (tA is not None and tB is not None) else None,
                "compulsory_bytes_per_product": comp,
                "traffic_over_compulsory": round((tA + tB) / comp, 2) if (tA is not None and tB is not None)
                else None,
                "algorithmic_flops_per_launch": d_fl, "avg_launch_ms": round(d_ms, 3),
                "both_phases_tflops": round(head["kernel_tflops"], 3),
                "measured_peak": round(mpeak[args.prec], 1) if args.prec in mpeak else None,
                "peak_note": ("BF16 dense 2516.6 TFLOP/s / 3 MFMA products per algorithmic flop"
                              if args.prec == "bf16x3" else "dense MFMA peak of the dtype")}
    line = {
        "metric": ("H_eff*psi TFLOP/s (% MFMA peak) at D=4096, mixed vs FP64, at 1e-8 Ha" if args.config == "d4096"
                   else "H_eff*psi TFLOP/s (%% MFMA peak), %s workload" % args.config),
        "value": round(head["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": ("%s: L=%d N=%d 2Sz=%d, exact blocks of %d states from seeded molecular integrals "
                                "(seed %d), %d terms" % (args.config, cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"],
                                                          cfg["seed"], P.nTerms)) if cfg.get("exact") else
                               ("%s: L=%d N=%d 2Sz=%d D=%d per block (mean sector %d, max %d), %d terms%s, seed %d"
                                % (args.config, cfg["L"], cfg["N"], cfg["twoSz"], cfg["D"], cfg["mean"],
                                   cfg["dmax"], P.nTerms, " + gapped diagonal" if cfg["gapped"] else "",
                                   cfg["seed"])),
                   "tasks": H.ntasks, "flops_per_step": flops, "psi_dim": P.psi_dim,
                   "operator_GB_f64": round(P.op_vals.nbytes / 1e9, 2), "parallelism": "single GPU",
                   "tile_table": "%08x" % H.tiles, "autotuned": bool(args.autotune)},
        "pct_mfma_peak": round(head["pct_peak"], 2),
        "measured_mfma_peak": {k: round(v, 1) for k, v in mpeak.items() if isinstance(v, float)},
        "precisions": {k: {kk: (float("%.4g" % vv) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                       for k, v in res.items()},
        "mixed_vs_f64_speedup": round(res[args.prec]["tflops"] / res["f64"]["tflops"], 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_parity": oracle_parity,
        "davidson": dav,
        "hipgraph": graph,
        "setup_seconds": {"generate": round(t_gen, 2), "upload": round(t_up, 2), "task_table": round(t_build, 4)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
