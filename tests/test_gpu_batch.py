"""Batched products (many uneven instances, one launch per GEMM phase) on the
GPU: bitwise equal to separate products, accumulate form, hipGraph replay,
and the oracle on every instance."""
import numpy as np
import pytest
import torch

from synth import synthetic_problem, gaussian_psi, molecular_integrals
from oracle import heff as oheff
from oracle.blocks import Construction

from gpu_common import say, rel, to_dev, SIGMA_TOL

pytestmark = pytest.mark.gpu

TOL = SIGMA_TOL


@pytest.fixture(scope="module")
def batch():
    from paper_2305_05581_amd.tns import HeffProblem, HeffBatch
    makers = [
        lambda: synthetic_problem(22, 22, 0, 700, 23, 187, 120, seed=12),
        lambda: synthetic_problem(16, 16, 0, 96, 8, 24, 60, seed=5, gapped=True),
        lambda: synthetic_problem(21, 21, 1, 300, 17, 136, 90, seed=4001),
        lambda: Construction(*molecular_integrals(6, 11), 6, 0, l=2).problem(),
        lambda: synthetic_problem(12, 12, 0, 40, 6, 16, 30, seed=8),
    ]
    Ps, Hs = [], []
    for i, mk in enumerate(makers):
        say("build instance", i)
        P = mk()
        Ps.append(P)
        Hs.append(HeffProblem(P))
    return Ps, Hs, HeffBatch(Hs)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_batch_equals_separate_and_oracle(batch, prec):
    Ps, Hs, B = batch
    dt = torch.float64 if prec == "f64" else torch.float32
    psis = [to_dev(gaussian_psi(P, 3 + i), dt) for i, P in enumerate(Ps)]
    say("batch apply", prec)
    outs = B.apply(psis, prec)
    torch.cuda.synchronize()
    for i, (P, H, x, y) in enumerate(zip(Ps, Hs, psis, outs)):
        ref = H.apply(x, prec)
        assert torch.equal(y, ref), "instance %d differs from its separate product" % i
        e = rel(y.double().cpu().numpy(), oheff.sigma(P, x.double().cpu().numpy()))
        say("  instance %d rel err vs oracle %.2e" % (i, e))
        assert e <= TOL[prec]


def test_batch_accumulate(batch):
    Ps, Hs, B = batch
    psis = [to_dev(gaussian_psi(P, 7 + i), torch.float32) for i, P in enumerate(Ps)]
    base = [to_dev(gaussian_psi(P, 20 + i), torch.float32) for i, P in enumerate(Ps)]
    outs = [b.clone() for b in base]
    B.apply(psis, "f32", outs=outs, beta=1.0)
    for H, x, b, y in zip(Hs, psis, base, outs):
        ref = b.clone()
        H.apply(x, "f32", out=ref, beta=1.0)
        assert torch.equal(y, ref)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_batch_graph_replay(batch, prec):
    Ps, Hs, B = batch
    psis = [to_dev(gaussian_psi(P, 30 + i), torch.float32) for i, P in enumerate(Ps)]
    outs = [torch.empty_like(x) for x in psis]
    B.apply(psis, prec, outs=outs)
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.apply(psis, prec, outs=outs)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), "replay %d instance %d" % (rep, i)


def test_batch_rejects_bad_arguments(batch):
    Ps, Hs, B = batch
    from paper_2305_05581_amd.tns import TnsError
    psis = [to_dev(gaussian_psi(P, 1), torch.float32) for P in Ps]
    with pytest.raises(ValueError):
        B.apply(psis[:-1], "f32")
    with pytest.raises(TnsError):
        B.apply(psis, "f32", outs=[torch.empty_like(x) for x in psis], beta=0.5)


TABLES = [0x80808080, 0x40404040, 0x20202020, 0x80404020, 0x20408080, 0x80804020, 0x00000000]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_tile_tables_give_identical_results(batch, prec):
    """Every tile table computes every output element in the same order."""
    Ps, Hs, B = batch
    dt = torch.float64 if prec == "f64" else torch.float32
    H = Hs[0]
    x = to_dev(gaussian_psi(Ps[0], 41), dt)
    ref = H.apply(x, prec)
    default = H.tiles
    try:
        for tab in TABLES:
            say("tiles %08x %s" % (tab, prec))
            H.set_tiles(tab)
            assert H.tiles == tab
            assert torch.equal(H.apply(x, prec), ref)
    finally:
        H.set_tiles(default)


def test_set_tiles_rejects_invalid(batch):
    from paper_2305_05581_amd.tns import TnsError
    Ps, Hs, B = batch
    with pytest.raises(TnsError):
        Hs[1].set_tiles(0x80804010)
    with pytest.raises(TnsError):
        Hs[1].set_tiles(0x00804030)


def test_autotune_single_and_batch(batch):
    Ps, Hs, B = batch
    x = to_dev(gaussian_psi(Ps[0], 43), torch.float32)
    ref = Hs[0].apply(x, "f32")
    tab = Hs[0].autotune(x, "f32")
    say("autotuned single table %08x" % tab)
    assert all(((tab >> (8 * b)) & 0xff) in (0, 32, 64, 128) for b in range(4))
    assert Hs[0].tiles == tab
    assert torch.equal(Hs[0].apply(x, "f32"), ref)
    psis = [to_dev(gaussian_psi(P, 50 + i), torch.float32) for i, P in enumerate(Ps)]
    refs = [H.apply(p, "f32") for H, p in zip(Hs, psis)]
    tb = B.autotune(psis, "f32")
    say("autotuned batch table %08x" % tb)
    assert all(H.tiles == tb for H in Hs)
    outs = B.apply(psis, "f32")
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
