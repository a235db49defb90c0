"""The forward product captured in a HIP graph (torch.cuda.CUDAGraph) replays
bitwise equal to the eager call, replay after replay, with eager work and
synchronisations in between; the library records no memset in the graph."""
import pytest
import torch

from synth import synthetic_problem, gaussian_psi

from gpu_common import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_graph_replay_matches_eager(prec):
    from paper_2305_05581_amd.tns import HeffProblem
    P = synthetic_problem(22, 22, 0, 700, 23, 187, 120, seed=12)
    H = HeffProblem(P)
    dt = torch.float64 if prec == "f64" else torch.float32
    x = to_dev(gaussian_psi(P, 1), dt)
    out = torch.empty_like(x)
    H.apply(x, prec, out=out)          # warm-up: operands, workspace
    ref = out.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.apply(x, prec, out=out)
    for rep in range(4):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        say(prec, "replay", rep)
        assert torch.equal(out, ref)
        y = H.apply(x, prec)           # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
