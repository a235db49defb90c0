"""Degenerate inputs on the GPU, each against the oracle: a problem without
terms (no tasks at all), a single term (most output sectors receive no task),
terms with the identity on both blocks (site operators only), an empty
instance inside a batch, and one-element sectors."""
import dataclasses

import numpy as np
import pytest
import torch

from synth import synthetic_problem, gaussian_psi
from synth.problem import mono_id
from oracle import grad as ograd
from oracle import heff as oheff

from gpu_common import say, rel, to_dev, SIGMA_TOL

pytestmark = pytest.mark.gpu

TOL = SIGMA_TOL
PRECS = ["f64", "f32", "bf16x3"]


def _base():
    # bond dimension 24 over many sectors: most sectors hold 1 to 3 states
    return synthetic_problem(10, 10, 0, 24, 3, 8, 40, seed=77)


def _with_terms(P, rows):
    """Copy of P with the terms replaced by rows (L, ma, mb, R, coef)."""
    cols = list(zip(*rows)) if rows else [(), (), (), (), ()]
    return dataclasses.replace(
        P,
        term_L=np.asarray(cols[0], dtype=np.int32), term_ma=np.asarray(cols[1], dtype=np.int32),
        term_mb=np.asarray(cols[2], dtype=np.int32), term_R=np.asarray(cols[3], dtype=np.int32),
        term_coef=np.asarray(cols[4], dtype=np.float64))


def _cases():
    P = _base()
    first = (int(P.term_L[0]), int(P.term_ma[0]), int(P.term_mb[0]), int(P.term_R[0]), float(P.term_coef[0]))
    site_only = [
        (-1, mono_id(1, 0), 0, -1, 0.7),                  # n_up on site a
        (-1, mono_id(2, 0), mono_id(3, 0), -1, -0.3),     # up hop a <- b
        (-1, mono_id(3, 0), mono_id(2, 0), -1, -0.3),     # its adjoint
        (-1, mono_id(1, 1), 0, -1, 1.1),                  # n_up n_down on site a
        (-1, 0, mono_id(0, 1), -1, 0.25),                 # n_down on site b
    ]
    return {
        "no_terms": _with_terms(P, []),
        "single_term": _with_terms(P, [first]),
        "site_only": _with_terms(P, site_only),
        "one_element": synthetic_problem(8, 8, 0, 6, 1, 2, 20, seed=3),
    }


@pytest.fixture(scope="module")
def edge():
    from paper_2305_05581_amd.tns import HeffProblem
    out = {}
    for name, P in _cases().items():
        say("build", name, "terms", P.nTerms)
        out[name] = (P, HeffProblem(P), oheff.enumerate_tasks(P))
    return out


def test_task_table(edge):
    for name, (P, H, tasks) in edge.items():
        say(name, "tasks", H.ntasks, "oracle", len(tasks))
        t, ptr = H.tasks()
        ref, rptr = oheff.task_table(P)
        assert t.tobytes() == ref.tobytes(), name
        assert np.array_equal(ptr, rptr), name
        assert H.total_flops == int(ref["cost"].sum())
    assert edge["no_terms"][1].ntasks == 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["no_terms", "single_term", "site_only", "one_element"])
def test_sigma(edge, name, prec):
    P, H, tasks = edge[name]
    dt = torch.float64 if prec == "f64" else torch.float32
    x = to_dev(gaussian_psi(P, 11), dt)
    ref = oheff.sigma(P, x.double().cpu().numpy())
    # beta = 0 overwrites whatever the output held
    out = torch.full((H.psi_dim,), float("nan"), dtype=dt, device="cuda")
    H.apply(x, prec, out=out, beta=0.0)
    y = out.double().cpu().numpy()
    assert np.all(np.isfinite(y))
    # sectors that receive no task are exact zeros
    _, ptr = H.tasks()
    for s in range(P.nS):
        if ptr[s + 1] == ptr[s]:
            assert not np.any(y[P.psi_off[s]:P.psi_off[s + 1]]), (name, s)
    if len(tasks) == 0:
        assert not np.any(y)
    else:
        e = rel(y, ref)
        say("%s %s rel err %.2e" % (name, prec, e))
        assert e <= TOL[prec]
    # beta = 1 adds to what the output held
    base = to_dev(gaussian_psi(P, 12), dt)
    acc = base.clone()
    H.apply(x, prec, out=acc, beta=1.0)
    want = base.double().cpu().numpy() + ref
    assert rel(acc.double().cpu().numpy(), want) <= TOL[prec]


@pytest.mark.parametrize("name", ["no_terms", "single_term", "site_only"])
def test_backward(edge, name):
    P, H, tasks = edge[name]
    psi, G = gaussian_psi(P, 1), gaussian_psi(P, 2)
    gp, go = H.backward(to_dev(psi), to_dev(G), "f64")
    if len(tasks) == 0:
        assert not torch.any(gp) and not torch.any(go)
        return
    dpsi, dvals, _ = ograd.backward(P, psi, G, tasks)
    e1 = rel(gp.cpu().numpy(), dpsi)
    e2 = rel(go.cpu().numpy(), dvals) if np.any(dvals) else float(np.abs(go.cpu().numpy()).max())
    say("%s backward rel err dpsi %.2e dops %.2e" % (name, e1, e2))
    assert e1 <= 1e-12 and e2 <= 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_batch_with_empty_instance(edge, prec):
    from paper_2305_05581_amd.tns import HeffBatch
    names = ["single_term", "no_terms", "site_only"]
    Hs = [edge[n][1] for n in names]
    dt = torch.float64 if prec == "f64" else torch.float32
    xs = [to_dev(gaussian_psi(edge[n][0], 21 + i), dt) for i, n in enumerate(names)]
    outs = HeffBatch(Hs).apply(xs, prec)
    for n, H, x, y in zip(names, Hs, xs, outs):
        assert torch.equal(y, H.apply(x, prec)), n
    assert not torch.any(outs[1])
