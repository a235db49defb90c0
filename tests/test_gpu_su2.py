"""GPU parity of the spin-adapted (SU(2)) product (Section IV.E) against the
oracle: Fock-space instances (exact reduced blocks, whole and truncated
multiplet bases) against V^T H V psi, a synthetic instance with larger spins
and ragged sectors against the reduced route, in FP64, FP32 and BF16x3; the
device task table against the library's host table; the spin-adapted
Davidson ground state against the oracle's lowest eigenvalue."""
import numpy as np
import pytest
import torch

from synth.su2 import su2_instance, su2_synthetic
from oracle import su2 as osu

from gpu_common import say, rel, to_dev, SIGMA_TOL

pytestmark = pytest.mark.gpu


def _instances():
    return {
        "fock3x3_S0": lambda: su2_instance(3, 3, (6, 0), seed=31),
        "fock3x3_S1_cut": lambda: su2_instance(3, 3, (6, 2), seed=32, keep_frac=0.6),
        "fock3x2_S1/2": lambda: su2_instance(3, 2, (5, 1), seed=33),
        "synthetic_ragged": lambda: su2_synthetic(7, 600, 96, 40, 300, (14, 2), seed=5, max_2S=6),
    }


@pytest.fixture(scope="module")
def built():
    from paper_2305_05581_amd.tns import Su2Heff
    out = {}
    for name, mk in _instances().items():
        I = mk()
        say("su2 build", name, "psi", I.psi_dim, "blocks", len(I.blk_op), "terms", len(I.term_L))
        H = Su2Heff(I)
        psi = np.random.default_rng(7).standard_normal(I.psi_dim)
        ref = osu.sigma(I, psi) if I.lL else osu.sigma_reduced(I, psi)
        out[name] = (I, H, psi, ref)
    return out


@pytest.mark.parametrize("name", list(_instances()))
def test_task_table(built, name):
    from paper_2305_05581_amd.tns import su2_tables
    I, H, psi, ref = built[name]
    secL, secR, off, tasks, ptr = su2_tables(I)
    dt, dp = H.tasks()
    say("su2 tasks", name, len(dt))
    assert dt.tobytes() == tasks.tobytes() and np.array_equal(dp, ptr)
    assert H.psi_dim == int(off[-1]) and H.n_sectors == len(secL)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("name", list(_instances()))
def test_sigma_parity(built, name, prec):
    I, H, psi, ref = built[name]
    dt = torch.float64 if prec == "f64" else torch.float32
    got = H.apply(to_dev(psi, dt), prec)
    torch.cuda.synchronize()
    e = rel(got.cpu().numpy(), ref)
    say("su2 sigma", name, prec, "rel err %.2e" % e)
    assert e <= SIGMA_TOL[prec]


@pytest.mark.parametrize("inner", ["f64", "bf16x3"])
def test_davidson_ground_state(built, inner):
    I, H, psi, ref = built["fock3x3_S0"]
    V = osu.coupled_basis(I)
    e_ref = float(np.linalg.eigvalsh(V.T @ (osu.hamiltonian(I) @ V))[0])
    x0 = torch.from_numpy(np.random.default_rng(8).standard_normal(I.psi_dim))
    e, x, info = H.davidson(x0, inner=inner, tol_res=1e-7)
    say("su2 davidson", inner, "E %.12f ref %.12f" % (e, e_ref), info)
    assert info["converged"]
    assert abs(e - e_ref) < 1e-8
