import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def cfg1():
    """L=8, N=8, 2Sz=0 exact blocks from seeded integrals, FCI dim 4900."""
    from synth import molecular_integrals
    from oracle.blocks import Construction
    from oracle.fock import fci_hamiltonian
    h, eri = molecular_integrals(8, 1)
    C = Construction(h, eri, 8, 0)
    P = C.problem()
    H, dets = fci_hamiltonian(h, eri, 8, 0)
    return dict(h=h, eri=eri, C=C, P=P, H=H, dets=dets, idx=C.fci_map(P, dets))
