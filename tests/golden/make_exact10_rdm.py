"""Writes exact10_rdm.json: the spin-summed one- and two-particle reduced
density matrices of a fixed normalised vector on the exact-block L = 10
instance (10 orbitals, 10 electrons, 2Sz = 0, blocks of 4 orbitals with all
256 states each, integrals from seed 21), computed by brute force over the
63504 FCI determinants.

Calls only the oracle (block construction, determinant list, RDMs) on inputs
from the seeded generators.  The energy <x, H x> is linear in the integrals,
so dE/dh_ij = gamma_ij and dE/d(ij|kl) = Gamma_ijkl / 2 for any x: the GPU
test contracts the device's operator-block gradients to these.

    python tests/golden/make_exact10_rdm.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from synth import molecular_integrals, gaussian_psi  # noqa: E402
from oracle.blocks import Construction  # noqa: E402
from oracle.fock import determinants, rdms  # noqa: E402

L, N, TWO_SZ, INT_SEED, PSI_SEED = 10, 10, 0, 21, 7
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact10_rdm.json")


def main():
    t = time.time()
    h, eri = molecular_integrals(L, INT_SEED)
    C = Construction(h, eri, N, TWO_SZ)
    P = C.problem()
    dets = determinants(L, N, TWO_SZ)
    idx = C.fci_map(P, dets)
    x = gaussian_psi(P, PSI_SEED)
    xf = np.zeros(len(dets))
    xf[idx] = x
    g1, g2 = rdms(xf, dets, L)
    rec = {"L": L, "N": N, "twoSz": TWO_SZ, "integral_seed": INT_SEED, "psi": "gaussian_psi(P, %d)" % PSI_SEED,
           "fci_dim": int(len(dets)), "psi_dim": int(P.psi_dim),
           "gamma": g1.tolist(), "Gamma": g2.reshape(-1).tolist(),
           "seconds": round(time.time() - t, 1), "written_by": "tests/golden/make_exact10_rdm.py (oracle only)"}
    with open(OUT, "w") as fh:
        json.dump(rec, fh)
    print("written %s (%.0f s), trace gamma %.12f" % (OUT, time.time() - t, float(np.trace(g1))))


if __name__ == "__main__":
    main()
