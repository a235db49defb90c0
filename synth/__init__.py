"""Seeded synthetic inputs for the two-site effective-Hamiltonian product.

This package produces *inputs only*: one- and two-electron integrals, block
sector tables, random block-sparse operators, Hamiltonian term lists and
wavefunctions. It holds none of the arithmetic of the method (no operator
products, no fermionic signs of the product rule, no task lists); both the
CPU oracle and the GPU path read what it produces.

Array conventions shared by every consumer (the "problem" dictionary):

* Sectors are ``(N, 2Sz)`` pairs, sorted ascending (N first).
* Site states: 0 = empty, 1 = up, 2 = down, 3 = doubly occupied; the
  quantum numbers are (0,0), (1,1), (1,-1), (2,0).
* Site monomials carry the id ``4*u + d`` where ``u`` (up spin) and ``d``
  (down spin) are in {0: 1, 1: n, 2: c^dagger, 3: c}; the up factor stands
  to the left of the down factor.
* Wavefunction sectors ``(iL, sa, sb, iR)`` are sorted by ``(iL, sa, sb)``;
  each is a dense ``dimL[iL] x dimR[iR]`` row-major matrix, packed in that
  order (offsets ``psi_off``).
* Operator blocks are dense row-major matrices stored in one flat array at
  element offset ``blk_off`` with leading dimension ``blk_ld``; blocks are
  listed per operator in ascending in-sector order.
"""

from .problem import (SHIFTS, MONO_SHIFT, mono_id, mono_parity, site_q,
                      Problem, block_profile, synthetic_problem, gaussian_psi, gapped_guess)
from .integrals import molecular_integrals, hubbard_integrals

__all__ = ["SHIFTS", "MONO_SHIFT", "mono_id", "mono_parity", "site_q", "Problem",
           "block_profile", "synthetic_problem", "gaussian_psi", "gapped_guess",
           "molecular_integrals", "hubbard_integrals"]
