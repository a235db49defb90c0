"""Plain FP64 CPU oracle for the two-site effective-Hamiltonian product.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this
package; the GPU library never does, and this package imports nothing from
it.  Inputs come from :mod:`synth` (seeded generators without any of the
method's arithmetic) or from this package's own construction of block
operators from integrals.

Modules (each function cites the passage of the paper it follows):

* :mod:`oracle.fock`     Fock space, Jordan-Wigner strings, brute-force FCI
                         Hamiltonian of Eq. (1) and reduced density matrices.
* :mod:`oracle.blocks`   Exact block bases with (N, 2Sz) sectors, site
                         monomials, string splitting over the four subsystems
                         of the two-site topology, naive and complementary
                         (partially summed) term tables.
* :mod:`oracle.heff`     sigma = H_eff psi by the definition of Eq. (2), the
                         canonical task table, and the full-form (dense)
                         assembly used as the level-4 self-check.
* :mod:`oracle.davidson` FP64 Davidson iteration for the lowest eigenpair.
* :mod:`oracle.grad`     Gradients of a scalar loss on sigma with respect to
                         psi and to the operator blocks.

Parity pins: every function is checked by the CPU test suite against
brute-force FCI, closed forms (free fermions, Hubbard dimer, two-orbital
two-electron spectra), invariants (Hermiticity, particle number, spin),
brute-force enumeration and finite differences.  Items with no such pin are
marked "parity unpinned" in their docstring.
"""
