"""MI355X (gfx950) two-site effective-Hamiltonian product sigma = H_eff psi.

The compute path lives in ``libtns.so`` (HIP kernels behind the C ABI of
``include/tns.h``); :mod:`paper_2305_05581_amd.tns` is its ctypes binding.
Importing this package loads nothing; the library is opened on first use.
"""
