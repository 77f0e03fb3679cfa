"""MI355X (gfx950) engine for the classical simulation of Quantum Hamiltonian
Descent (arXiv 2303.01471): batched split-operator pseudo-spectral evolution in
hand-written HIP behind a C ABI (include/qhd.h).

``paper_2303_01471_amd.qhd`` is the ctypes binding; importing this package does
not load the library.
"""
__all__ = ["qhd"]
