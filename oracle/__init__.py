"""CPU FP64 oracle for the TLR Matérn log-likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the ``paper_1804_09137_amd``
package, its HIP kernels, its C-ABI) imports, calls or links anything here.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: its only common
dependency is the seeded input generator module ``synth``.

Contents (each function cites the passage of arXiv 1804.09137 it follows):

* ``matern``       Eq. (MaternCov) and its range derivative (Section IV).
* ``ordering``     Morton (Z-order) point ordering (the paper is silent on the
                   ordering; this is the reading the build adopts).
* ``dense``        exact log-likelihood Eq. (1) (Section III) by a dense
                   Cholesky, its gradient in (sigma^2, beta), and the
                   measurement generator z = L eps (Section VIII-D).
* ``tlr``          a CPU tile low-rank Cholesky likelihood (Section V): SVD
                   compression of off-diagonal tiles at an absolute threshold,
                   right-looking TLR Cholesky with QR+SVD recompression.

Parity pins: see ``tests/test_oracle_*.py``.  Every function here is pinned by
at least one closed form, brute-force or invariant test; none is "parity
unpinned".
"""
