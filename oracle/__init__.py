"""CPU oracle for the Liouville-Lanczos magnon hot path (arXiv:2203.01120).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(the HIP library and its Python binding) never does, and shares no code with
it.  Everything here is plain, slow, obviously-correct NumPy/SciPy in FP64:

* ``grid``        plane-wave sphere <-> FFT-grid transforms and field Fourier series
* ``xc``          Slater-exchange LSDA potentials and the ALSDA response kernel
* ``scf``         dense-matrix Kohn-Sham Hamiltonian, noncollinear SCF, non-SCF points
* ``liouvillian`` batch representation, matrix-free Liouvillian, u/v vectors
* ``dense``       transition-space ("sum over transitions") Liouvillian
* ``lanczos``     non-Hermitian and pseudo-Hermitian Lanczos recursions
* ``chi``         susceptibility from the tridiagonal matrix, plus Kubo K=0 sum

Pins against things other than itself live in ``tests/test_oracle_*.py``.
The SCF ground state is pinned by its homogeneous-electron-gas limit (closed
form), self-consistency and the Goldstone check; the absolute energies of
the atom-laden synthetic systems have no published values to compare with.
"""
