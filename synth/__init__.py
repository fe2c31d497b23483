"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This package only *generates inputs*: unit cells, atom positions, the
pseudopotential-like system definition (Gaussian local wells and Gaussian
Kleinman-Bylander projectors with a time-reversal-invariant spin-orbit D
matrix), plane-wave spheres, k/q point sets, random response vectors and,
for the large benchmark shapes, a synthetic occupied manifold.  None of the
Liouville-Lanczos arithmetic (densities, kernels, Liouvillian, Lanczos,
susceptibility) lives here, and nothing here imports the oracle or the GPU
package.
"""
from .systems import *  # noqa: F401,F403
