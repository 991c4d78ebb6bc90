"""FP64 CPU oracle for the reciprocal incoherent-light average.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path never imports, calls or links it, and it shares no code with the GPU path:
the only module both sides read is ``workloads`` (seeded inputs, no arithmetic).

What it computes (Pestourie, Yao, Kante, Johnson, "Efficient inverse design of
large-area metasurfaces for incoherent light"):

* ``fdfd``     the 2D scalar (TM) frequency-domain operator A with a stretched-
               coordinate PML, the pillar permittivity map, planewave
               equivalent sources b0(theta) and the objective vectors w
               (Sec. "Reciprocal approach": u = A^{-1} b, FOM |w^dag u|^2).
* ``light``    the mean-square amplitude alpha(theta) and the equivalent-current
               cross-correlation C(Delta) (Sec. "Incoherent light", Eq. 3-4 and
               the annulus formula of Sec. "Designs"), and W of a finite
               ensemble of correlated planewaves (Eq. 1 and 3 as sums).
* ``average``  the brute-force angle average of Eq. 6 by Gauss-Legendre
               quadrature over forward solves, the reciprocal average of Eq. 7 by
               a direct O(M^2) double sum (no FFT), and the adjoint gradient of
               Sec. "Reciprocal approach"; the same for any (non-Toeplitz)
               correlation W and several outputs on the same factors, and the
               forward average of Eq. 5 over a finite ensemble of correlated
               planewaves.

* ``fdfd3d``   the 3D vector (Yee) operator with a uniaxial PML, sheet-current
               sources over two incidence angles and both polarisations, and the
               3D reciprocal average with one solve per field component the
               figure of merit reads (Sec. "Concluding remarks").

All arithmetic is float64 / complex128; sparse solves use SciPy's SuperLU.
"""
from . import fdfd, light, average, fdfd3d  # noqa: F401
