"""FP64 CPU oracle for the smoothed-circulant-embedding MLMC level sampler.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct statement of what the GPU path computes, written from the paper
(Istratuca & Teckentrup, "Smoothed Circulant Embedding with Applications
to Multilevel Monte Carlo Methods for PDEs with Random Coefficients").
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The product path (the HIP library and its
Python binding) never imports, links or calls anything in here, and this
package imports nothing from the product path.

All arithmetic is IEEE float64 (NumPy / SciPy).  Library primitives used
as single steps: numpy FFT (the 2-D DFT of Section 2.1.2), scipy's
modified Bessel function K_nu (the Matern formula), scipy's sparse direct
solver (the finite element solve).

Modules
-------
covariance  Matern and separable-exponential covariance (Section 2.1)
embedding   first column of the (padded) embedding, eigenvalues, PSD
            policy, orbit symmetrisation, smoothing mask (Sections 2.1-2.4,
            Algorithm 1 steps 1-3, Algorithm 2)
normals     Philox4x32-10 counter-based generator and a Box-Muller
            transform built only from IEEE +, -, * (bit-reproducible)
field       per-sample Gaussian field and log-normal coefficient
            (Algorithm 1 step 4(a)-(f))
fem         P1 finite elements with nodal quadrature, boundary
            conditions, direct solve (Section 3.1-3.2)
qoi         quantities of interest (Sections 3.1 and 4)
sampler     one MLMC level sample Y = Q_f - Q_c (Sections 3.4-3.5)
mlmc        adaptive MLMC estimator over level samples (Sections 3.3,
            3.5, 4)
qmc         randomly shifted lattice rules for the Hartley xi and the
            multilevel QMC estimator (extension named in Section 5)
smoothing   tau from the balance of smoothing and discretisation error
            (Section 3.5) and the smoothing error Q_h - Q~_h (Section 4.1)

Parity status per function is listed in each module header.
"""

from . import covariance, embedding, normals, field, fem, qoi, sampler, mlmc, qmc, smoothing  # noqa: F401
