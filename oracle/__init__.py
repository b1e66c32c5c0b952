"""CPU FP64 oracle for banded FEAST spectrum slicing.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
numpy implementation of what the GPU path computes.  It exists to check the
GPU library; it is never part of the product path.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call it.  It shares no code with the GPU library (no kernels,
headers, helpers or tables); the two meet only in the seeded input
generators of the separate ``synth`` module.

Modules (each function names the passage of the paper it follows):

* ``band``       band storage helpers: expansion, band product, 1-norm, Gershgorin
* ``jacobi``     cyclic Jacobi eigensolver for small dense Hermitian matrices
* ``quadrature`` Gauss-Legendre by Golub-Welsch, half-circle contour, filter r(x)
* ``inertia``    Sylvester inertia by band LDL^H without pivoting
* ``bandlu``     band LU with partial pivoting of zI - B, N and H solves
* ``feast``      the FEAST iteration: filter, orthonormalisation, Rayleigh-Ritz,
                 residuals and the slice count check
* ``planner``    slice placement: equal width and equal count by bisection
* ``chebyshev``  stochastic Chebyshev moments with SplitMix64 Rademacher probes
* ``mlp``        the slice-planner MLP forward/backward with BF16 operand rounding

Parity status of each function is stated in its docstring ("pinned by" /
"parity unpinned").
"""
