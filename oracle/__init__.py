"""Oracle: plain, slow FP64 CPU implementation of the registration hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The product (the HIP library and its Python binding) never imports this
package, and this package imports nothing from the product.

It follows the method of Mang, Gholami, Davatzikos and Biros, "CLAIRE:
A distributed-memory solver for constrained large deformation diffeomorphic
image registration" (arXiv 1808.04487), step by step in the paper's order:

* ``core``   - grid, pseudospectral operators, interpolation, departure
               points, state / adjoint / incremental transport, objective,
               reduced gradient and Gauss-Newton Hessian matvec.
* ``solver`` - preconditioned CG (Algorithm "inner iteration") and the
               inexact Gauss-Newton-Krylov loop with Armijo line search
               (Algorithm "outer iteration").
* ``prep``   - spectral Gaussian smoothing, rescaling and the velocity
               recipe used to turn raw seeded draws into solver inputs.

FP64 throughout.  FFTs are the library primitive ``scipy.fft``; off-grid
interpolation is a small C library (``interp.c``) built with gcc.
"""
