"""CPU FP64 oracle of one PSATD step with guard cells -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library never does, and it never imports the
library.  It shares no code with the HIP path: the only common dependency is
the seeded input generator package ``synth``.

Contents (each function cites the passage of Kallala, Vay & Vincenti,
"A generalized massively parallel ultra-high order FFT-based Maxwell solver",
arXiv:1812.07357, that it follows):

* ``kspace``      wavenumbers, order-p modified wavenumbers, PSATD coefficients
                  and the analytic k-space push (Sec. 1.1 and 1.3 state the
                  properties; the equations are derived from Maxwell's
                  equations in Fourier space with J constant over the step).
* ``step``        forward FFT -> push -> inverse FFT of one periodic box.
* ``domain``      guard fill / merge between the G1 grid and the FFT boxes
                  (Sec. 2.5.2) and the local-with-guards driver (Fig. 1(a)).
* ``diagnostics`` Gauss residual, div B, field energy, relative L2.
* ``modes``       exact output of the step for inputs made of a few grid
                  modes, usable at any grid size.
* ``mlp``         FP64 reference of the guard-width surrogate network.

Precision is FP64 throughout.  The FFT is a library primitive (complex C2C
from scipy/numpy); it is pinned by a naive DFT in the tests.
"""
