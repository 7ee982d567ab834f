"""FP64 CPU oracle of the vectorial lattice Boltzmann scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the GPU path: the only common
inputs are the seeded fields of the separate `inputs` package.

Modules
-------
scheme       the scheme of Section 2, written in the paper's notation (numpy FP64)
brute        the same scheme as scalar Python loops with push-style transport,
             for tiny grids
spectrum     linearised amplification matrix E(theta) of Section 4 and the
             closed forms it must satisfy
diagnostics  FP64 definitions of the reduced quantities (mass, momentum,
             kinetic energy, enstrophy, divergence norm, ...)
cnn          plain FP64 convolutional network (forward, backward, Adam) for the
             learned coarse-grid correction
closure      restriction fine -> coarse and the moment correction + guard
"""
