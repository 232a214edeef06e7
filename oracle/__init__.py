"""FP64 CPU oracle for extended diffraction tomography -- TEST INFRASTRUCTURE.

This package is a plain, slow, obviously-correct NumPy/SciPy statement of what
the GPU library computes.  It exists only to check that library: the only
callers allowed are the test-suite, the smoke check and the CPU-baseline leg
of the benchmark.  The product path never imports, calls or links anything
here, and this package never imports the product package; the two share only
the seeded input generator ``edt_inputs`` (geometry and random draws, no
arithmetic of the method).

Modules
-------
green   reference Green's function g(z; |k|, w) of the 1D layered medium by a
        generalised reflection/transmission recursion, with forward-mode
        (tangent) derivatives with respect to the layer velocities.
rows    the decoupled 1D problems: wavenumber bookkeeping, the evanescent
        cut, the +/-k_m pairing and the Born rows A = w^2 dz g(k_r) g(k_s).
solve   the normal equations with relative Tikhonov damping, the
        real/imaginary split and the recombination into V~(k_m, z).
grad    gradient of a model misfit with respect to data, damping and layer
        velocities (adjoint of the normal equations + tangent-mode G0).
born    brute-force space-domain Born data on tiny periodic grids.
tsvd    the paper's own solver: truncated SVD of each pair's system (through
        the eigen-decomposition of its Gram), with a relative tolerance.
kz      the restriction of the solution to a disk in (k_m, k_z): the truncated
        SVD of each pair's system on the kept discrete Fourier modes in depth.
aperture  finite aperture on the 2D line: the offset window as a discrete sinc
        over the receiver index, the windowed Gram Re(A^H S A) and its solve.
shots   the transforms on either side: 2D shot records to the packed rows, and
        the solution spectrum V~ to the model V(x, z).
lines3d the 3D survey of parallel 2D lines (Section 2.2): rows that sum, over
        the line wavenumbers, products of Green's functions of 2D horizontal
        wavevectors (the decoupled 3D equation's k_h'' integral), per (k_m, k_y).

Every function is pinned by a test in ``tests/test_oracle_*.py`` against a
closed form, an invariant, a library routine that solves the same problem a
different way, or brute force.
"""
