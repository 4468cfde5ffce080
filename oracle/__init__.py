"""CPU FP64 oracle for the FFT-VIE / far-field / HOM path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import anything from here.  The product
path (the HIP library and its Python binding) never calls into this package
and shares no code with it; both consume the seeded inputs of ``synth``.

Modules
-------
vie_dense  Dense O(N^2) discrete volume integral equation in the contrast
           current w = chi E (pulse basis, centre collocation), direct matvec
           (full or row-sampled), dense LU solve, textbook BiCGSTAB, far-field
           radiation sum, extinction/scattering cross sections.
mie        Lorenz-Mie series for a homogeneous sphere (Bohren-Huffman
           convention) and its far-field amplitude for any incidence.
hom        Two-photon observables: g2 of two populated channels, coincidence
           number Nc(dtau) and its two normalisations, the beam-splitter model,
           brute-force Fock-space and tau-quadrature checks.
conv_ref   Plain 3-D convolution forward/backward (learned warm start).
detect     Finite-aperture detectors: cone quadrature of the far field.
precond    Block-Jacobi preconditioner on a lateral partition, k-step GMRES
           block solves, restarted flexible GMRES.
selfterm   Exact-cube self term (the voxel's own singular integral).
rooftop    Rooftop basis with pulse testing (eq. Js_expand): face unknowns on
           the staggered grids, surface half-rooftops, dense operator, LU
           solve and far field.

Every function states the passage of the paper it follows.  Functions with
no independent pin say "parity unpinned" in their docstring (none at
present).
"""
