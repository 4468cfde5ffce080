"""MI355X-native FFT-accelerated volume-integral-equation solver, far-field
projection and two-photon (HOM) observables for lossless dielectric bodies.

The compute path is ``libvie.so`` (hand-written HIP kernels for gfx950 behind
the C ABI of ``include/vie.h``); ``paper_2508_16471_amd.vie`` is its thin
ctypes binding.  Importing this package does not load the library; the
first call into ``vie`` does, and fails loudly if it has not been built.
"""

__all__ = ["vie"]
