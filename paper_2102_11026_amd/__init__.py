"""MI355X-native reduced implicit-Euler Newton iteration for deep-autoencoder
subspaces (high-order differentiable autoencoder for nonlinear model reduction).

The compute path is the HIP library ``libnmr.so`` behind the C ABI in
``include/nmr.h``; ``paper_2102_11026_amd.nmr`` is its thin ctypes binding.
``paper_2102_11026_amd.synth`` generates the seeded synthetic problems.
Nothing is imported eagerly so that the generator can be used without the
library.
"""
__all__ = ["synth", "nmr"]
