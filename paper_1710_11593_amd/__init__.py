"""fracsolve: MI355X-native divide-and-conquer solver for the L1 time-stepping
system of Caputo time-fractional diffusion and diffusion-wave equations.

The solver itself is the HIP library ``csrc/libfracsolve.so`` behind the C ABI
in ``include/fracsolve.h``; ``binding`` marshals arguments to it.  Importing
this package does not load the library; ``binding.lib()`` does, and raises if
the library is missing.
"""
__all__ = ["binding", "workloads"]
