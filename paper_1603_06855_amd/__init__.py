"""MI355X-native mixed-variational phononic band structures with adjoint sensitivities.

The compute path lives in the HIP library ``libphx.so`` (sources under
``csrc/``, C ABI in ``include/phx.h``); ``phx`` is its thin ctypes binding.
Importing this package loads nothing: ``synth`` (seeded inputs) stays usable
without the library.
"""
__all__ = ["phx", "synth", "autograd"]
