"""MI355X-native CSF lattice Boltzmann step for thermocapillary flow.

The product is ``liblbe_csf.so`` (HIP for gfx950 behind a C ABI, declared in
``include/lbe_csf.h``); ``paper_1412_6238_amd.lbe_csf`` is its thin ctypes
binding and ``paper_1412_6238_amd.workloads`` generates seeded inputs.  This
package file imports neither, so that input generation works without the
library; the binding raises at import if the library has not been built.
"""
__all__ = ["lbe_csf", "workloads"]
