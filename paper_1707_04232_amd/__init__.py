"""MI355X-native SDPD with the Metropolized fluctuation/dissipation scheme.

The compute path is the HIP library ``libsdpd.so`` behind the C ABI declared in
``include/sdpd.h``; :mod:`paper_1707_04232_amd.sdpd` is its thin ctypes
binding.  The binding is imported lazily so that the synthetic-input module
can be used without the GPU library.
"""
__all__ = ["sdpd", "workload"]
