"""MI355X-native lattice-Boltzmann solver for Maxwell's equations in
heterogeneous media (pseudo-vector lattice BGK of Hanasoge, Succi & Orszag).

The compute path is ``liblbem.so`` (hand-written HIP for gfx950 behind a
C ABI, ``include/lbem.h``); ``paper_1108_2651_amd.lbem`` is its thin ctypes
binding.  Submodules are imported lazily so that the input generators can be
used without loading the GPU library.
"""
__all__ = ["lbem", "inputs"]
