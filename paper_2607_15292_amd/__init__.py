"""MI355X-native hot path of the 3D-ACA / H-matrix accelerated Laplace-domain elastodynamic BEM.

The compute path lives in the C-ABI library ``libbem.so`` (HIP for gfx950, built from
``csrc/``); :mod:`paper_2607_15292_amd.binding` marshals arguments to it.  The library is
loaded on first use, not at import, so that the input generators in
:mod:`paper_2607_15292_amd.workloads` can be used without it.
"""
__all__ = ["workloads", "binding"]
