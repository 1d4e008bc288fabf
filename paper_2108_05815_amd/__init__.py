"""MI355X-native Independent algorithm for neutral Moran biodiversity models.

The compute path is the C-ABI HIP library ``libnecsim_hip.so`` (kernels for
gfx950); ``binding`` is its thin ctypes wrapper and ``workloads`` generates
seeded synthetic inputs.  Submodules are imported lazily so that importing the
input generator does not load the GPU library.
"""
__all__ = ["binding", "workloads"]
