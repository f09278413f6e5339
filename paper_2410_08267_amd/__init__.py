"""MI355X-native backward N-1-body relic profiles (arXiv:2410.08267).

The compute path is the C-ABI library ``libnuhalo.so`` (HIP kernels for gfx950);
``paper_2410_08267_amd.nuhalo`` is its thin ctypes binding.  ``request`` and
``workloads`` hold no arithmetic of the method and import without a GPU.
"""
from .request import Request  # noqa: F401

__all__ = ["Request"]
