"""MI355X-native differentiable tile-based Gaussian rasterizer (HIP, gfx950).

The compute path lives in the C-ABI library ``libgsmi.so`` built from
``csrc/``; ``gs`` is its thin ctypes binding.  Submodules are imported on use
so that the input generators (``scenes``) load without a GPU.
"""
__all__ = ["gs", "scenes", "autograd", "replay"]
