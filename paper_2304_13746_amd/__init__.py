"""MI355X-native ideal-MHD box update (Godunov finite volume, Lesur et al. 2023,
arXiv:2304.13746) behind the C ABI of include/mhd.h.

Importing the package loads nothing; ``paper_2304_13746_amd.box.MHDBox`` loads
libmhd.so and raises if it has not been built.
"""
__all__ = ["inputs", "box", "build"]
