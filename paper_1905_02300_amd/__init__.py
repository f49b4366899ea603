"""MI355X-native Yin-Yang artificial-compressibility direction-splitting
step (Takhirov, Frolov & Minev, arXiv 1905.02300).

The compute path is the HIP library libyy.so (C-ABI in include/yy.h);
paper_1905_02300_amd.yy is its thin ctypes binding.
"""
