"""ANLS-BPP nonnegative matrix factorisation on one MI355X (gfx950).

The computation lives in libnmf.so (hand-written HIP kernels behind the C-ABI
declared in include/libnmf.h); `binding` is its thin Python binding.
"""
