"""MI355X (gfx950) evaluator of compound linear-algebra expressions.

The compute path is libhexla.so (hand-written HIP kernels behind a C ABI,
declared in include/hexla.h); ``hexla`` is its Python binding.
"""
