"""MI355X (gfx950) implementation of the CHR hot path of arXiv 2408.05462.

Compressed Hierarchical Representation with topology preservation for 3D
float32 fields, reconstruction at any level, and marching cubes, as a C-ABI
HIP library (``libchr.so``, declared in ``include/chr.h``) with a thin torch
binding in ``api``.  Importing the package does not load the library; the
first call into ``api`` does, and raises if it has not been built.
"""
__all__ = ["api", "inputs", "build"]
