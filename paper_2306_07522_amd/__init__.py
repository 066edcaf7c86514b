"""heomx: matrix-free HEOM Liouvillian on MI355X (gfx950), after arXiv 2306.07522.

Importing the package loads nothing; ``paper_2306_07522_amd.api`` loads the
HIP library libheom.so built in-tree (``build_lib.py``) and raises if it is
missing -- there is no CPU fallback.
"""
__all__ = ["api", "workloads"]
