"""GaBP solver for large-scale SVMs on MI355X (gfx950).

The solver runs as hand-written HIP kernels behind the C ABI declared in
include/gabp_svm.h (library libgabp_svm.so in this package).  The Python
binding is paper_0810_1648_amd.gabp; seeded synthetic inputs live in
paper_0810_1648_amd.inputs.  Importing the package loads nothing.
"""
__all__ = ["gabp", "inputs"]
