"""MI355X-native HSGD (Hierarchical Sparse Gradient Descent) MPI refinement.

Submodules load lazily: ``scenes`` is pure NumPy input generation; ``hsgd`` (the ctypes
binding over the HIP library) is imported on first use.
"""

__all__ = ["scenes", "hsgd"]
