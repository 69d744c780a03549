"""MI355X-native residual of the unstructured-mesh finite-difference Euler solver
(Zhen, Qu, Cai: "A Novel Finite Difference Method for Euler Equations in 2D
Unstructured Meshes").

Importing the package loads nothing native.  ``paper_2102_12933_amd.inputs`` holds
the seeded workload generators (meshes, initial states); the HIP library is loaded
on first use of ``paper_2102_12933_amd.fdu`` (the ctypes binding), which raises if
the shared library has not been built.
"""

__all__ = ["inputs"]
