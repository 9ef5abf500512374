"""MI355X (gfx950) library for the two-level Strang splitting of the 2D/3D spatial
fractional Allen-Cahn equation: a C-ABI shared library of HIP kernels (libsfac.so) and a
thin ctypes binding (`sfac`). Importing the package does not load the library; the first
call into `sfac` does, and raises if it has not been built."""

__all__ = ["sfac", "workloads"]
