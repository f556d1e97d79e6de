"""libtdse: MI355X-native FDTD integration of the 3D time-dependent
Schrodinger equation (arXiv 2401.07416), with a C-ABI HIP library underneath.

Importing the package loads nothing native; ``paper_2401_07416_amd.tdse``
loads ``libtdse.so`` and raises if it is missing.
"""
__all__ = ["tdse", "workloads"]
