"""MI355X-native FEAST hot path (Polizzi, 'A Density Matrix-based Algorithm for
Solving Eigenvalue Problems').

Importing the package is cheap: the HIP library is loaded lazily by
``paper_0901_2665_amd.feast`` and the seeded input recipes live in
``paper_0901_2665_amd.workloads``.
"""
__all__ = ["feast", "workloads"]
