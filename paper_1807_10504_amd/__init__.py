"""MI355X-native immersed-boundary projection step (Ong & Miura, irrotational
discrete delta vector). The compute path lives in the HIP library built from
``csrc/``; :mod:`paper_1807_10504_amd.ibproj` is its thin ctypes binding.

Importing the package does not load the library; import ``ibproj`` for that.
"""
__all__ = ["ibproj", "workloads"]
