"""MI355X-native density-matrix superoperator engine (TANQ-Sim method, arXiv 2404.13184).

``workloads`` holds the seeded input generators.  The HIP library ``libtanq.so`` and its
ctypes binding are in :mod:`paper_2404_13184_amd.tanq`; importing this package does not
load them.
"""
__all__ = ["workloads", "tanq"]
