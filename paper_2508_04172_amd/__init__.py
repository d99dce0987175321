"""MI355X-native meshfree RBF likelihood (arXiv:2508.04172).

The compute path lives in the HIP library ``librbfl.so`` (see ``include/rbfl.h``);
``rbfl`` is a thin ctypes binding to it and ``workloads`` holds seeded inputs.
"""
