"""MI355X-native BHEM thin-shell hot path (arXiv 2312.14839).

The compute path is the HIP library ``libbhem.so`` behind the C ABI declared
in ``include/bhem_shell.h``; ``paper_2312_14839_amd.shell`` is its ctypes
binding and ``paper_2312_14839_amd.workloads`` builds seeded synthetic inputs.
Importing the package itself loads nothing.
"""
__all__ = ["shell", "workloads"]
