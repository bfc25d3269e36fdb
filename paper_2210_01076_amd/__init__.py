"""MI355X-native incremental state-vector simulation (qTask method).

The compute path lives in the HIP/C++ library ``libqtask.so`` behind the C
ABI declared in ``include/qtask.h``; ``paper_2210_01076_amd.qtask`` is its thin
ctypes binding.  Importing this package does not load the library.
"""
__all__ = ["qtask", "workloads"]
