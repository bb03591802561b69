"""MI355X-native dust-in-ion-flow hot path (arXiv 2205.06557, "OpenDust").

The compute lives in ``libodust.so`` (HIP kernels for gfx950 behind a C-ABI,
declared in ``include/odust.h``).  ``paper_2205_06557_amd.binding`` marshals
arguments to it with ctypes; ``workloads`` describes synthetic inputs.
"""
