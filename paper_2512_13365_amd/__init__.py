"""MI355X-native randomized CSE engine for ternary fast-matmul linear forms.

The compute path is the HIP library ``libcse.so`` (kernels for gfx950 behind
a C ABI declared in ``include/cse.h``); ``cse`` is its thin ctypes binding and
``workloads`` draws the seeded synthetic inputs.  Submodules are imported on
demand so that loading the input generator needs no GPU library.
"""
__all__ = ["cse", "workloads"]
