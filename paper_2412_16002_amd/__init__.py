"""MI355X-native bound-preserving compact-stencil RKDG (cRKDG) hot path.

The compute lives in the HIP library libcrkdg.so (C ABI: include/crkdg.h);
`paper_2412_16002_amd.crkdg` is its ctypes binding and
`paper_2412_16002_amd.inputs` holds the seeded synthetic workloads.  The
binding is imported lazily so that the input generators can be used without
a GPU.
"""

__all__ = ["crkdg", "inputs", "build"]
