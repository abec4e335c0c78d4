"""MI355X engine for batched scalarised value iteration over agent-task
product MDPs (point-oriented Pareto queries, Robinson & Su).

The compute path is libmorap.so (HIP kernels for gfx950 behind a C ABI,
include/morap.h); ``paper_2305_04397_amd.morap`` is its ctypes binding and is
imported on demand so that building does not need the library.
"""
__all__ = ["morap", "build"]
