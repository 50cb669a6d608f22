"""MI355X-native dual-stencil FDTD particle-in-cell hot path (arXiv:2004.03754).

The computation lives in the HIP library libyeepic.so (built in-tree by
``paper_2004_03754_amd.build``); ``binding`` is its ctypes front end and
``workloads`` holds the seeded synthetic inputs.
"""
