"""MI355X-native ADER-CG time step for 3D Euler flows on periodic meshes.

The hot path lives in ``libader_hip.so`` (HIP kernels for gfx950 behind the
C ABI declared in ``include/ader.h``); ``paper_1006_2146_amd.ader`` is a thin
ctypes binding with the same names.  Importing this package loads nothing;
``paper_1006_2146_amd.ader.load()`` loads the library and raises if it is
missing.
"""
