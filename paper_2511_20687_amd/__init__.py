"""MI355X-native overlapping-Schwarz / Operator-Inference hot path.

The compute lives in ``libosam.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/osam.h``); :mod:`paper_2511_20687_amd.osam` is the ctypes
binding.  :mod:`paper_2511_20687_amd.inputs` holds the seeded synthetic
workload generators shared by the tests and the benchmark.  Importing this
package loads nothing heavy.
"""
