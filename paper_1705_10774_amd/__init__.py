"""MI355X-native local-time-step MHD patch engine (DISPATCH hot path).

The GPU library lives in csrc/ (HIP kernels + C ABI, built into
libdsp.so); `paper_1705_10774_amd.dsp` is its thin ctypes binding and
`paper_1705_10774_amd.inputs` holds the seeded synthetic input generators.
Importing the package itself loads nothing.
"""
