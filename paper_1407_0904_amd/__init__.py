"""MI355X-native finite element local assembly (COFFEE's problem, GPU-first).

The compute path is libcoffee.so (HIP kernels for gfx950 behind a C ABI,
declared in include/coffee.h); `paper_1407_0904_amd.coffee` is its thin
Python binding. `paper_1407_0904_amd.inputs` holds the seeded synthetic
mesh generators.
"""
