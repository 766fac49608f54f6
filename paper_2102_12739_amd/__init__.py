"""MI355X-native 3D degridding (hand-written HIP for gfx950 behind a C ABI).

Submodules:
  workload  seeded synthetic inputs (tables, coordinates, subgrid stacks)
  degrid    the Python binding of the C-ABI library and its autograd wrapper

Importing the package loads nothing; ``paper_2102_12739_amd.degrid`` loads the
HIP library on first use and raises if it has not been built.
"""
