"""MI355X-native (gfx950) hot path of the lambda-PIC electromagnetic PIC timestep.

Modules:
  lpic        ctypes binding of the C ABI in include/lpic.h (liblpic.so, HIP kernels)
  simulation  torch-tensor harness: boxes, species, hooks and callbacks, ensembles
  workloads   seeded synthetic inputs
  build       in-tree hipcc build of liblpic.so

Importing the package loads nothing; the HIP library is loaded on first use and its
absence is an error (there is no CPU fallback).
"""
__all__ = ["lpic", "simulation", "workloads", "build"]
