"""MI355X (gfx950) implementation of the Dressi rasterization hot path.

Submodules:
  binding  -- ctypes marshalling onto libdressi.so (C ABI in include/dressi.h)
  ops      -- torch.autograd.Functions (rasterize, interpolate, texture, softras)
  scenes   -- seeded synthetic workloads (inputs only)
  build    -- hipcc build of libdressi.so

Importing the package does not load the GPU library; ``binding`` does, and it
raises if libdressi.so has not been built.
"""
