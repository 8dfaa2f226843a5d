"""MI355X (gfx950) modified-Ehrenfest propagation library.

The compute path is libmodehr.so (HIP kernels behind the C ABI declared in
include/modehr.h); ``binding`` marshals arguments to it from Python with
torch tensors for device memory.  Importing this package does not load the
library; ``binding.load()`` (called by ``binding.System``) does, and raises
if it is missing.
"""
__all__ = ["binding"]
