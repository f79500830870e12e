"""MI355X (gfx950) energy and force evaluation of an Allegro-style neural-network
interatomic potential, behind a C ABI (include/nnqmd.h).

`paper_2303_08169_amd.binding` loads the HIP library (libnnqmd.so, built in-tree
by `paper_2303_08169_amd.build`); `paper_2303_08169_amd.potential` wraps it for
PyTorch tensors. Importing this package does not load the library.
"""

__all__ = ["binding", "potential", "build"]
