"""MI355X-native unsplit MUSCL-Hancock Godunov step for ghost-zoned AMR patches.

The compute path is a C-ABI HIP library (``libgodunov.so``, built for gfx950);
``paper_1412_0934_amd.godunov`` is its thin Python binding. Importing the
package itself loads nothing.
"""
__all__ = ["godunov", "inputs"]
