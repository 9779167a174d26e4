"""MI355X-native alternating-minimisation multi-agent trajectory optimiser.

The compute path lives in ``libmato.so`` (HIP for gfx950, C ABI declared in
``include/mato.h``); ``paper_2011_04240_amd.mato`` is its ctypes binding and
``paper_2011_04240_amd.scenarios`` the seeded input generators.  Importing the
package itself loads nothing.
"""
