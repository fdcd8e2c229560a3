"""MI355X-native reconstruction of single-photon lidar data with plug-and-play
point-cloud denoisers (Tachella et al.).

The compute path lives in the HIP library ``librt3d.so`` (``csrc/``) behind the
C ABI declared in ``include/rt3d.h``; ``paper_1905_06700_amd.rt3d`` is its
ctypes binding.  ``synth`` generates seeded synthetic scenes.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["rt3d", "synth"]
