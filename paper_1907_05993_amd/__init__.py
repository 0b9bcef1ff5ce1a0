"""MI355X-native demons-based HR-EBSD remapping (arXiv:1907.05993).

The HIP library is loaded lazily by :mod:`paper_1907_05993_amd.ebsd` on first
use; importing the package itself loads nothing native.
"""
__all__ = ["ebsd", "synth"]
