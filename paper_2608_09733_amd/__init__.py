"""MI355X-native state-vector engine (hand-written HIP for gfx950).

Importing the package loads nothing native; `paper_2608_09733_amd.sv` loads
the HIP library on first use and raises if it is missing.
"""
__all__ = ["inputs"]
