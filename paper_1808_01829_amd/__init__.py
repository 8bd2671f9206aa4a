"""bms: block multi-shift staggered solver for RHMC on MI355X (gfx950).

Importing the package is cheap: the HIP library is loaded by
`paper_1808_01829_amd.bms` on first use and raises if it is not built.
"""
__all__ = ["inputs"]
