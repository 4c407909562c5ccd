"""Batched Whittaker-Henderson smoother for MI355X (gfx950).

``paper_2604_00048_amd.whs`` binds the HIP library ``libwhs.so`` (built by
``paper_2604_00048_amd.build``); ``paper_2604_00048_amd.synth`` draws the
seeded synthetic workloads.  Importing the package loads nothing.
"""

__all__ = ["whs", "synth", "build"]
