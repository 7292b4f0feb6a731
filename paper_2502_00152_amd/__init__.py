"""HISQ even-odd CG with low-mode deflation on MI355X (gfx950).

The GPU library and its binding live in `paper_2502_00152_amd.hisq`; importing
this package does not load it, so `paper_2502_00152_amd.inputs` can be used on
machines without a GPU.
"""
