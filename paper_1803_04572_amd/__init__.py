"""COPA (constrained PARAFAC2 fitted by AO-ADMM) on AMD MI355X.

The fitting path runs in hand-written HIP kernels (gfx950) behind a C ABI (``libcopa.so``);
``paper_1803_04572_amd.copa`` is the thin Python binding. ``synth`` draws seeded inputs.
"""
