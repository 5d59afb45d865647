"""Whole-body MPPI for a quadruped on MI355X (gfx950): HIP kernels behind a C ABI."""
