"""Algorithmic flop counts and MI355X peaks used by the roofline reports.

Flops per rollout-step are counted from the step's formulation by compiling the device
step on the host with a counting number type (csrc/flop_count.cpp): adds, multiplies,
divisions, square roots and transcendental calls count 1 each; the work repeated by
every lane of a quad (base rotation, the 6x6 solves, integration) is counted once; a
4-way quad sum counts 3 adds.  The representative state has two feet in ground contact
(and, in the pushing scene, the box resting on four corners).
"""

FLOPS_DYN_PER_STEP = {0: 6838, 1: 7222, 2: 6910, 3: 9092}   # by scene
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}                  # MI355X vector peaks
HBM_TBPS = 8.0


def flops_per_rollout_step(scene: int, nk: int) -> int:
    """Dynamics + spline interpolation (3 joints x nk x 2 per lane, 4 lanes) + cost."""
    return FLOPS_DYN_PER_STEP[scene] + 24 * nk + 17
