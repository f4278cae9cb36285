"""Default seeds and output biases of the synthetic networks.

The output bias of the regression nets puts the raw output in the range of the
puzzle's distances, so that floor(y) sometimes exceeds and sometimes undercuts
the Manhattan distance (both branches of min(floor(y), MD) are exercised).
"""
DEFAULTS = {
    "stp3_small": dict(seed=11, head_bias=14.0),
    "stp4_res": dict(seed=22, head_bias=40.0),
    "rc_cls": dict(seed=33, head_bias=0.0),
}
