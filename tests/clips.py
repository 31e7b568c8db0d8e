"""YCoCg planes of the synthetic clips for the transform tests.

The frames come from the seeded generator; the colour conversion is the
oracle's (Table I, equations (1)-(3)), so no test input passes through the
library under test.
"""
import numpy as np

from oracle import color
from paper_1510_00561_amd import synth


def clip_planes(n_frames, height, width, workload):
    """[n_frames * 3, height, width] float32: Y, Co, Cg of each frame in turn."""
    out = []
    for frame in synth.clip_rgb(n_frames, height, width, workload):
        out.extend(color.rgb_to_ycocg(frame))
    return np.stack(out).astype(np.float32)
