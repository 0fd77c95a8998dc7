"""Tiny hand-built scenes and cameras for closed-form checks."""
import numpy as np

from paper_2605_30342_amd.scenes import Cameras, Scene


def axis_camera(width=1, height=1, f=100.0, center=(0.0, 0.0, 0.0)):
    """Camera at `center` looking along world +z with axes x right, y down."""
    R = np.eye(3, dtype=np.float32)
    t = (-np.asarray(center, dtype=np.float64)).astype(np.float32)
    K = np.array([[f, f, width / 2.0, height / 2.0]], dtype=np.float32)
    return Cameras(R[None], t[None], K, np.array([[width, height]], dtype=np.int32))


def stack_scene(zs, opac, scale=0.05, x=0.0, y=0.0):
    n = len(zs)
    means = np.stack([np.full(n, x), np.full(n, y), np.asarray(zs, dtype=np.float64)], 1)
    return Scene(means.astype(np.float32), np.full((n, 3), scale, np.float32),
                 np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
                 np.asarray(opac, dtype=np.float32))
