"""Tiny hand-built scenes and cameras for closed-form checks."""
import numpy as np

from paper_2605_30342_amd import scenes
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


def stress_scene(train):
    """Object-scene Gaussians plus the geometry the binning's conservative
    tests and the multi-batch tile lists must handle: large Gaussians that
    cover many tiles, needle-thin ones in random orientations, fully opaque
    (o = 1) and fully transparent (o = 0, still measured) ones, and small
    Gaussians just in front of and just behind the near plane of the
    training cameras (huge footprints, or culled)."""
    rng = np.random.default_rng(7100)

    def quats(n):
        q = rng.standard_normal((n, 4))
        return q / np.linalg.norm(q, axis=1, keepdims=True)
    parts = []
    n = 1500   # object-scene base
    parts.append((rng.uniform(-1, 1, (n, 3)), np.exp(rng.normal(-3.0, 0.5, (n, 3))), quats(n),
                  1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, n)))))
    n = 12     # large, faint
    parts.append((rng.uniform(-0.8, 0.8, (n, 3)), rng.uniform(0.3, 0.8, (n, 3)), quats(n),
                  rng.uniform(0.05, 0.3, n)))
    n = 150    # needles
    sc = np.stack([rng.uniform(0.2, 0.5, n), np.full(n, 0.002), np.full(n, 0.002)], axis=1)
    parts.append((rng.uniform(-1, 1, (n, 3)), sc, quats(n), 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, n)))))
    n = 100    # opaque
    parts.append((rng.uniform(-1, 1, (n, 3)), np.exp(rng.normal(-3.0, 0.5, (n, 3))), quats(n), np.ones(n)))
    n = 50     # transparent but not virtual
    parts.append((rng.uniform(-1, 1, (n, 3)), np.exp(rng.normal(-3.0, 0.5, (n, 3))), quats(n), np.zeros(n)))
    # around the near plane (0.2) of each training camera: depths 0.15 .. 0.3
    # along the view axis, small lateral offsets
    cen = train.centers
    for v in range(train.n):
        fwd = train.R[v, 2].astype(np.float64)
        right = train.R[v, 0].astype(np.float64)
        down = train.R[v, 1].astype(np.float64)
        n = 10
        d = rng.uniform(0.15, 0.3, n)
        m = (cen[v][None] + d[:, None] * fwd[None] + rng.uniform(-0.05, 0.05, (n, 1)) * right[None]
             + rng.uniform(-0.05, 0.05, (n, 1)) * down[None])
        parts.append((m, np.full((n, 3), 0.01), quats(n), rng.uniform(0.1, 0.9, n)))
    cat = [np.concatenate([p[i] for p in parts]).astype(np.float32) for i in range(4)]
    return Scene(cat[0], cat[1], cat[2], cat[3], 0, ((-1, 1), (-1, 1), (-1, 1)))


def translucent_stack():
    """A fog of 4000 faint Gaussians (opacity 0.003) in a 0.4 m cube and two
    training and two candidate views of 96x96 at 30 degrees: long lists in
    which few pixels terminate."""
    rng = np.random.default_rng(7200)
    n = 4000
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = Scene(rng.uniform(-0.2, 0.2, (n, 3)).astype(np.float32), np.full((n, 3), 0.05, np.float32),
               q.astype(np.float32), np.full(n, 0.003, np.float32), 0, ((-1, 1), (-1, 1), (-1, 1)))
    train = scenes.sphere_cameras(2, 7201, width=96, height=96, fov=30.0)
    cand = scenes.sphere_cameras(2, 7202, width=96, height=96, fov=30.0)
    return sc, train, cand
