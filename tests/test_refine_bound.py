"""The chunk refinement's cull test against the oracle's projection, on the CPU.

gs_lod_refine drops a chunk (a box of Gaussian centres with a largest scale
component) only if every corner of the box is behind the near plane less 1e-6,
or the box is in front of the camera and the projected corners, widened by
3 sqrt((|J|_F^2 s_max^2 + 0.6)(1 + 1e-6)) + 3 pixels with |J|_F^2 taken at the
box's smallest depth through the 1.3 guard band, miss the image.  That test is
restated here from its derivation (not from the kernel), and adversarial
chunks — boxes just outside that margin, Gaussians at the corners with the
largest scale along each axis, boxes across the near plane — are pushed through
the oracle's FP64 projection: every Gaussian of a chunk the test drops must be
one the projection culls.  The GPU tests compare the refined frames with the
unrefined ones; this pins the bound itself.  Planted mistakes that make the
bound unsafe fail it (one sigma instead of three, a margin of -6 pixels instead
of +3, the depth taken four times too far); the bound is about twice the true
radius in these geometries, so milder changes stay safe and pass."""
import math

import numpy as np

import oracle
from paper_2404_01133_amd import synth


def chunk_dropped(lo, hi, smax, cam):
    """The refinement's test for a box [lo, hi] of centres and largest scale smax."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    corners = np.array([[x, y, z] for z in (lo[2], hi[2]) for y in (lo[1], hi[1]) for x in (lo[0], hi[0])])
    pc = corners @ R.T + t
    behind = ~(pc[:, 2] > cam.znear - 1e-6)
    if behind.all():
        return True
    if behind.any():
        return False
    u = cam.fx * (pc[:, 0] / pc[:, 2]) + cam.cx
    v = cam.fy * (pc[:, 1] / pc[:, 2]) + cam.cy
    zmin = pc[:, 2].min()
    limx = 1.3 * (0.5 * cam.width / cam.fx)
    limy = 1.3 * (0.5 * cam.height / cam.fy)
    jf2 = (cam.fx / zmin) ** 2 * (1 + limx ** 2) + (cam.fy / zmin) ** 2 * (1 + limy ** 2)
    rb = 3.0 * math.sqrt((jf2 * smax * smax + 0.6) * (1.0 + 1e-6)) + 3.0
    return bool(u.max() + rb - 0.5 < 0 or u.min() - rb - 0.5 > cam.width - 1 or
                v.max() + rb - 0.5 < 0 or v.min() - rb - 0.5 > cam.height - 1)


def rotation_to(axis_to):
    """Unit quaternion (w, x, y, z) turning the x axis onto `axis_to`."""
    a = np.array([1.0, 0.0, 0.0])
    b = axis_to / np.linalg.norm(axis_to)
    c = np.cross(a, b)
    w = 1.0 + float(a @ b)
    if w < 1e-9:
        return np.array([0.0, 0.0, 1.0, 0.0])
    q = np.array([w, *c])
    return q / np.linalg.norm(q)


def adversarial_chunk(rng, cam):
    """Centres and scales of one chunk placed near the culling margin of `cam`."""
    W, H = cam.width, cam.height
    smax = float(np.exp(rng.uniform(np.log(0.01), np.log(1.5))))
    half = rng.uniform(0.0, 2.0, size=3)
    kind = rng.integers(0, 3)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    if kind == 2:  # across or just behind the near plane, anywhere in x, y
        pcam = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), cam.znear + rng.uniform(-2.5, 0.5)])
    else:  # a box just outside an image edge, by about the margin the test uses
        z = float(np.exp(rng.uniform(np.log(0.5), np.log(80.0))))
        limx = 1.3 * (0.5 * W / cam.fx)
        limy = 1.3 * (0.5 * H / cam.fy)
        jf2 = (cam.fx / z) ** 2 * (1 + limx ** 2) + (cam.fy / z) ** 2 * (1 + limy ** 2)
        margin = 3.0 * math.sqrt(jf2 * smax * smax + 0.6) + 3.0
        spread = 1.5 * max(cam.fx, cam.fy) * float(half.max()) / max(z - 2.0, 0.25)  # the box's own extent
        off = (margin + spread) * rng.uniform(0.7, 1.4)
        side = rng.integers(0, 4)
        u = [-0.5 - off, W - 0.5 + off, rng.uniform(0, W), rng.uniform(0, W)][side]
        v = [rng.uniform(0, H), rng.uniform(0, H), -0.5 - off, H - 0.5 + off][side]
        pcam = np.array([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z])
    centre = R.T @ (pcam - np.asarray(cam.t, np.float64))
    lo, hi = centre - half, centre + half
    corners = np.array([[x, y, zz] for zz in (lo[2], hi[2]) for y in (lo[1], hi[1]) for x in (lo[0], hi[0])])
    inner = lo + (hi - lo) * rng.uniform(size=(8, 3))
    pts = np.concatenate([corners, inner])
    means, scales, quats = [], [], []
    for p in pts:
        # the largest scale along each world axis and each camera axis, plus a round one
        cam_axes = [R.T @ np.eye(3)[k] for k in range(3)]
        for ax in (np.eye(3)[0], np.eye(3)[1], np.eye(3)[2], *cam_axes, None):
            means.append(p)
            if ax is None:
                scales.append([smax, smax, smax])
                quats.append([1.0, 0.0, 0.0, 0.0])
            else:
                scales.append([smax, smax * rng.uniform(0.05, 1.0), smax * rng.uniform(0.05, 1.0)])
                quats.append(rotation_to(ax))
    n = len(means)
    means = np.asarray(means, np.float32).T.copy()
    scales = np.asarray(scales, np.float32).T.copy()
    quats = np.asarray(quats, np.float32).T.copy()
    g = synth.GaussianSet(means, scales, quats, np.ones(n, np.float32), np.zeros((16, 3, n), np.float32))
    return g


def test_chunk_drop_test_never_drops_a_projected_gaussian():
    rng = np.random.default_rng(2404)
    dropped = kept = 0
    for case in range(600):
        W, H = [(1600, 900), (333, 197), (64, 64)][case % 3]
        cam = synth.look_camera(rng.uniform(-50, 50, size=3), rng.uniform(0, 2 * math.pi),
                                rng.uniform(-1.4, 1.4), W, H, fov_x_deg=rng.uniform(30.0, 100.0),
                                znear=float(rng.choice([0.01, 0.2, 1.0])))
        g = adversarial_chunk(rng, cam)
        # the chunk table holds float32 centres and scales, as gs_chunk_bounds writes it
        lo = g.means.min(axis=1).astype(np.float64)
        hi = g.means.max(axis=1).astype(np.float64)
        smax = float(np.abs(g.scales).max())
        visible = oracle.project(g, cam)["visible"]
        if chunk_dropped(lo, hi, smax, cam):
            dropped += 1
            assert not visible.any(), "case %d: a dropped chunk holds a projected Gaussian" % case
        else:
            kept += 1
    # both outcomes are exercised, and often: the boxes sit around the margin
    assert dropped >= 150 and kept >= 150, (dropped, kept)


def test_chunk_drop_test_keeps_visible_chunks_and_is_not_vacuous():
    # a chunk at the image centre is kept; the same chunk far past the margin is dropped
    cam = synth.look_camera((0.0, 0.0, 0.0), 0.0, 0.0, 320, 180)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    ahead = R.T @ np.array([0.0, 0.0, 10.0])
    assert not chunk_dropped(ahead - 0.5, ahead + 0.5, 0.1, cam)
    far_right = R.T @ np.array([40.0, 0.0, 10.0])
    assert chunk_dropped(far_right - 0.5, far_right + 0.5, 0.1, cam)
    behind = R.T @ np.array([0.0, 0.0, -5.0])
    assert chunk_dropped(behind - 0.5, behind + 0.5, 0.1, cam)
    # across the near plane: kept whatever its projection
    near = R.T @ np.array([40.0, 0.0, cam.znear])
    assert not chunk_dropped(near - 0.5, near + 0.5, 0.1, cam)
