"""Vessel-like phantoms: Gaussian-profile line segments and branching trees.

Pixel value = max over segments of a * exp(-d^2 / (2 sigma^2)), d being the
distance (in pixels) from the pixel centre to the segment.  Works for 2D
images [ny][nx] and 3D volumes [nz][ny][nx].
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np


def _rasterize(shape, segs):
    """segs: list of (p0, p1, sigma, amp) in pixel coordinates ordered (x, y[, z])."""
    nd = len(shape)
    img = np.zeros(shape, dtype=np.float64)
    dims = shape[::-1]  # (nx, ny[, nz])
    for p0, p1, sig, amp in segs:
        p0 = np.asarray(p0, dtype=np.float64)
        p1 = np.asarray(p1, dtype=np.float64)
        m = 3.5 * sig
        lo = np.maximum(np.floor(np.minimum(p0, p1) - m).astype(int), 0)
        hi = np.minimum(np.ceil(np.maximum(p0, p1) + m).astype(int) + 1, np.asarray(dims))
        if np.any(hi <= lo):
            continue
        axes = [np.arange(lo[a], hi[a], dtype=np.float64) for a in range(nd)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # grids[a] has shape of box, axis a coord
        d = p1 - p0
        dd = float(d @ d)
        rel = [grids[a] - p0[a] for a in range(nd)]
        if dd > 0:
            t = sum(rel[a] * d[a] for a in range(nd)) / dd
            t = np.clip(t, 0.0, 1.0)
        else:
            t = 0.0
        dist2 = sum((rel[a] - t * d[a]) ** 2 for a in range(nd))
        val = amp * np.exp(-dist2 / (2.0 * sig * sig))
        sl = tuple(slice(lo[a], hi[a]) for a in range(nd))[::-1]
        np.maximum(img[sl], val, out=img[sl])
    return img


def segment_phantom(shape, n_segments, seed, sigma_px=(1.0, 3.0), amp=(0.3, 1.0)):
    """Random straight segments with endpoints uniform in a disk/ball of radius 0.8*half-width."""
    rng = np.random.default_rng(seed)
    nd = len(shape)
    dims = np.asarray(shape[::-1], dtype=np.float64)
    ctr = (dims - 1.0) / 2.0
    rad = 0.8 * 0.5 * float(np.min(dims[: max(nd, 2)] if nd == 2 else dims))
    segs = []
    for _ in range(n_segments):
        pts = []
        for _e in range(2):
            while True:
                u = rng.uniform(-1.0, 1.0, size=nd)
                if u @ u <= 1.0:
                    break
            pts.append(ctr + rad * u)
        sig = rng.uniform(*sigma_px)
        a = rng.uniform(*amp)
        segs.append((pts[0], pts[1], sig, a))
    return _rasterize(shape, segs)


def _rotate2(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1]])


def _branch3(v, ang, rng):
    """Rotate unit vector v by angle ang towards a random azimuth around v."""
    v = v / np.linalg.norm(v)
    a = np.array([1.0, 0.0, 0.0]) if abs(v[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(v, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(v, e1)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    perp = math.cos(phi) * e1 + math.sin(phi) * e2
    return math.cos(ang) * v + math.sin(ang) * perp


def vessel_tree(shape, n_segments, seed, sigma0=3.0, amp=(0.3, 1.0)):
    """Branching tree grown breadth-first until n_segments segments exist.

    Root: random point on a circle/sphere of radius 0.7*half-width pointing to
    the centre, length 0.25*width, sigma0 px.  Each segment spawns two
    children at +-U[20,45] degrees (3D: random azimuth), length x U[0.6,0.85],
    sigma x 0.85 clamped at >= 1 px, amplitude U[amp].  End points are pulled
    back inside the ball of radius 0.9*half-width.
    """
    rng = np.random.default_rng(seed)
    nd = len(shape)
    dims = np.asarray(shape[::-1], dtype=np.float64)
    ctr = (dims - 1.0) / 2.0
    half = 0.5 * float(np.min(dims))
    lim = 0.9 * half

    def clip(p):
        r = p - ctr
        n = float(np.linalg.norm(r))
        return p if n <= lim else ctr + r * (lim / n)

    segs = []
    roots = 0
    queue = deque()
    while len(segs) < n_segments:
        if not queue:
            # (re)seed a root
            if nd == 2:
                ang = rng.uniform(0.0, 2.0 * math.pi)
                u = np.array([math.cos(ang), math.sin(ang)])
            else:
                u = rng.normal(size=3)
                u /= np.linalg.norm(u)
            start = ctr + 0.7 * half * u
            direction = -u
            length = 0.25 * 2.0 * half
            queue.append((start, direction, length, sigma0))
            roots += 1
        start, direction, length, sig = queue.popleft()
        end = clip(start + direction * length)
        segs.append((start, end, max(sig, 1.0), rng.uniform(*amp)))
        for sign in (-1.0, 1.0):
            ang = math.radians(rng.uniform(20.0, 45.0))
            if nd == 2:
                nd_dir = _rotate2(direction, sign * ang)
            else:
                nd_dir = _branch3(direction, ang, rng)
            queue.append((end, nd_dir / np.linalg.norm(nd_dir), length * rng.uniform(0.6, 0.85),
                          max(sig * 0.85, 1.0)))
    return _rasterize(shape, segs[:n_segments])
