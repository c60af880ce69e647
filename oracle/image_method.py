"""Image-source paths in an axis-aligned box room (closed form; test infrastructure).

The image method is the classical way to turn a reflection sequence into an
exact path (paper, Introduction and Section 2.3): mirror the TX across the
reflecting planes in order, draw the straight line from the last image to
the RX, and walk it back through the planes.  The sequence is a valid path
iff every walked-back intersection lies on its face (inside the room's face
rectangle) and the order of the intersections along the path matches the
sequence.

This module is independent of the brute-force launcher in ``oracle.c``: it
never traces a ray against points, so it can pin that launcher on box rooms.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# face id -> (axis, coordinate is the low (0) or the high (1) end)
_FACES = {0: (2, 0), 1: (2, 1), 2: (0, 0), 3: (0, 1), 4: (1, 0), 5: (1, 1)}


def _plane(face, size):
    axis, hi = _FACES[face]
    return axis, (size[axis] if hi else 0.0)


def _mirror(p, face, size):
    axis, c = _plane(face, size)
    q = np.array(p, dtype=np.float64)
    q[axis] = 2.0 * c - q[axis]
    return q


def image_path(seq, tx, rx, size, tol=1e-9):
    """Exact path for the reflection sequence ``seq`` (face ids) or None.

    Returns (length, [interaction points]) when the sequence is realisable.
    """
    tx = np.asarray(tx, np.float64)
    rx = np.asarray(rx, np.float64)
    images = [tx]
    for f in seq:
        images.append(_mirror(images[-1], f, size))
    pts = []
    target = rx
    for k in range(len(seq) - 1, -1, -1):
        f = seq[k]
        axis, c = _plane(f, size)
        src = images[k + 1]
        denom = target[axis] - src[axis]
        if abs(denom) < 1e-15:
            return None
        lam = (c - src[axis]) / denom
        if not (tol < lam < 1.0 - tol):
            return None
        q = src + lam * (target - src)
        for ax in range(3):
            if ax != axis and not (-tol <= q[ax] <= size[ax] + tol):
                return None
        pts.append(q)
        target = q
    pts = pts[::-1]
    # the straight segments must stay inside the room (they do whenever every
    # walked-back point lies on its face of a convex room)
    length = float(np.linalg.norm(images[-1] - rx))
    return length, pts


def box_room_paths(tx, rx, size=(10.0, 8.0, 3.0), max_reflections=2):
    """All realisable reflection sequences with at most ``max_reflections`` bounces.

    Consecutive repeats of a face are impossible (a plane cannot reflect into
    itself).  Returns {sequence tuple: (length, points)}.
    """
    out = {}
    for k in range(max_reflections + 1):
        for seq in itertools.product(range(6), repeat=k):
            if any(seq[i] == seq[i + 1] for i in range(len(seq) - 1)):
                continue
            r = image_path(seq, tx, rx, size)
            if r is not None:
                out[tuple(seq)] = r
    return out


def lattice_edge_clearance(seq, tx, rx, size):
    """Smallest distance from the walked-back interaction points to a face edge."""
    r = image_path(seq, tx, rx, size)
    if r is None:
        return math.nan
    best = math.inf
    for q, f in zip(r[1], seq):
        axis, _ = _FACES[f]
        for ax in range(3):
            if ax != axis:
                best = min(best, q[ax], size[ax] - q[ax])
    return best
