"""2D cross-sections of infinitely long catalytic fibres (paper Sec. "System
geometry" and Sec. "Membrane generation"): a channel with solid wall rows, discs
rasterised on the lattice, and their surface nodes marked catalytic.

Node types: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B), 3 catalyst type 2
(B->C).  Arrays are ``[ny, nx]`` with x fastest.
"""
from __future__ import annotations

import numpy as np

FLUID, SOLID, CAT1, CAT2 = 0, 1, 2, 3


def channel(nx: int, ny: int) -> np.ndarray:
    """Empty channel: rows 0 and ny-1 are solid walls, the rest fluid."""
    t = np.zeros((ny, nx), dtype=np.uint8)
    t[0, :] = SOLID
    t[-1, :] = SOLID
    return t


def disc_offsets(r: int):
    """Integer offsets (dx, dy) with dx^2 + dy^2 <= r^2."""
    d = np.arange(-r, r + 1)
    dx, dy = np.meshgrid(d, d, indexing="xy")
    m = dx * dx + dy * dy <= r * r
    return dx[m], dy[m]


def rasterize(node_type: np.ndarray, centres, r: int) -> np.ndarray:
    """Mark every node of each disc solid; returns an int32 map of the fibre
    index owning each node (-1 elsewhere)."""
    ny, nx = node_type.shape
    owner = np.full((ny, nx), -1, dtype=np.int32)
    dx, dy = disc_offsets(r)
    for f, (cx, cy) in enumerate(centres):
        xs, ys = cx + dx, cy + dy
        ok = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny)
        node_type[ys[ok], xs[ok]] = SOLID
        owner[ys[ok], xs[ok]] = f
    return owner


def classify_surface(node_type: np.ndarray, owner: np.ndarray) -> np.ndarray:
    """Boolean map of fibre nodes with at least one fluid node among their four
    lattice neighbours (E, N, W, S) -- the catalytic surface."""
    ny, nx = node_type.shape
    fluid = node_type == FLUID
    nb = np.zeros_like(fluid)
    nb[:, :-1] |= fluid[:, 1:]
    nb[:, 1:] |= fluid[:, :-1]
    nb[:-1, :] |= fluid[1:, :]
    nb[1:, :] |= fluid[:-1, :]
    return (owner >= 0) & nb


def surface_counts(r: int) -> int:
    """Number of surface nodes of one isolated disc of radius r."""
    n = 2 * r + 7
    t = np.zeros((n, n), dtype=np.uint8)
    owner = rasterize(t, [(n // 2, n // 2)], r)
    return int(classify_surface(t, owner).sum())


def place_discs(rng: np.random.Generator, count: int, r: int, band, ny: int, gap: int,
                existing=(), max_tries: int = 100000):
    """Random sequential placement of ``count`` discs with integer centres.

    Centre x in [x0 + r, x1 - r] (the disc lies inside the band), centre y in
    [r + gap + 1, ny - 2 - r - gap] (``gap`` fluid rows from the walls), and
    centre distance >= 2r + gap + 1 from every disc already placed (including
    ``existing``), so at least ``gap`` fluid nodes separate two discs along any
    axis.  Overlapping draws are discarded, as in the paper's generator.
    """
    x0, x1 = band
    lo_x, hi_x = x0 + r, x1 - r
    lo_y, hi_y = r + gap + 1, ny - 2 - r - gap
    if hi_x < lo_x or hi_y < lo_y:
        raise ValueError("band too small for the disc radius")
    placed = list(existing)
    out = []
    dmin2 = (2 * r + gap + 1) ** 2
    for _ in range(count):
        for _try in range(max_tries):
            cx = int(rng.integers(lo_x, hi_x + 1))
            cy = int(rng.integers(lo_y, hi_y + 1))
            if all((cx - px) ** 2 + (cy - py) ** 2 >= dmin2 for px, py in placed):
                placed.append((cx, cy))
                out.append((cx, cy))
                break
        else:
            raise RuntimeError("disc placement failed: band too crowded")
    return out
