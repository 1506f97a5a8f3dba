"""3D membranes of randomly oriented, capped cylindrical fibres (paper Sec.
"System geometry: Cascade reaction" and Sec. "Membrane generation").

The box is periodic in y and z (the flow is periodic in every direction; the
ADR has its inlet at x = 0 and outlet at x = nx-1), so a fibre is rasterised
with the minimum-image distance in y and z.  Each fibre is a solid cylinder of
radius r and length ``length`` closed by flat caps, with its axis drawn
uniformly on the unit sphere and its centre uniformly in the membrane band;
draws whose voxels leave the band in x or come within ``gap`` voxels of an
earlier fibre are discarded, as in the paper's generator.

Node types: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B), 3 catalyst type
2 (B->C).  Arrays are ``[nz, ny, nx]`` with x fastest.
"""
from __future__ import annotations

import numpy as np

FLUID, SOLID, CAT1, CAT2 = 0, 1, 2, 3


def _unit_vector(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def cylinder_voxels(shape, centre, axis, r, length):
    """(z, y, x) index arrays of the voxels of one capped cylinder, with y and
    z wrapped (minimum image); x is not wrapped and may fall outside."""
    nz, ny, nx = shape
    h = int(np.ceil(0.5 * length + r)) + 1
    cx, cy, cz = centre
    ox, oy, oz = np.meshgrid(np.arange(-h, h + 1), np.arange(-h, h + 1), np.arange(-h, h + 1),
                             indexing="ij")
    X = np.floor(cx).astype(int) + ox
    Y = np.floor(cy).astype(int) + oy
    Z = np.floor(cz).astype(int) + oz
    d = np.stack([X - cx, Y - cy, Z - cz], axis=-1).astype(np.float64)
    t = d @ axis
    radial = np.linalg.norm(d - t[..., None] * axis, axis=-1)
    inside = (np.abs(t) <= 0.5 * length) & (radial <= r)
    return Z[inside] % nz, Y[inside] % ny, X[inside], d[inside]


def place_cylinders(rng, shape, count, r, length, band, gap=2, solid=None, max_tries=100000):
    """Place ``count`` fibres in the band x in [band[0], band[1]).  Returns
    (solid mask, list of (centre, axis)) with the new fibres added to
    ``solid`` (a bool array or None)."""
    nz, ny, nx = shape
    solid = np.zeros(shape, dtype=bool) if solid is None else solid.copy()
    fibres = []
    tries = 0
    while len(fibres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place the fibres without overlap")
        centre = np.array([rng.uniform(band[0], band[1]), rng.uniform(0, ny), rng.uniform(0, nz)])
        axis = _unit_vector(rng)
        z, y, x, _ = cylinder_voxels(shape, centre, axis, r, length)
        if x.size == 0 or x.min() < band[0] or x.max() >= band[1]:
            continue
        # overlap test on the fibre grown by gap voxels (radius and caps)
        zg, yg, xg, _ = cylinder_voxels(shape, centre, axis, r + gap, length + 2 * gap)
        ok = (xg >= 0) & (xg < nx)
        if solid[zg[ok], yg[ok], xg[ok]].any():
            continue
        solid[z, y, x] = True
        fibres.append((centre, axis))
    return solid, fibres


def classify_surface(solid):
    """Solid voxels with a fluid voxel among their 6 neighbours (periodic in
    y and z, not in x) -- the catalytic surface."""
    fluid = ~solid
    nb = np.zeros_like(fluid)
    nb[:, :, :-1] |= fluid[:, :, 1:]
    nb[:, :, 1:] |= fluid[:, :, :-1]
    nb |= np.roll(fluid, 1, axis=1) | np.roll(fluid, -1, axis=1)
    nb |= np.roll(fluid, 1, axis=0) | np.roll(fluid, -1, axis=0)
    return solid & nb


def membrane(shape, bands, counts, kinds, r, length, seed, gap=2):
    """Fibres of band j carry catalyst kinds[j] on their whole surface."""
    rng = np.random.default_rng(seed)
    solid = None
    owner_kind = np.zeros(shape, dtype=np.uint8)
    for band, cnt, kind in zip(bands, counts, kinds):
        before = np.zeros(shape, dtype=bool) if solid is None else solid
        solid, _ = place_cylinders(rng, shape, cnt, r, length, band, gap, solid)
        owner_kind[solid & ~before] = kind
    t = np.where(solid, SOLID, FLUID).astype(np.uint8)
    surf = classify_surface(solid)
    t[surf] = owner_kind[surf]
    return t


def side_by_side_membrane(shape, band, count, r, length, seed, gap=2):
    """Every fibre carries catalyst 1 on one side of a plane through its axis
    and catalyst 2 on the other; the plane's normal is drawn uniformly among
    the directions perpendicular to the axis."""
    rng = np.random.default_rng(seed)
    solid, fibres = place_cylinders(rng, shape, count, r, length, band, gap)
    surf = classify_surface(solid)
    t = np.where(solid, SOLID, FLUID).astype(np.uint8)
    for centre, axis in fibres:
        n = _unit_vector(rng)
        n = n - (n @ axis) * axis
        n /= np.linalg.norm(n)
        z, y, x, d = cylinder_voxels(shape, centre, axis, r, length)
        on = surf[z, y, x]
        side = d @ n < 0
        t[z[on & side], y[on & side], x[on & side]] = CAT1
        t[z[on & ~side], y[on & ~side], x[on & ~side]] = CAT2
    return t
