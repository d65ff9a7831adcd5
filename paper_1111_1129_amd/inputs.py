"""Seeded synthetic geometries for the list-based lattice Boltzmann solver.

This module produces *inputs only*: flag fields (uint8, 1 = fluid, 0 = solid,
indexed ``[z][y][x]`` with x fastest) and, for the partial-bounce-back workload,
a per-cell solid fraction field.  It holds none of the method's arithmetic
(no numbering, no compaction, no collision), so both the CPU oracle and the
GPU path can consume the same arrays without sharing any code of the method.

The paper benchmarks two geometries (Sec. 6, Fig. 2): an empty channel and a
tube filled with a random sphere packing.  Neither the geometry files nor the
packing generator are published, so the generators below are stand-ins with
the stated shapes, sizes and porosities:

* ``channel``        -- (5d) x d x d box with 1-cell solid wall layers on the
                          y and z faces (the 500x100x100 case has 500*98*98 =
                          4.802e6 fluid cells, the count quoted in Sec. 7).
* ``packing_small``  -- 32^3 box, walls on y/z faces, non-overlapping spheres
                          of radius 4 placed by random sequential addition (RSA).
* ``packing_tube``   -- 256^3 box, cylindrical tube of diameter 240 along x,
                          filled with non-overlapping radius-12 spheres by RSA.
* ``packing_boolean``-- box with walls on y/z faces and overlapping spheres of
                          random radius (Boolean model) placed until the box
                          porosity reaches a target.
* ``ns_field``       -- smoothed random solid-fraction field in [0, 1].
* ``batch_packings`` -- many Boolean packings of random cube edge length.

RSA stops after a fixed number of consecutive rejections (or at a target
solid fraction); non-overlapping RSA saturates near 38 % sphere fraction in
3-D, so the achieved fraction is recorded rather than forced.

A sphere makes the cell whose centre sits at integer coordinates p solid iff
|p - c|^2 <= r^2, with the x distance taken periodically (x is the periodic
flow direction in every workload).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FLUID = np.uint8(1)
SOLID = np.uint8(0)

# periodic bit mask: bit0 = x, bit1 = y, bit2 = z
PERIODIC_X = 1
PERIODIC_ALL = 7


@dataclasses.dataclass
class Geometry:
    """A flag field plus the metadata that travels with it."""

    name: str
    flags: np.ndarray            # uint8 [nz][ny][nx], 1 = fluid
    periodic: int                # bit mask (bit0 x, bit1 y, bit2 z)
    ns: np.ndarray | None = None  # float64 [nz][ny][nx] solid fraction or None
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.flags.shape
        return nx, ny, nz

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.flags))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def box_with_walls(nx: int, ny: int, nz: int, walls_y: bool = True,
                   walls_z: bool = True) -> np.ndarray:
    """All-fluid box with 1-cell solid layers on the requested faces."""
    f = np.ones((nz, ny, nx), dtype=np.uint8)
    if walls_y:
        f[:, 0, :] = 0
        f[:, ny - 1, :] = 0
    if walls_z:
        f[0, :, :] = 0
        f[nz - 1, :, :] = 0
    return f


def _sphere_cells(shape, centre, radius):
    """Index arrays (z, y, x) of the cells a sphere covers.

    x wraps periodically; y and z are clipped to the box.
    """
    nz, ny, nx = shape
    cx, cy, cz = centre
    r = radius
    x0, x1 = int(math.ceil(cx - r)), int(math.floor(cx + r))
    y0, y1 = max(0, int(math.ceil(cy - r))), min(ny - 1, int(math.floor(cy + r)))
    z0, z1 = max(0, int(math.ceil(cz - r))), min(nz - 1, int(math.floor(cz + r)))
    if y0 > y1 or z0 > z1:
        return None
    xs = np.arange(x0, x1 + 1)
    ys = np.arange(y0, y1 + 1)
    zs = np.arange(z0, z1 + 1)
    d2 = ((zs[:, None, None] - cz) ** 2 + (ys[None, :, None] - cy) ** 2
          + (xs[None, None, :] - cx) ** 2)
    mask = d2 <= r * r
    return zs, ys, np.mod(xs, nx), mask


def _stamp(flags, centre, radius):
    """Mark a sphere solid; return the number of cells that turned solid."""
    got = _sphere_cells(flags.shape, centre, radius)
    if got is None:
        return 0
    zs, ys, xs, mask = got
    sub = flags[np.ix_(zs, ys, xs)]
    newly = int(np.count_nonzero(sub & mask))
    sub[mask] = 0
    flags[np.ix_(zs, ys, xs)] = sub
    return newly


def _rsa(rng, nx, radius, sample_batch, max_rejects, max_spheres):
    """Random sequential addition of equal non-overlapping spheres.

    ``sample_batch(rng, k)`` returns k candidate centres (k x 3, columns x y z).
    Candidates are examined in the order drawn; a candidate is accepted when
    it overlaps no accepted sphere (periodic distance in x).  Stops after
    ``max_rejects`` consecutive rejections or ``max_spheres`` acceptances.
    """
    acc = np.empty((0, 3))
    rejects = 0
    min_d2 = (2.0 * radius) ** 2
    while rejects < max_rejects and len(acc) < max_spheres:
        cand = sample_batch(rng, 4096)
        while len(cand):
            if len(acc):
                dx = np.abs(cand[:, None, 0] - acc[None, :, 0])
                dx = np.minimum(dx, nx - dx)
                d2 = (dx ** 2 + (cand[:, None, 1] - acc[None, :, 1]) ** 2
                      + (cand[:, None, 2] - acc[None, :, 2]) ** 2)
                ok = np.all(d2 >= min_d2, axis=1)
            else:
                ok = np.ones(len(cand), dtype=bool)
            idx = np.flatnonzero(ok)
            if len(idx) == 0:
                rejects += len(cand)
                break
            j = int(idx[0])
            rejects += j
            if rejects >= max_rejects:
                break
            acc = np.vstack([acc, cand[j:j + 1]])
            rejects = 0
            if len(acc) >= max_spheres:
                break
            cand = cand[j + 1:]
    return acc


def packing_small(seed: int = 1, n: int = 32, radius: float = 4.0,
                  target_solid: float = 0.60, max_rejects: int = 100_000) -> Geometry:
    """n^3 box, walls on y/z faces, periodic x, RSA spheres of one radius.

    Centres are uniform in x in [0, n) and in y, z in [1, n-1) (the interior);
    spheres are clipped by the wall layers.  Placement stops at the target
    solid fraction of the box (spheres only) or after ``max_rejects``
    consecutive rejections, whichever comes first.
    """
    rng = _rng(seed)
    flags = box_with_walls(n, n, n)
    sphere_vol = 4.0 / 3.0 * math.pi * radius ** 3
    max_spheres = int(target_solid * n ** 3 / sphere_vol) + 1

    def sample(r, k):
        u = r.random((k, 3))
        return np.column_stack([u[:, 0] * n, 1.0 + u[:, 1] * (n - 2),
                                1.0 + u[:, 2] * (n - 2)])

    centres = _rsa(rng, n, radius, sample, max_rejects, max_spheres)
    for c in centres:
        _stamp(flags, c, radius)
    g = Geometry("packing_small", flags, PERIODIC_X)
    g.info = dict(seed=seed, spheres=len(centres), radius=radius,
                  solid_fraction=1.0 - g.n_fluid / flags.size)
    return g


def packing_tube(seed: int = 2, n: int = 256, diameter: float = 240.0,
                 radius: float = 12.0, max_rejects: int = 100_000,
                 target_porosity: float = 0.40) -> Geometry:
    """n^3 box holding a tube along x packed with equal RSA spheres.

    Cells whose (y, z) centre lies outside the disc of the given diameter
    centred on the box axis are solid; spheres lie fully inside the tube.
    """
    rng = _rng(seed)
    flags = np.ones((n, n, n), dtype=np.uint8)
    c0 = (n - 1) / 2.0
    R = diameter / 2.0
    y = np.arange(n) - c0
    outside = (y[:, None] ** 2 + y[None, :] ** 2) > R * R  # [z][y]
    flags[outside, :] = 0
    rmax = R - radius
    fluid_box = int(np.count_nonzero(flags))
    sphere_vol = 4.0 / 3.0 * math.pi * radius ** 3
    max_spheres = int(max(0.0, fluid_box - target_porosity * flags.size) / sphere_vol) + 1

    def sample(r, k):
        out = []
        while sum(len(o) for o in out) < k:
            u = r.random((k, 3))
            yz = (u[:, 1:] * 2.0 - 1.0) * rmax
            keep = (yz ** 2).sum(axis=1) <= rmax * rmax
            out.append(np.column_stack([u[keep, 0] * n, c0 + yz[keep, 0], c0 + yz[keep, 1]]))
        return np.vstack(out)[:k]

    centres = _rsa(rng, n, radius, sample, max_rejects, max_spheres)
    for c in centres:
        _stamp(flags, c, radius)
    g = Geometry("packing_tube", flags, PERIODIC_X)
    g.info = dict(seed=seed, spheres=len(centres), radius=radius,
                  porosity=g.n_fluid / flags.size)
    return g


def packing_boolean(seed: int, nx: int, ny: int, nz: int, r_min: float, r_max: float,
                    target_porosity: float) -> Geometry:
    """Box with walls on y/z faces, periodic x, overlapping random spheres.

    Centres are uniform in x in [0, nx), y in [1, ny-1), z in [1, nz-1); the
    radius of each sphere is uniform in [r_min, r_max].  Spheres are stamped
    one at a time until the fluid fraction of the whole box is <= target.
    """
    rng = _rng(seed)
    flags = box_with_walls(nx, ny, nz)
    n_box = flags.size
    fluid = int(np.count_nonzero(flags))
    target = target_porosity * n_box
    count = 0
    while fluid > target:
        u = rng.random((1024, 4))
        for row in u:
            c = (row[0] * nx, 1.0 + row[1] * (ny - 2), 1.0 + row[2] * (nz - 2))
            r = r_min + row[3] * (r_max - r_min)
            fluid -= _stamp(flags, c, r)
            count += 1
            if fluid <= target:
                break
    g = Geometry("packing_boolean", flags, PERIODIC_X)
    g.info = dict(seed=seed, spheres=count, r_min=r_min, r_max=r_max,
                  porosity=g.n_fluid / n_box)
    return g


def channel(d: int = 100, length_factor: int = 5) -> Geometry:
    """The paper's empty channel: (5d) x d x d with 1-cell walls on y/z faces."""
    flags = box_with_walls(length_factor * d, d, d)
    return Geometry("channel", flags, PERIODIC_X, info=dict(d=d))


def plate_channel(H: int, nx: int = 1, nz: int = 1) -> Geometry:
    """Plane Poiseuille cell: fluid rows y = 1..H between solid rows y = 0, H+1.

    Periodic in x and z.
    """
    flags = np.ones((nz, H + 2, nx), dtype=np.uint8)
    flags[:, 0, :] = 0
    flags[:, H + 1, :] = 0
    return Geometry("plate_channel", flags, PERIODIC_X | 4, info=dict(H=H))


def all_fluid(nx: int, ny: int, nz: int, periodic: int = PERIODIC_ALL) -> Geometry:
    return Geometry("all_fluid", np.ones((nz, ny, nx), dtype=np.uint8), periodic)


def random_flags(seed: int, nx: int, ny: int, nz: int, fluid_fraction: float = 0.6,
                 periodic: int | None = None) -> Geometry:
    """i.i.d. Bernoulli flag field (for small brute-force tests)."""
    rng = _rng(seed)
    flags = (rng.random((nz, ny, nx)) < fluid_fraction).astype(np.uint8)
    if periodic is None:
        periodic = int(rng.integers(0, 8))
    return Geometry("random", flags, periodic, info=dict(seed=seed))


def ns_field(seed: int, nx: int, ny: int, nz: int, sigma: float = 2.0) -> np.ndarray:
    """Smoothed random solid-fraction field in [0, 1].

    White noise is smoothed with a periodic Gaussian of width ``sigma`` cells
    (FFT), standardised, and mapped through ns = clip(1/2 + (phi - median)/2,
    0, 1), so the median cell is half solid.
    """
    rng = _rng(seed)
    noise = rng.standard_normal((nz, ny, nx))
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    k2 = (2 * math.pi) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2)
    phi = np.fft.irfftn(np.fft.rfftn(noise) * np.exp(-0.5 * sigma ** 2 * k2), s=(nz, ny, nx),
                         axes=(0, 1, 2))
    phi = (phi - phi.mean()) / phi.std()
    return np.clip(0.5 + (phi - np.median(phi)) / 2.0, 0.0, 1.0)


def pbb_box(seed: int = 4, n: int = 128) -> Geometry:
    """n^3 box, walls on y/z faces, periodic x, every interior cell listed and
    carrying a partial-bounce-back solid fraction from ``ns_field``."""
    flags = box_with_walls(n, n, n)
    ns = ns_field(seed, n, n, n)
    ns = np.where(flags == 1, ns, 0.0)
    g = Geometry("pbb_box", flags, PERIODIC_X, ns=ns, info=dict(seed=seed))
    return g


def batch_packings(seed: int = 5000, count: int = 64, l_min: int = 48, l_max: int = 160,
                   por_min: float = 0.3, por_max: float = 0.6, r_min: float = 4.0,
                   r_max: float = 10.0):
    """``count`` Boolean packings of cube edge L ~ U{l_min..l_max} and porosity
    ~ U[por_min, por_max]; geometry k uses child seed ``seed + k``."""
    out = []
    for k in range(count):
        rng = _rng(seed + k)
        L = int(rng.integers(l_min, l_max + 1))
        por = float(por_min + rng.random() * (por_max - por_min))
        g = packing_boolean(int(rng.integers(0, 2 ** 31)), L, L, L, r_min, r_max, por)
        g.name = f"batch{k}"
        g.info.update(edge=L, target_porosity=por)
        out.append(g)
    return out


# ---------------------------------------------------------------------------
# Named workloads.  Each returns Geometry objects; parameters beside them.
# ---------------------------------------------------------------------------

TRT_DEFAULT = dict(tau_plus=0.8, magic=3.0 / 16.0, force=(1e-6, 0.0, 0.0))


def workload(name: str, **kw):
    """Return the geometry (or list of geometries) for a named workload.

    small_packing  32^3 RSA packing, 100 steps, FP64 (parity workload)
    tube_packing   256^3 tube with RSA spheres, 1000 steps, FP64 (throughput)
    large_packing  512 x 512 x 1024 Boolean packing, porosity 0.4 (precision)
    pbb_box        128^3 box with a partial-bounce-back field (adjoint)
    batch          64 uneven Boolean packings (batched launch)
    channel        the paper's 500 x 100 x 100 empty channel
    """
    if name == "small_packing":
        return packing_small(seed=kw.get("seed", 1))
    if name == "tube_packing":
        return packing_tube(seed=kw.get("seed", 2))
    if name == "large_packing":
        s = kw.get("scale", 1)
        return packing_boolean(kw.get("seed", 3), 512 // s, 512 // s, 1024 // s,
                               8.0 / s, 16.0 / s, 0.40)
    if name == "pbb_box":
        return pbb_box(seed=kw.get("seed", 4), n=kw.get("n", 128))
    if name == "batch":
        return batch_packings(seed=kw.get("seed", 5000), count=kw.get("count", 64))
    if name == "channel":
        return channel(d=kw.get("d", 100))
    raise KeyError(name)
