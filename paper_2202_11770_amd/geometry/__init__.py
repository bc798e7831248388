"""Seeded synthetic vessel geometries (inputs for the sparse D3Q19 update).

This module produces the inputs that both the CPU oracle and the GPU library
consume: fluid-site coordinates, site types and the push-direction neighbour
table ``nbr[x][i]`` (id of the site at ``x + c_i``, ``-1`` for a wall link,
``-(2+k)`` for a link through iolet ``k``).  It contains no part of the
lattice-Boltzmann arithmetic.

The velocity order is the D3Q19 set of the paper (Sec. 2.2) with opposite
directions adjacent: ``opp(i) = i+1`` for odd ``i``.

Geometries (all seeded, all starting from rest):

* ``cylinder``  straight pipe, radius 8, length 64 in a 20x20x64 box
  (13,312 sites); parabolic velocity inlet at z=0, pressure outlet at z=63.
* ``tree``      recursive binary branching of capsules (Murray radii,
  branch angle 30-60 deg, branch length 6-10 radii), one inlet at the root
  and one outlet per leaf, scaled to a target number of fluid sites;
  ``subtree`` cuts a branch of it out as its own vessel.
* ``tortuous``  a single vessel with a sinusoidal centre line.
* ``forest``    a grid of independent trees.
* ``duct``, ``sealed_box``, ``periodic_box``, ``couette_column``: the small
  closed-form test cases.
"""
from __future__ import annotations

import ctypes
import math
import os
import sys
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = os.path.join(_HERE, "libhlbgeom.so")
_lib = None

# Same velocity order as every consumer of the table (see module docstring).
C = np.array(
    [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
     [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
     [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int32)
OPP = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, 19)], dtype=np.int32)

SITE_BULK, SITE_WALL, SITE_INLET, SITE_OUTLET, SITE_INLET_WALL, SITE_OUTLET_WALL = range(6)
LINK_WALL = -1
VELOCITY, PRESSURE = 0, 1
INLET, OUTLET = 0, 1


def build_library(verbose: bool = False) -> str:
    """Compile ``libhlbgeom.so`` next to this file (g++, OpenMP)."""
    import subprocess
    src = os.path.join(_HERE, "geom.cpp")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", src, "-o", _LIBNAME]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIBNAME


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBNAME):
        build_library()
    lib = ctypes.CDLL(_LIBNAME)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.gm_count.argtypes = [P, i64]
    lib.gm_count.restype = i64
    lib.gm_capsules.argtypes = [i64, P, P, P, P, P, i64, i64, i64, P, P]
    lib.gm_capsules.restype = None
    lib.gm_build.argtypes = [i64, i64, i64, P, P, ctypes.c_int32, P, P, P, P, i64, P, P, P]
    lib.gm_build.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Iolet:
    kind: int            # VELOCITY (Ladd) or PRESSURE (ghost density)
    role: int            # INLET or OUTLET
    centre: tuple        # a point of the iolet plane
    normal: tuple        # unit normal pointing into the fluid
    radius: float        # disk radius; <= 0 means unbounded / uniform profile
    vdir: tuple = (0.0, 0.0, 0.0)  # imposed velocity direction (zero: the normal)
    table: np.ndarray = None       # per-step amplitude A_k(s) or density rho_k(s)


@dataclass
class Geometry:
    coords: np.ndarray   # (n, 3) int32
    types: np.ndarray    # (n,) uint8
    nbr: np.ndarray      # (n, 19) int32
    iolets: list
    dims: tuple
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.types.shape[0])

    def wall_sites(self) -> np.ndarray:
        return np.nonzero((self.nbr == LINK_WALL).any(axis=1))[0]


def _bitmap(nx, ny, nz):
    return np.zeros((nx * ny * nz + 63) // 64, dtype=np.uint64)


def voxelise_capsules(a, b, r, cut_a, cut_b, dims, origin):
    lib = _load()
    nx, ny, nz = (int(d) for d in dims)
    bits = _bitmap(nx, ny, nz)
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    ca = np.ascontiguousarray(cut_a, dtype=np.int32)
    cb = np.ascontiguousarray(cut_b, dtype=np.int32)
    org = np.ascontiguousarray(origin, dtype=np.float64)
    lib.gm_capsules(len(r), _ptr(a), _ptr(b), _ptr(r), _ptr(ca), _ptr(cb), nx, ny, nz, _ptr(org), _ptr(bits))
    return bits


def count(bits, dims) -> int:
    nx, ny, nz = dims
    return int(_load().gm_count(_ptr(bits), nx * ny * nz))


def build_sites(bits, dims, iolets, periodic=(0, 0, 0), meta=None) -> Geometry:
    """Site list, types and neighbour table of a voxel bitmap."""
    lib = _load()
    nx, ny, nz = (int(d) for d in dims)
    n = count(bits, dims)
    coords = np.empty((n, 3), dtype=np.int32)
    types = np.empty(n, dtype=np.uint8)
    nbr = np.empty((n, 19), dtype=np.int32)
    k = len(iolets)
    centre = np.array([io.centre for io in iolets], dtype=np.float64).reshape(k, 3)
    normal = np.array([io.normal for io in iolets], dtype=np.float64).reshape(k, 3)
    radius = np.array([io.radius for io in iolets], dtype=np.float64).reshape(k)
    role = np.array([io.role for io in iolets], dtype=np.int32).reshape(k)
    per = np.array(periodic, dtype=np.int32)
    rc = lib.gm_build(nx, ny, nz, _ptr(bits), _ptr(per), k, _ptr(centre), _ptr(normal), _ptr(radius),
                      _ptr(role), n, _ptr(coords), _ptr(types), _ptr(nbr))
    if rc != 0:
        raise ValueError(f"gm_build failed ({rc}): a site touches an inlet and an outlet")
    return Geometry(coords, types, nbr, list(iolets), (nx, ny, nz), dict(meta or {}))


# ---------------------------------------------------------------------------
# small closed-form test geometries
# ---------------------------------------------------------------------------

def cylinder(radius: float = 8.0, length: int = 64, box: int = 20, u_max: float = 0.01,
             rho_out: float = 1.0) -> Geometry:
    """Straight pipe along z; parabolic velocity inlet, pressure outlet.

    Axis at (box/2 - 1/2, box/2 - 1/2); fluid iff the squared distance to the
    axis is below radius^2 and 0 <= z < length.  The inlet plane is z = -1/2
    (normal +z), the outlet plane z = length - 1/2 (normal -z).
    """
    c = box / 2.0 - 0.5
    a = np.array([[c, c, -0.5]])
    b = np.array([[c, c, length - 0.5]])
    bits = voxelise_capsules(a, b, [radius], [1], [1], (box, box, length), (0.0, 0.0, 0.0))
    iolets = [
        Iolet(VELOCITY, INLET, (c, c, -0.5), (0.0, 0.0, 1.0), radius, table=np.array([u_max])),
        Iolet(PRESSURE, OUTLET, (c, c, length - 0.5), (0.0, 0.0, -1.0), radius, table=np.array([rho_out])),
    ]
    return build_sites(bits, (box, box, length), iolets,
                       meta=dict(name="cylinder", radius=radius, length=length, axis=(c, c)))


def duct(a: int = 16, b: int = 16, length: int = 64, rho_in: float = 1.006, rho_out: float = 1.0) -> Geometry:
    """Rectangular duct a x b x length; pressure iolets at both ends, walls elsewhere."""
    bits = _pack(np.ones(a * b * length, dtype=bool))
    big = float(a + b)
    cx, cy = (a - 1) / 2.0, (b - 1) / 2.0
    iolets = [
        Iolet(PRESSURE, INLET, (cx, cy, -0.5), (0.0, 0.0, 1.0), big, table=np.array([rho_in])),
        Iolet(PRESSURE, OUTLET, (cx, cy, length - 0.5), (0.0, 0.0, -1.0), big, table=np.array([rho_out])),
    ]
    return build_sites(bits, (a, b, length), iolets, meta=dict(name="duct", a=a, b=b, length=length))


def _pack(occ: np.ndarray) -> np.ndarray:
    """Pack a flat boolean occupancy (lexicographic z,y,x) into a uint64 bitmap."""
    nv = occ.size
    pad = (-nv) % 64
    o = np.concatenate([occ.astype(np.uint8), np.zeros(pad, dtype=np.uint8)])
    by = np.packbits(o, bitorder="little")  # bit j of byte k = voxel 8k + j
    return by.view("<u8").astype(np.uint64)


def sealed_box(nx: int, ny: int | None = None, nz: int | None = None) -> Geometry:
    """Closed box of fluid; every outward link is a wall link."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    bits = _pack(np.ones(nx * ny * nz, dtype=bool))
    return build_sites(bits, (nx, ny, nz), [], meta=dict(name="sealed_box"))


def periodic_box(nx: int, ny: int, nz: int, periodic=(1, 1, 1)) -> Geometry:
    """Box of fluid, wrapping along the flagged axes (walls on the others)."""
    bits = _pack(np.ones(nx * ny * nz, dtype=bool))
    return build_sites(bits, (nx, ny, nz), [], periodic=periodic, meta=dict(name="periodic_box"))


def couette_column(H: int = 8, U: float = 0.01) -> Geometry:
    """1x1xH column periodic in x and y; wall below z=0, moving lid above z=H-1.

    The lid is a uniform velocity iolet with tangential direction +x.
    """
    bits = _pack(np.ones(H, dtype=bool))
    lid = Iolet(VELOCITY, INLET, (0.0, 0.0, H - 0.5), (0.0, 0.0, -1.0), 0.0, vdir=(1.0, 0.0, 0.0),
                table=np.array([U]))
    return build_sites(bits, (1, 1, H), [lid], periodic=(1, 1, 0), meta=dict(name="couette", H=H, U=U))


# ---------------------------------------------------------------------------
# trees
# ---------------------------------------------------------------------------

def _rot_frame(d):
    """Two unit vectors orthogonal to unit vector d."""
    d = np.asarray(d, dtype=np.float64)
    t = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(d, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return e1, e2


def tree_segments(seed: int, generations: int = 8, base_radius: float = 40.0, scale: float = 1.0,
                  origin=(0.0, 0.0, 0.0)):
    """Random binary tree of capsules (all random draws depend only on the seed).

    Root starts at ``origin`` along +z with radius base_radius*scale.  Each
    branching halves the flow: child radius = parent * 2^(-1/3) (Murray).
    Child axes make an angle U(30,60) deg with the parent axis; the first
    child's azimuth is U(0, 2 pi), its sibling's is opposite.  Lengths are
    U(6, 10) radii.  Returns a dict of arrays over segments in breadth-first
    order: a, b, r, parent, depth.
    """
    rng = np.random.default_rng(seed)
    a_list, b_list, r_list, parent, depth = [], [], [], [], []
    r0 = base_radius * scale
    L0 = rng.uniform(6.0, 10.0) * r0
    start = np.asarray(origin, dtype=np.float64)
    d0 = np.array([0.0, 0.0, 1.0])
    queue = [(start, d0, r0, L0, -1, 0)]
    head = 0
    dirs = []
    while head < len(queue):
        s, d, r, L, par, g = queue[head]
        head += 1
        idx = len(a_list)
        a_list.append(s)
        e = s + L * d
        b_list.append(e)
        r_list.append(r)
        parent.append(par)
        depth.append(g)
        dirs.append(d)
        if g < generations:
            rc = r * 2.0 ** (-1.0 / 3.0)
            phi = rng.uniform(0.0, 2.0 * math.pi)
            e1, e2 = _rot_frame(d)
            for side in range(2):
                theta = math.radians(rng.uniform(30.0, 60.0))
                ph = phi + side * math.pi
                dc = math.cos(theta) * d + math.sin(theta) * (math.cos(ph) * e1 + math.sin(ph) * e2)
                dc /= np.linalg.norm(dc)
                Lc = rng.uniform(6.0, 10.0) * rc
                queue.append((e, dc, rc, Lc, idx, g + 1))
    return dict(a=np.array(a_list), b=np.array(b_list), r=np.array(r_list), parent=np.array(parent),
                depth=np.array(depth), d=np.array(dirs))


def _subtree_ids(seg, root):
    ids = [root]
    head = 0
    children = {}
    for i, p in enumerate(seg["parent"]):
        children.setdefault(int(p), []).append(i)
    while head < len(ids):
        ids.extend(children.get(ids[head], []))
        head += 1
    return np.array(sorted(ids))


def _tree_geometry(seg, ids, root, inlet_kind, outlet_kind, name, extra_meta, build=True, trees=None,
                   verbose=False):
    """Voxelise segments `ids` of one or more trees; inlets at the roots, outlets at leaves."""
    t0 = time.time()
    a, b, r = seg["a"][ids], seg["b"][ids], seg["r"][ids]
    parent = seg["parent"]
    idset = set(int(i) for i in ids)
    has_child = set(int(p) for i, p in enumerate(parent) if i in idset and int(p) in idset)
    roots = [root] if trees is None else trees
    cut_a = np.array([1 if int(i) in roots else 0 for i in ids], dtype=np.int32)
    cut_b = np.array([0 if int(i) in has_child else 1 for i in ids], dtype=np.int32)
    lo = np.minimum(a, b) - r[:, None]
    hi = np.maximum(a, b) + r[:, None]
    lo = np.floor(lo.min(axis=0)) - 2
    hi = np.ceil(hi.max(axis=0)) + 2
    dims = tuple(int(v) for v in (hi - lo + 1))
    origin = lo
    bits = voxelise_capsules(a, b, r, cut_a, cut_b, dims, origin)
    n = count(bits, dims)
    if verbose:
        print(f"{name}: voxelised {dims} -> {n} sites in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    if not build:
        return n, dims
    iolets = []
    d = seg["d"]
    for i in ids:
        i = int(i)
        if i in roots:
            c = seg["a"][i] - origin
            iolets.append(Iolet(inlet_kind, INLET, tuple(c), tuple(d[i]), float(seg["r"][i])))
    for i in ids:
        i = int(i)
        if i not in has_child:
            c = seg["b"][i] - origin
            iolets.append(Iolet(outlet_kind, OUTLET, tuple(c), tuple(-d[i]), float(seg["r"][i])))
    meta = dict(name=name, fill=n / float(np.prod(dims)), n_segments=len(ids))
    meta.update(extra_meta)
    g = build_sites(bits, dims, iolets, meta=meta)
    if verbose:
        print(f"{name}: site list and neighbour table built, {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    return g


def tree(seed: int = 2, generations: int = 8, target_sites: int | None = 20_000_000,
         scale: float | None = None, inlet_kind: int = VELOCITY, outlet_kind: int = PRESSURE,
         rel_tol: float = 0.01, verbose: bool = False) -> Geometry:
    """Seeded bifurcating tree scaled to about ``target_sites`` fluid sites.

    The root starts on the plane z = -1/2 (its inlet) with its axis through a
    voxel-centre column; each leaf ends on its own outlet plane.
    """
    origin = (0.5, 0.5, -0.5)
    if scale is None:
        s = 1.0
        for _ in range(12):
            seg = tree_segments(seed, generations, scale=s, origin=origin)
            n, _ = _tree_geometry(seg, np.arange(len(seg["r"])), 0, inlet_kind, outlet_kind, "tree", {}, build=False)
            if abs(n - target_sites) <= rel_tol * target_sites:
                break
            s *= (target_sites / n) ** (1.0 / 3.0)
        scale = s
    seg = tree_segments(seed, generations, scale=scale, origin=origin)
    g = _tree_geometry(seg, np.arange(len(seg["r"])), 0, inlet_kind, outlet_kind, "tree",
                       dict(seed=seed, generations=generations, scale=scale), verbose=verbose)
    g.meta["segments"] = seg
    return g


def subtree(parent_tree=None, target_sites: int = 2_000_000, inlet_kind: int = VELOCITY,
            outlet_kind: int = PRESSURE, segments=None, scale: float | None = None) -> Geometry:
    """The subtree rooted at the first child of the generation whose subtree
    size is closest to ``target_sites`` (by ratio), voxelised at the same
    spacing.

    Pass either the parent tree (its segments are in ``meta``) or the
    parent's ``segments`` and ``scale``.  Generations are tried from the
    deepest up and the search stops once a subtree exceeds twice the target,
    so the large subtrees near the root are never voxelised.  The subtree's
    root segment gets its own inlet (flat cut at the branch start).
    """
    seg = segments if segments is not None else parent_tree.meta["segments"]
    sc = scale if scale is not None else parent_tree.meta["scale"]
    depth = seg["depth"]
    best = None
    for g in range(int(depth.max()), 0, -1):
        first = int(np.nonzero(depth == g)[0][0])
        ids = _subtree_ids(seg, first)
        n, _ = _tree_geometry(seg, ids, first, inlet_kind, outlet_kind, "subtree", {}, build=False)
        if best is None or abs(np.log(n / target_sites)) < abs(np.log(best[1] / target_sites)):
            best = (first, n, ids, g)
        if n > 2 * target_sites:
            break
    first, n, ids, g = best
    return _tree_geometry(seg, ids, first, inlet_kind, outlet_kind, "subtree",
                          dict(root_segment=first, generation=g, scale=sc))


def forest(seed: int = 5, grid: int = 8, generations: int = 4, target_sites: int | None = 600_000_000,
           scale: float | None = None, spacing_radii: float = 12.0, rel_tol: float = 0.01,
           verbose: bool = False) -> Geometry:
    """grid x grid independent trees side by side (seed + tree index)."""
    def segs(s):
        allseg = dict(a=[], b=[], r=[], parent=[], depth=[], d=[])
        roots = []
        off = 0
        pitch = spacing_radii * 40.0 * s
        for t in range(grid * grid):
            gx, gy = t % grid, t // grid
            sg = tree_segments(seed * 1000 + t, generations, scale=s,
                               origin=(0.5 + round(gx * pitch), 0.5 + round(gy * pitch), -0.5))
            roots.append(off)
            for key in ("a", "b", "r", "depth", "d"):
                allseg[key].append(sg[key])
            allseg["parent"].append(np.where(sg["parent"] >= 0, sg["parent"] + off, -1))
            off += len(sg["r"])
        return {k: np.concatenate(v) for k, v in allseg.items()}, roots
    if scale is None:
        s = 1.0
        for _ in range(12):
            seg, roots = segs(s)
            n, _ = _tree_geometry(seg, np.arange(len(seg["r"])), roots[0], VELOCITY, PRESSURE, "forest", {},
                                  build=False, trees=roots)
            if abs(n - target_sites) <= rel_tol * target_sites:
                break
            s *= (target_sites / n) ** (1.0 / 3.0)
        scale = s
    seg, roots = segs(scale)
    return _tree_geometry(seg, np.arange(len(seg["r"])), roots[0], VELOCITY, PRESSURE, "forest",
                          dict(seed=seed, scale=scale, trees=len(roots)), trees=roots, verbose=verbose)


def tortuous(radius: float = 12.0, length: int = 256, amplitude: float = 12.0, period: float = 128.0,
             n_pieces: int = 256) -> Geometry:
    """Single vessel whose centre line is (A sin(2 pi z / P) + c, c, z), 0 <= z < length.

    Built as a chain of short capsules along the centre line; flat velocity
    inlet at z = -1/2 and pressure outlet at z = length - 1/2.
    """
    c = amplitude + radius + 2.5
    zs = np.linspace(-0.5, length - 0.5, n_pieces + 1)
    pts = np.stack([amplitude * np.sin(2 * np.pi * zs / period) + c, np.full_like(zs, c), zs], axis=1)
    a, b = pts[:-1], pts[1:]
    r = np.full(n_pieces, radius)
    nx = int(2 * c + 1)
    ny = int(2 * c + 1)
    dims = (nx, ny, length)
    # cut the ends with the planes z = -1/2 and z = length - 1/2 by restricting the box
    bits = voxelise_capsules(a, b, r, np.zeros(n_pieces, np.int32), np.zeros(n_pieces, np.int32), dims,
                             (0.0, 0.0, 0.0))
    # the end planes cut the tilted vessel in an ellipse whose long semi-axis
    # is radius / cos(tilt); the iolet disks use that radius
    slope = lambda z: 2 * np.pi * amplitude / period * np.cos(2 * np.pi * z / period)
    cl = lambda z: (amplitude * np.sin(2 * np.pi * z / period) + c, c, z)
    r_in = radius * math.hypot(1.0, slope(-0.5))
    r_out = radius * math.hypot(1.0, slope(length - 0.5))
    iolets = [
        Iolet(VELOCITY, INLET, cl(-0.5), (0.0, 0.0, 1.0), r_in),
        Iolet(PRESSURE, OUTLET, cl(length - 0.5), (0.0, 0.0, -1.0), r_out),
    ]
    return build_sites(bits, dims, iolets, meta=dict(name="tortuous", radius=radius, length=length))


def permute(g: Geometry, perm: np.ndarray) -> Geometry:
    """Renumber sites: new site j is old site perm[j]."""
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    nbr = g.nbr[perm].copy()
    m = nbr >= 0
    nbr[m] = inv[nbr[m]].astype(np.int32)
    return Geometry(g.coords[perm].copy(), g.types[perm].copy(), nbr, list(g.iolets), g.dims, dict(g.meta))
