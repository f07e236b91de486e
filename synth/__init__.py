"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and builds input geometry (point
clouds and triangle meshes).  It holds none of the fast-multipole or
boundary-element arithmetic: no Green's functions, no quadrature rules, no
trees.  The paper's own inputs (PDB structures meshed by Nanoshaper) are not
available, so sphere and sphere-union surfaces with the paper's sizes stand in
for them (the workloads of the paper's performance and convergence sections).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "unit_sphere_cloud",
    "octa_sphere",
    "SphereUnion",
    "sphere_union_spheres",
    "sphere_union_mesh",
    "centroid_points",
    "three_point_cloud",
    "charges_in_spheres",
    "random_rotation",
    "surface_cloud",
    "molecule_batch",
    "used_vertices_only",
]


def unit_sphere_cloud(n: int, seed: int = 0):
    """n points x = v/|v| with v ~ N(0, I3); densities uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    x = v / np.linalg.norm(v, axis=1, keepdims=True)
    q = rng.uniform(-1.0, 1.0, n)
    return np.ascontiguousarray(x), q


def octa_sphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Octahedron subdivided `level` times (each triangle split in four) and
    projected onto a sphere: 8 * 4**level triangles, counter-clockwise seen
    from outside (outward normals).  Returns (verts (nv,3), tris (nt,3) int32)."""
    verts = [
        (1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
        (0.0, -1.0, 0.0), (0.0, 0.0, 1.0), (0.0, 0.0, -1.0),
    ]
    tris = [
        (0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4),
        (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5),
    ]
    vlist = [np.array(v, dtype=np.float64) for v in verts]
    for _ in range(level):
        cache: dict = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = 0.5 * (vlist[a] + vlist[b])
                vlist.append(m / np.linalg.norm(m))
                cache[key] = len(vlist) - 1
            return cache[key]

        new = []
        for (a, b, c) in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = new
    v = np.array(vlist) * radius + np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(v), np.ascontiguousarray(np.array(tris, dtype=np.int32))


def random_rotation(rng) -> np.ndarray:
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    a = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


@dataclass
class SphereUnion:
    centers: np.ndarray  # (m, 3)
    radii: np.ndarray    # (m,)


def sphere_union_spheres(n_spheres: int, seed: int, box: float = 40.0,
                         rmin: float = 1.5, rmax: float = 2.0,
                         shell_radius: float | None = None,
                         shell_width: float = 10.0) -> SphereUnion:
    """Sphere centres U[0, box]^3 (or, with `shell_radius`, uniform directions
    at a radius U[R - w/2, R + w/2]) and radii U[rmin, rmax]."""
    rng = np.random.default_rng(seed)
    if shell_radius is None:
        c = rng.uniform(0.0, box, (n_spheres, 3))
    else:
        d = rng.standard_normal((n_spheres, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rr = rng.uniform(shell_radius - shell_width / 2, shell_radius + shell_width / 2, n_spheres)
        c = d * rr[:, None]
    r = rng.uniform(rmin, rmax, n_spheres)
    return SphereUnion(c, r)


def _fibonacci_sphere(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = k * (math.pi * (3.0 - math.sqrt(5.0)))
    return np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)


def _hull_tris(n: int):
    from scipy.spatial import ConvexHull
    p = _fibonacci_sphere(n)
    h = ConvexHull(p)
    t = h.simplices.astype(np.int64)
    # orient counter-clockwise seen from outside
    a, b, c = p[t[:, 0]], p[t[:, 1]], p[t[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    t[flip] = t[flip][:, [0, 2, 1]]
    return p, t


def _exposed_mesh(su: SphereUnion, density: float, seed: int, cell: float, gap: float | None = None):
    """Triangulate each sphere with ~density * 4 pi r^2 hull triangles and drop
    triangles whose centroid lies inside another sphere (gap=None), or, with
    gap = g, every triangle with a vertex closer than g mean edge lengths to
    the inside of another sphere: the caps of two intersecting spheres then
    stop short of their intersection curve, about g edge lengths apart,
    instead of crossing each other there."""
    rng = np.random.default_rng(seed + 7919)
    m = len(su.radii)
    # spatial hash of sphere centres for the "inside another sphere" test
    keys = np.floor(su.centers / cell).astype(np.int64)
    buckets: dict = {}
    for i, k in enumerate(map(tuple, keys)):
        buckets.setdefault(k, []).append(i)
    cache: dict = {}
    vs, ts, nv = [], [], 0
    for i in range(m):
        r = su.radii[i]
        npts = max(8, int(round(density * 4.0 * math.pi * r * r / 2.0)) + 2)
        if npts not in cache:
            cache[npts] = _hull_tris(npts)
        p, t = cache[npts]
        rot = random_rotation(rng)
        v = (p @ rot.T) * r + su.centers[i]
        cen = v[t].mean(axis=1)
        keep = np.ones(len(t), dtype=bool)
        if gap is not None:
            e = v[t[:, 1]] - v[t[:, 0]]
            margin = gap * float(np.mean(np.sqrt(np.sum(e * e, axis=1))))
        k0 = keys[i]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in buckets.get((k0[0] + dx, k0[1] + dy, k0[2] + dz), ()):
                        if j == i:
                            continue
                        if gap is None:
                            d2 = np.sum((cen - su.centers[j]) ** 2, axis=1)
                            keep &= d2 >= su.radii[j] ** 2
                        else:
                            dv2 = np.sum((v - su.centers[j]) ** 2, axis=1)
                            keep &= ~(dv2 < (su.radii[j] + margin) ** 2)[t].any(axis=1)
        t = t[keep]
        if len(t) == 0:
            continue
        used = np.unique(t)
        remap = -np.ones(len(v), dtype=np.int64)
        remap[used] = np.arange(len(used)) + nv
        vs.append(v[used])
        ts.append(remap[t])
        nv += len(used)
    if not vs:
        return np.zeros((0, 3)), np.zeros((0, 3), dtype=np.int64)
    return np.concatenate(vs), np.concatenate(ts)


def sphere_union_mesh(su: SphereUnion, n_triangles: int, seed: int, exact: bool = True,
                      gap: float | None = None):
    """Exposed surface of a union of spheres with exactly `n_triangles`
    triangles (counter-clockwise seen from outside).  The per-sphere
    triangle density is raised by bisection until the exposed count reaches
    the target; the surplus is dropped in a seeded shuffle order (holes are
    harmless for point-cloud workloads).  exact=False keeps the whole
    exposed surface of the final density instead (n_triangles to 1.02
    n_triangles triangles, no holes).  gap: see _exposed_mesh (boundary-
    element meshes use gap=0.5, so that no two triangles of different
    spheres cross or nearly touch).  Returns (verts, tris int32)."""
    cell = 2.0 * float(su.radii.max())
    area = float(np.sum(4.0 * math.pi * su.radii ** 2))
    lo, hi = 0.5 * n_triangles / area, 0.5 * n_triangles / area
    v, t = _exposed_mesh(su, hi, seed, cell, gap)
    while len(t) < n_triangles:
        lo = hi
        hi *= 1.6
        v, t = _exposed_mesh(su, hi, seed, cell, gap)
    for _ in range(12):
        if len(t) <= n_triangles * 1.02:
            break
        mid = 0.5 * (lo + hi)
        v2, t2 = _exposed_mesh(su, mid, seed, cell, gap)
        if len(t2) >= n_triangles:
            hi, v, t = mid, v2, t2
        else:
            lo = mid
    if exact:
        rng = np.random.default_rng(seed + 104729)
        sel = np.sort(rng.permutation(len(t))[:n_triangles])
        t = t[sel]
    used = np.unique(t)
    remap = -np.ones(len(v), dtype=np.int64)
    remap[used] = np.arange(len(used))
    return np.ascontiguousarray(v[used]), np.ascontiguousarray(remap[t].astype(np.int32))


def used_vertices_only(verts, tris):
    """(verts, tris) without the vertices no triangle uses (the sphere-union
    meshes drop buried triangles but keep every lattice point), triangle
    indices renumbered in order."""
    verts = np.asarray(verts)
    tris = np.asarray(tris)
    used = np.zeros(len(verts), dtype=bool)
    used[tris.reshape(-1)] = True
    new = np.cumsum(used) - 1
    return np.ascontiguousarray(verts[used]), new[tris].astype(tris.dtype)


def three_point_cloud(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Point cloud of three points per triangle at barycentric (2/3, 1/6, 1/6)
    and its permutations: the sample layout of a 3-point regular rule.  Used
    only to build point-cloud workloads with the shape of the paper's
    quadrature-point sets; the boundary-element code computes its own points."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    p0 = (4 * a + b + c) / 6.0
    p1 = (a + 4 * b + c) / 6.0
    p2 = (a + b + 4 * c) / 6.0
    return np.ascontiguousarray(np.stack([p0, p1, p2], axis=1).reshape(-1, 3))


def centroid_points(verts, tris):
    return verts[tris].mean(axis=1)


def charges_in_spheres(su: SphereUnion, n_charges: int, seed: int, frac: float = 0.5):
    """Point charges U[-1, 1] e, each inside a random sphere within frac*r of
    its centre."""
    rng = np.random.default_rng(seed + 15485863)
    idx = rng.integers(0, len(su.radii), n_charges)
    d = rng.standard_normal((n_charges, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = rng.uniform(0.0, 1.0, n_charges) ** (1.0 / 3.0) * frac * su.radii[idx]
    x = su.centers[idx] + d * rad[:, None]
    q = rng.uniform(-1.0, 1.0, n_charges)
    return np.ascontiguousarray(x), q


def surface_cloud(n_spheres: int, n_triangles: int, seed: int, box: float | None = None,
                  shell_radius: float | None = None):
    """Point-cloud workload: three points per triangle of an n_triangles
    exposed-surface mesh of n_spheres spheres (radii U[1.5, 2.0] A), centres in
    a cube of side `box` (default 40 (n_spheres / 200)^(1/3) A, the density of
    200 spheres in a 40 A cube) or, with shell_radius, in a 10 A thick shell;
    densities N(0, 1).  Returns (points (3 n_triangles, 3), densities)."""
    if box is None:
        box = 40.0 * (n_spheres / 200.0) ** (1.0 / 3.0)
    su = sphere_union_spheres(n_spheres, seed=seed, box=box, shell_radius=shell_radius)
    v, t = sphere_union_mesh(su, n_triangles, seed=seed)
    x = three_point_cloud(v, t)
    q = np.random.default_rng(seed).standard_normal(len(x))
    return x, q


def molecule_batch(nmol: int = 64, seed: int = 5):
    """nmol molecules of N_m = 3 round(exp(U[ln 5000, ln 60000]) / 3) points
    (log-uniform sizes), each a surface_cloud of ceil(N_m / 400) spheres;
    densities N(0, 1).  Returns (list of points, list of densities)."""
    rng = np.random.default_rng(seed)
    xs, qs = [], []
    for m in range(nmol):
        nm = 3 * int(round(math.exp(rng.uniform(math.log(5000), math.log(60000))) / 3))
        nsph = int(math.ceil(nm / 400))
        su = sphere_union_spheres(nsph, seed=seed * 1000 + m, box=40.0 * (nsph / 200) ** (1 / 3))
        v, t = sphere_union_mesh(su, nm // 3, seed=seed * 1000 + m)
        xs.append(three_point_cloud(v, t))
        qs.append(rng.standard_normal(nm))
    return xs, qs
