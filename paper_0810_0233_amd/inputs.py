"""Seeded synthetic inputs (geometry and magnetisation configurations).

This module holds input generation only -- none of the method's arithmetic --
and is the one piece shared by the GPU path's tests/benchmark and the CPU
oracle's tests.  Every generator is deterministic in its seed (numpy PCG64).

The workloads stand in for the paper's benchmark of randomly oriented dipoles
on a simple cubic lattice (Sec. 4) and extend it to the geometries the method
is meant for (ferrofluids, clusters, thin films with holes):

* ``lattice``        simple cubic lattice, sites at integer coordinates, root
                     cell = unit cells around the sites.
* ``ferrofluid``     hard-core points by random sequential addition.
* ``sphere_cut``     the N lattice sites nearest the centre of a cubic lattice.
* ``clusters``       Gaussian clusters in a cubic box.
* ``film_with_holes`` thin-film lattice with circular holes through all layers.

Moments are unit vectors, uniform on the sphere: z = 2u - 1, phi = 2 pi v.
"""
import math

import numpy as np


def unit_moments(n, rng):
    """n unit vectors uniform on S^2 (z = 2u-1, phi = 2 pi v), shape (n, 3)."""
    uv = rng.random((n, 2))
    z = 2.0 * uv[:, 0] - 1.0
    phi = 2.0 * math.pi * uv[:, 1]
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def random_moments(n, seed):
    return unit_moments(n, np.random.default_rng(seed))


def lattice(nx, ny, nz, spacing=1.0):
    """Sites (i, j, k)*spacing, i < nx etc., x slowest.  Box = [-s/2, n*s - s/2]."""
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pos = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * spacing
    lo = np.array([-0.5, -0.5, -0.5]) * spacing
    hi = np.array([nx - 0.5, ny - 0.5, nz - 0.5]) * spacing
    return pos, (lo, hi)


def ferrofluid_side(n, volume_fraction=0.1, dmin=1.0):
    """Cube side for n spheres of diameter dmin at the given volume fraction."""
    return (n * math.pi * dmin ** 3 / (6.0 * volume_fraction)) ** (1.0 / 3.0)


def ferrofluid(n, seed, volume_fraction=0.1, dmin=1.0, batch=1 << 15):
    """Random sequential addition: candidates uniform in [0, side)^3, taken in
    candidate order, accepted iff at distance >= dmin from every accepted point.
    Returns (pos (n,3), box)."""
    from scipy.spatial import cKDTree

    side = ferrofluid_side(n, volume_fraction, dmin)
    rng = np.random.default_rng(seed)
    nc = max(1, int(side // dmin))
    csize = side / nc
    slots = 8  # at most 8 points with mutual distance >= dmin fit in a cube of side < 2 dmin/sqrt(3)
    grid = np.full((nc, nc, nc, slots), -1, dtype=np.int32)
    fill = np.zeros((nc, nc, nc), dtype=np.int8)
    out = np.empty((n, 3))
    count = 0
    d2 = dmin * dmin
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    while count < n:
        cand = rng.random((batch, 3)) * side
        ci = np.minimum((cand / csize).astype(np.int64), nc - 1)
        ok = np.ones(batch, dtype=bool)
        # conflicts with already accepted points
        for o in offs:
            cj = ci + o
            valid = np.all((cj >= 0) & (cj < nc), axis=1)
            idx = np.where(valid)[0]
            if idx.size == 0:
                continue
            sl = grid[cj[idx, 0], cj[idx, 1], cj[idx, 2]]  # (k, slots)
            for s in range(slots):
                pj = sl[:, s]
                has = pj >= 0
                if not np.any(has):
                    continue
                ii = idx[has]
                dd = np.sum((cand[ii] - out[pj[has]]) ** 2, axis=1)
                ok[ii[dd < d2]] = False
        # conflicts inside the batch, resolved in candidate order
        okidx = np.where(ok)[0]
        if okidx.size > 1:
            tree = cKDTree(cand[okidx])
            pairs = tree.query_pairs(dmin * (1.0 - 1e-12), output_type="ndarray")
            if pairs.size:
                # exact re-check of the distance criterion
                a = okidx[pairs[:, 0]]
                b = okidx[pairs[:, 1]]
                lo_ = np.minimum(a, b)
                hi_ = np.maximum(a, b)
                dd = np.sum((cand[lo_] - cand[hi_]) ** 2, axis=1)
                sel = dd < d2
                lo_ = lo_[sel]
                hi_ = hi_[sel]
                order = np.argsort(hi_, kind="stable")
                for t in order:
                    if ok[lo_[t]]:
                        ok[hi_[t]] = False
        acc = np.where(ok)[0][: n - count]
        for t in acc:  # insert accepted candidates into the grid
            c0, c1, c2 = ci[t]
            f = fill[c0, c1, c2]
            grid[c0, c1, c2, f] = count
            fill[c0, c1, c2] = f + 1
            out[count] = cand[t]
            count += 1
    box = (np.zeros(3), np.full(3, side))
    return out, box


def sphere_cut(n, lattice_side, seed=None):
    """The n sites of a lattice_side^3 lattice nearest its centre, ordered by the
    doubled-coordinate squared distance and then by linear index."""
    L = lattice_side
    i, j, k = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    k = k.ravel()
    d2 = (2 * i - (L - 1)) ** 2 + (2 * j - (L - 1)) ** 2 + (2 * k - (L - 1)) ** 2
    lin = (i * L + j) * L + k
    order = np.lexsort((lin, d2))[:n]
    order = np.sort(order)
    pos = np.stack([i[order], j[order], k[order]], axis=1).astype(np.float64)
    box = (np.full(3, -0.5), np.full(3, L - 0.5))
    return pos, box


def aligned_moments(n, nbatch, seed_base):
    """Batch of nbatch configurations: configuration b has round(f_b * n) seeded
    sites set to +z (f_b = 0.5*b/(nbatch-1)), the rest random on the sphere.
    Returns (nbatch, n, 3)."""
    out = np.empty((nbatch, n, 3))
    for b in range(nbatch):
        rng = np.random.default_rng(seed_base + b)
        m = unit_moments(n, rng)
        f = 0.5 * b / max(1, nbatch - 1)
        na = int(round(f * n))
        if na:
            sel = rng.permutation(n)[:na]
            m[sel] = np.array([0.0, 0.0, 1.0])
        out[b] = m
    return out


def clusters(nclusters, per_cluster, seed, sigma=8.0, box_side=512.0, margin=24.0):
    """Gaussian clusters: centres uniform in [margin, side-margin)^3, points
    N(centre, sigma^2 I); points outside [0, side)^3 are redrawn."""
    rng = np.random.default_rng(seed)
    centers = margin + rng.random((nclusters, 3)) * (box_side - 2 * margin)
    pos = np.repeat(centers, per_cluster, axis=0) + sigma * rng.standard_normal((nclusters * per_cluster, 3))
    while True:
        bad = np.where(np.any((pos < 0.0) | (pos >= box_side), axis=1))[0]
        if bad.size == 0:
            break
        cidx = bad // per_cluster
        pos[bad] = centers[cidx] + sigma * rng.standard_normal((bad.size, 3))
    box = (np.zeros(3), np.full(3, box_side))
    return pos, box


def film_with_holes(nx, ny, nz, nholes, seed, rmin=20.0, rmax=80.0):
    """nx*ny*nz lattice with nholes circular holes through all layers: holes
    have centres uniform in the plane of the film and radii U[rmin, rmax]; a
    site is removed if its in-plane distance to a hole centre is <= the radius."""
    rng = np.random.default_rng(seed)
    cx = -0.5 + rng.random(nholes) * nx
    cy = -0.5 + rng.random(nholes) * ny
    rad = rmin + rng.random(nholes) * (rmax - rmin)
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    keep = np.ones((nx, ny), dtype=bool)
    for h in range(nholes):
        keep &= (ix - cx[h]) ** 2 + (iy - cy[h]) ** 2 > rad[h] ** 2
    kx, ky = np.where(keep)
    nk = kx.size
    pos = np.empty((nk * nz, 3))
    for z in range(nz):
        pos[z::nz, 0] = kx
        pos[z::nz, 1] = ky
        pos[z::nz, 2] = z
    box = (np.array([-0.5, -0.5, -0.5]), np.array([nx - 0.5, ny - 0.5, nz - 0.5]))
    return pos, box


# ---------------------------------------------------------------------------
# The five workloads at full size, and small versions of the same recipes.
# ---------------------------------------------------------------------------

def config_lattice_1000():
    """10x10x10 lattice, spacing 1, p=4, theta=0.5, s=8 (seed 1001)."""
    pos, box = lattice(10, 10, 10)
    m = random_moments(pos.shape[0], 1001)
    return dict(name="lattice_10x10x10", pos=pos, box=box, m=m[None], order=4, theta=0.5,
                leaf_target=8.0)


def config_ferrofluid(n=1 << 20, pos_seed=2001, mom_seed=2002):
    """Ferrofluid, RSA at volume fraction 0.1, p=6, theta=0.5, s=s_o(6)."""
    pos, box = ferrofluid(n, pos_seed)
    m = random_moments(n, mom_seed)
    return dict(name="ferrofluid_%d" % n, pos=pos, box=box, m=m[None], order=6, theta=0.5,
                leaf_target=0.0)


def config_sphere(n=1 << 18, lattice_side=80, nbatch=64, seed_base=3000):
    """Sphere cut from a cubic lattice, nbatch aligned/random configurations, p=5."""
    pos, box = sphere_cut(n, lattice_side)
    m = aligned_moments(n, nbatch, seed_base)
    return dict(name="sphere_%d_x%d" % (n, nbatch), pos=pos, box=box, m=m, order=5, theta=0.5,
                leaf_target=0.0)


def config_clusters(nclusters=256, per_cluster=8192, pos_seed=4001, mom_seed=4002, box_side=512.0):
    pos, box = clusters(nclusters, per_cluster, pos_seed, box_side=box_side)
    m = random_moments(pos.shape[0], mom_seed)
    return dict(name="clusters_%dx%d" % (nclusters, per_cluster), pos=pos, box=box, m=m[None],
                order=6, theta=0.4, leaf_target=0.0)


def config_film(nx=1024, ny=1024, nz=16, nholes=16, hole_seed=5001, mom_seed_base=5002, nbatch=8):
    pos, box = film_with_holes(nx, ny, nz, nholes, hole_seed)
    n = pos.shape[0]
    m = np.stack([random_moments(n, mom_seed_base + b) for b in range(nbatch)])
    return dict(name="film_%dx%dx%d_holes%d_x%d" % (nx, ny, nz, nholes, nbatch), pos=pos, box=box,
                m=m, order=6, theta=0.4, leaf_target=0.0)


def config_film_training(seed, nx=1024, ny=1024, nz=16, nholes=16):
    """Training geometry for the learned selector on films: the film recipe at
    full size with other seeds (holes from `seed`, moments from seed + 1), so
    its tree has the same depth and smallest-cell shape (2 x 4 x 4 sites) as
    the film it serves; it is labelled on a sample of its cells."""
    pos, box = film_with_holes(nx, ny, nz, nholes, seed)
    m = random_moments(pos.shape[0], seed + 1)
    return dict(name="film_train_%d" % seed, pos=pos, box=box, m=m[None], order=6, theta=0.4, leaf_target=0.0)


def config_clusters_training(seed, nclusters=32, per_cluster=8192, box_side=256.0):
    """Training geometry for the learned selector: the cluster recipe on a box
    of half the side with 1/8 of the clusters.  The smallest cells then have
    the same shape (8 x 16 x 16 at s = s_o(6)) and the clusters the same
    density as in the 2^21-dipole geometry."""
    pos, box = clusters(nclusters, per_cluster, seed, box_side=box_side)
    m = random_moments(pos.shape[0], seed + 1)
    return dict(name="clusters_train_%d" % seed, pos=pos, box=box, m=m[None], order=6, theta=0.4,
                leaf_target=0.0)
