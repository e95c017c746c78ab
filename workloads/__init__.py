"""Seeded synthetic inputs for the SRHD step and the conversions.

This module is shared by the tests, the smoke check and the benchmark.  It only draws random
numbers and lays out primitive states (rho, Ux, Uy, Uz, p) and patch geometry; it holds none of
the method's arithmetic (no EoS, no conversion, no flux).  Conversion to conserved variables is
done by whichever side consumes the input (the CPU oracle in tests, the HIP library in the
benchmark).

Conventions: the box is [0, 1)^3 with base cell size dh0 = 1 / N_base; patch (px, py, pz) of
level l covers cells [8 px, 8 px + 8) x ... of the level-l grid (cell size dh0 / 2^l).  Patch
arrays are [patch][field][z][y][x]; field order (rho, Ux, Uy, Uz, p) for primitives.

Workloads (seeds are numpy PCG64 ``default_rng(seed)``):
  * shock tube, 32^3 (64 patches, outflow): left rho=1, p=1e3; right rho=1, p=1e-6; U=0;
    rho *= 1 + 1e-4 xi, xi ~ U[-1, 1)  (seed 1001)
  * conversion batch: rho log-U[1e-6, 1e6], Theta log-U[1e-8, 1e4], gamma log-U[1, 1e6],
    isotropic direction, p = rho Theta  (seed 1002)
  * blast wave, 256^3 periodic (32768 patches): ambient rho=1, Theta=1e-6; off-centre ellipsoid
    (semi-axes 0.05, 0.03, 0.03) at a seeded random rotation with rho=1e-2, p=1e4  (seed 1003)
  * jet on a multi-level patch list: 4 levels with 5/10/25/60 % of the patches; nozzle
    gamma=1e3, rho=1e-4, Theta=1e2 inside r < 0.02 near z = 0; ambient rho=1, Theta=1e-6;
    ghost cells evaluated from the same analytic state (seed 1005)
"""
import numpy as np

PS = 8


# ----------------------------------------------------------------------------- patch geometry
def neighbor_table(nx, ny, nz, periodic):
    """Neighbour table [P][27] of an nx*ny*nz block of same-level patches.

    Slot (oz+1)*9 + (oy+1)*3 + (ox+1) holds the patch at offset (ox, oy, oz); slot 13 is the
    patch's own index.  Outside a non-periodic box the entry is -1.  Patch id = (pz*ny + py)*nx + px.
    """
    P = nx * ny * nz
    nb = np.full((P, 27), -1, dtype=np.int32)
    pz, py, px = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pz, py, px = pz.ravel(), py.ravel(), px.ravel()
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                qx, qy, qz = px + ox, py + oy, pz + oz
                if periodic:
                    qx, qy, qz = qx % nx, qy % ny, qz % nz
                    ok = np.ones(P, dtype=bool)
                else:
                    ok = (qx >= 0) & (qx < nx) & (qy >= 0) & (qy < ny) & (qz >= 0) & (qz < nz)
                slot = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)
                nb[ok, slot] = ((qz * ny + qy) * nx + qx)[ok]
    return nb


def patch_cell_centres(nx, ny, nz, dh):
    """Cell-centre coordinates of every interior cell, shaped [P][8][8][8] each (x, y, z)."""
    pz, py, px = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pz, py, px = pz.ravel(), py.ravel(), px.ravel()
    c = np.arange(PS)
    x = (px[:, None, None, None] * PS + c[None, None, None, :] + 0.5) * dh
    y = (py[:, None, None, None] * PS + c[None, None, :, None] + 0.5) * dh
    z = (pz[:, None, None, None] * PS + c[None, :, None, None] + 0.5) * dh
    shape = (px.size, PS, PS, PS)
    return np.broadcast_to(x, shape), np.broadcast_to(y, shape), np.broadcast_to(z, shape)


def interior_to_grid(a, nx, ny, nz):
    """[P][F][8][8][8] patch-ordered cells -> [F][8nz][8ny][8nx] uniform grid."""
    F = a.shape[1]
    g = a.reshape(nz, ny, nx, F, PS, PS, PS).transpose(3, 0, 4, 1, 5, 2, 6)
    return g.reshape(F, nz * PS, ny * PS, nx * PS)


def grid_to_interior(g, nx, ny, nz):
    """[F][8nz][8ny][8nx] uniform grid -> [P][F][8][8][8] patch order."""
    F = g.shape[0]
    a = g.reshape(F, nz, PS, ny, PS, nx, PS).transpose(1, 3, 5, 0, 2, 4, 6)
    return np.ascontiguousarray(a.reshape(nz * ny * nx, F, PS, PS, PS))


def morton_order(nx, ny, nz):
    """Permutation of lexicographic patch ids ((pz*ny + py)*nx + px) into Z-order."""
    pz, py, px = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    key = np.zeros(pz.size, dtype=np.int64)
    for bit in range(21):
        for k, c in enumerate((px.ravel(), py.ravel(), pz.ravel())):
            key |= ((c >> bit) & 1).astype(np.int64) << (3 * bit + k)
    return np.argsort(key, kind="stable")


class PatchGrid:
    """A uniform single-level block of patches with its primitive initial state.

    With order="morton" the patches are stored along a Z-order curve (neighbour table and all
    per-patch arrays permuted consistently); `lex_index[i]` is the lexicographic id of patch i."""

    def __init__(self, name, prim, nx, ny, nz, periodic, dh, extra=None, order="lex"):
        self.name = name
        self.prim = prim                # [P][5][8][8][8] float64
        self.nx, self.ny, self.nz = nx, ny, nz
        self.periodic = periodic
        self.dh = dh
        self.neighbor = neighbor_table(nx, ny, nz, periodic)
        self.level = None
        self.dh_lev = np.array([dh])
        self.extra = extra or {}
        self.lex_index = np.arange(prim.shape[0])
        if order == "morton":
            perm = morton_order(nx, ny, nz)
            inv = np.empty_like(perm)
            inv[perm] = np.arange(perm.size)
            self.prim = np.ascontiguousarray(prim[perm])
            nb = self.neighbor[perm]
            self.neighbor = np.where(nb >= 0, inv[np.maximum(nb, 0)], -1).astype(np.int32)
            self.lex_index = perm
            for k, v in list(self.extra.items()):
                if isinstance(v, np.ndarray) and v.shape[:1] == (perm.size,):
                    self.extra[k] = np.ascontiguousarray(v[perm])
        elif order != "lex":
            raise ValueError(order)

    @property
    def n_patch(self):
        return self.prim.shape[0]


# ----------------------------------------------------------------------------- workloads
def shock_tube_32(seed=1001):
    """Relativistic shock tube along x on 32^3 cells (4x4x4 patches), outflow boundaries."""
    n = 4
    x, _, _ = patch_cell_centres(n, n, n, 1.0 / 32)
    rng = np.random.default_rng(seed)
    P = n ** 3
    prim = np.zeros((P, 5, PS, PS, PS))
    left = x < 0.5
    xi = rng.uniform(-1.0, 1.0, size=(P, PS, PS, PS))
    prim[:, 0] = 1.0 * (1.0 + 1e-4 * xi)
    prim[:, 4] = np.where(left, 1e3, 1e-6)
    return PatchGrid("shock_tube_32", prim, n, n, n, False, 1.0 / 32)


def conversion_batch(n, seed=1002, chunk=None):
    """Primitive states [5][n] spanning rho 1e-6..1e6, Theta 1e-8..1e4, gamma 1..1e6.

    With ``chunk=(start, count)`` only that slice is drawn, from the sub-stream seeded by
    (seed, start // 2**20) so that slices are reproducible independently of each other.
    """
    if chunk is None:
        rng = np.random.default_rng(seed)
        m = n
    else:
        start, m = chunk
        rng = np.random.default_rng([seed, start // (1 << 20)])
    lrho = rng.uniform(np.log(1e-6), np.log(1e6), size=m)
    lth = rng.uniform(np.log(1e-8), np.log(1e4), size=m)
    lgam = rng.uniform(0.0, np.log(1e6), size=m)
    dirn = rng.standard_normal(size=(3, m))
    rho = np.exp(lrho)
    th = np.exp(lth)
    gam = np.exp(lgam)
    dirn /= np.sqrt((dirn * dirn).sum(axis=0))
    U = np.sqrt((gam - 1.0) * (gam + 1.0))
    prim = np.empty((5, m))
    prim[0] = rho
    prim[1:4] = U * dirn
    prim[4] = rho * th
    return prim


def conversion_batch_chunks(n, seed=1002, chunk=1 << 20):
    """Yield (start, prim [5][count]) slices of the conversion batch of total size n."""
    start = 0
    while start < n:
        m = min(chunk, n - start)
        yield start, conversion_batch(n, seed, chunk=(start, m))
        start += m


def random_rotation(rng):
    """Uniform random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.sqrt((q * q).sum())
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def blast_labels(n_cells, seed=1003, semi=(0.05, 0.03, 0.03)):
    """Source mask of the off-centre rotated ellipsoid on an n_cells^3 periodic grid.

    Returns (labels [P][8][8][8] uint8 with 1 inside the source, geometry dict)."""
    rng = np.random.default_rng(seed)
    R = random_rotation(rng)
    v = rng.standard_normal(3)
    centre = 0.5 + 0.1 * v / np.sqrt((v * v).sum())
    n = n_cells // PS
    dh = 1.0 / n_cells
    x, y, z = patch_cell_centres(n, n, n, dh)
    rel = np.stack([x - centre[0], y - centre[1], z - centre[2]], axis=-1)
    body = rel @ R  # coordinates along the ellipsoid axes (columns of R)
    a = np.asarray(semi)
    inside = ((body / a) ** 2).sum(axis=-1) <= 1.0
    return inside.astype(np.uint8), {"rotation": R, "centre": centre, "semi": a}


BLAST_AMBIENT = (1.0, 0.0, 0.0, 0.0, 1e-6)     # rho=1, Theta=1e-6
BLAST_SOURCE = (1e-2, 0.0, 0.0, 0.0, 1e4)      # rho=1e-2, p=1e4 (Theta=1e6)


def blast(n_cells=256, seed=1003, order="lex"):
    """Off-centre ellipsoidal blast wave on n_cells^3 periodic cells (256^3 = 32768 patches)."""
    labels, geo = blast_labels(n_cells, seed)
    table = np.array([BLAST_AMBIENT, BLAST_SOURCE])
    n = n_cells // PS
    prim = np.ascontiguousarray(table[labels].transpose(0, 4, 1, 2, 3))
    g = PatchGrid("blast_%d" % n_cells, prim, n, n, n, True, 1.0 / n_cells,
                  extra=dict(geo, labels=labels, table=table), order=order)
    return g


def sine_wave(n_cells, theta0, amp=1e-6, seed=None):
    """Diagonal sinusoidal density perturbation on a static background (periodic).

    rho = 1 + amp sin(2 pi (x + y + z)), p = rho0 * theta0 (uniform), U = 0; the acoustic
    eigenvector is not imposed here (the test builds the velocity/pressure perturbation)."""
    n = n_cells // PS
    x, y, z = patch_cell_centres(n, n, n, 1.0 / n_cells)
    phase = 2.0 * np.pi * (x + y + z)
    P = n ** 3
    prim = np.zeros((P, 5, PS, PS, PS))
    prim[:, 0] = 1.0 + amp * np.sin(phase)
    prim[:, 4] = theta0
    return PatchGrid("sine_%d" % n_cells, prim, n, n, n, True, 1.0 / n_cells,
                     extra={"phase": phase})


def riemann_1d(n_cells_x, left, right, x0=0.5, length=1.0, ny=1, nz=1):
    """1D Riemann problem along x laid out as a row of patches (ny, nz patches across, outflow).

    left/right are primitive tuples (rho, Ux, Uy, Uz, p)."""
    n = n_cells_x // PS
    dh = length / n_cells_x
    x, _, _ = patch_cell_centres(n, ny, nz, dh)
    P = n * ny * nz
    prim = np.empty((P, 5, PS, PS, PS))
    L = np.asarray(left, dtype=np.float64)
    Rr = np.asarray(right, dtype=np.float64)
    for k in range(5):
        prim[:, k] = np.where(x < x0, L[k], Rr[k])
    return PatchGrid("riemann_%d" % n_cells_x, prim, n, ny, nz, False, dh,
                     extra={"x": np.ascontiguousarray(x)})


def jet_block(n_cells=32, seed=1006, radius=0.2, z_top=0.6, amp=1e-3):
    """The jet's two states (jet_states) on a small outflow block: the nozzle state inside a
    cylinder of the given radius around the z axis through the block centre, for z < z_top, the
    ambient state elsewhere; every density multiplied by 1 + amp xi, xi ~ U[-1, 1).  A small
    stand-in for the nozzle region of the jet patch list, with non-uniform nozzle cells."""
    n = n_cells // PS
    dh = 1.0 / n_cells
    x, y, z = patch_cell_centres(n, n, n, dh)
    st = jet_states()
    inside = ((x - 0.5) ** 2 + (y - 0.5) ** 2 < radius * radius) & (z < z_top)
    prim = np.ascontiguousarray(np.moveaxis(st[inside.astype(np.int64)], -1, 1))
    rng = np.random.default_rng(seed)
    prim[:, 0] *= 1.0 + amp * rng.uniform(-1.0, 1.0, size=prim[:, 0].shape)
    return PatchGrid("jet_block_%d" % n_cells, prim, n, n, n, False, dh,
                     extra={"labels": inside.astype(np.uint8)})


def moving_gas(n_cells=32, U=3.0, theta=1e-2, amp=1e-3, seed=1007):
    """Uniform flow of four-velocity magnitude U along (1, 1, 1) / sqrt(3) at temperature theta
    (rho = 1) on a periodic block, with rho and p each multiplied by an independent 1 + amp xi,
    xi ~ U[-1, 1)."""
    n = n_cells // PS
    P = n ** 3
    rng = np.random.default_rng(seed)
    prim = np.empty((P, 5, PS, PS, PS))
    prim[:, 0] = 1.0 + amp * rng.uniform(-1.0, 1.0, size=(P, PS, PS, PS))
    prim[:, 1:4] = U / np.sqrt(3.0)
    prim[:, 4] = theta * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(P, PS, PS, PS)))
    return PatchGrid("moving_gas_%d" % n_cells, prim, n, n, n, True, 1.0 / n_cells)


# ----------------------------------------------------------------------------- two AMR levels
def two_level(nc, lo, hi):
    """Geometry of a periodic two-level patch hierarchy (refinement ratio 2).

    Level 0: nc^3 patches (lexicographic ids, cell size 1 / (8 nc)).  The coarse patches
    [lo, hi)^3 (strictly inside the box) are refined: each has eight children on level 1, which
    form an nf^3 block of fine patches, nf = 2 (hi - lo), fine id ((fz nf) + fy) nf + fx relative
    to the block.  Returns a dict with
      coarse_neighbor [Pc][27]        same-level table (periodic)
      fine_neighbor   [Pf][27]        fine ids inside the block, -2 where level 0 covers the slot
      parent, octant  [Pf]            coarse id of the parent; child position bx | by<<1 | bz<<2
      parent_of [Pr], child [Pr][8]   refined coarse ids and their children (for restriction)
      faces [Nf][6]                   (coarse id, side 2 d + u, fine[4]) for every face of an
                                      unrefined coarse patch that touches a refined one; fine[t]
                                      covers the face cells (a, b) with t = (a >= 4) + 2 (b >= 4)
      refined [Pc] bool, dh_c, dh_f, coarse_xyz, fine_xyz (cell centres [P][8][8][8] each)
    """
    assert 0 < lo < hi < nc
    nf = 2 * (hi - lo)
    cnb = neighbor_table(nc, nc, nc, True)
    cid = lambda x, y, z: ((z % nc) * nc + (y % nc)) * nc + (x % nc)
    refined = np.zeros(nc ** 3, dtype=bool)
    for z in range(lo, hi):
        for y in range(lo, hi):
            for x in range(lo, hi):
                refined[cid(x, y, z)] = True
    Pf = nf ** 3
    fid = lambda x, y, z: ((z - 2 * lo) * nf + (y - 2 * lo)) * nf + (x - 2 * lo)
    inside = lambda x, y, z: all(2 * lo <= v < 2 * hi for v in (x, y, z))
    fnb = np.full((Pf, 27), -2, dtype=np.int32)
    parent = np.empty(Pf, dtype=np.int32)
    octant = np.empty(Pf, dtype=np.int8)
    fxyz = np.empty((Pf, 3), dtype=np.int64)
    for fz in range(2 * lo, 2 * hi):
        for fy in range(2 * lo, 2 * hi):
            for fx in range(2 * lo, 2 * hi):
                i = fid(fx, fy, fz)
                fxyz[i] = (fx, fy, fz)
                parent[i] = cid(fx // 2, fy // 2, fz // 2)
                octant[i] = (fx & 1) | ((fy & 1) << 1) | ((fz & 1) << 2)
                for oz in (-1, 0, 1):
                    for oy in (-1, 0, 1):
                        for ox in (-1, 0, 1):
                            q = (fx + ox, fy + oy, fz + oz)
                            if inside(*q):
                                fnb[i, (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)] = fid(*q)
    parent_of = np.flatnonzero(refined).astype(np.int32)
    child = np.empty((parent_of.size, 8), dtype=np.int32)
    for k, P in enumerate(parent_of):
        px, py, pz = P % nc, (P // nc) % nc, P // (nc * nc)
        for o in range(8):
            child[k, o] = fid(2 * px + (o & 1), 2 * py + ((o >> 1) & 1), 2 * pz + ((o >> 2) & 1))
    faces = []
    for P in np.flatnonzero(~refined):
        c = [P % nc, (P // nc) % nc, P // (nc * nc)]
        for d in range(3):
            for u in (0, 1):
                q = list(c)
                q[d] += 1 if u else -1
                Q = cid(*q)
                if not refined[Q]:
                    continue
                qx, qy, qz = q[0] % nc, q[1] % nc, q[2] % nc
                t0, t1 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
                fine = []
                for t in range(4):
                    bits = [0, 0, 0]
                    bits[d] = 0 if u else 1                 # the children on P's side of Q
                    bits[t0], bits[t1] = t & 1, t >> 1
                    fine.append(fid(2 * qx + bits[0], 2 * qy + bits[1], 2 * qz + bits[2]))
                faces.append([P, 2 * d + u] + fine)
    dh_c = 1.0 / (8 * nc)
    cx, cy, cz = patch_cell_centres(nc, nc, nc, dh_c)
    dh_f = dh_c / 2
    c = np.arange(PS)
    fx = (fxyz[:, 0, None, None, None] * PS + c[None, None, None, :] + 0.5) * dh_f
    fy = (fxyz[:, 1, None, None, None] * PS + c[None, None, :, None] + 0.5) * dh_f
    fz = (fxyz[:, 2, None, None, None] * PS + c[None, :, None, None] + 0.5) * dh_f
    shape = (Pf, PS, PS, PS)
    return {"coarse_neighbor": cnb, "fine_neighbor": fnb, "parent": parent, "octant": octant,
            "parent_of": parent_of, "child": child, "faces": np.array(faces, dtype=np.int32),
            "refined": refined, "dh_c": dh_c, "dh_f": dh_f, "nc": nc, "nf": nf,
            "coarse_xyz": (cx, cy, cz),
            "fine_xyz": tuple(np.broadcast_to(v, shape) for v in (fx, fy, fz))}


# ----------------------------------------------------------------------------- jet patch list
def jet_states():
    """Nozzle and ambient primitive states of the jet workload."""
    gam = 1e3
    Uz = np.sqrt((gam - 1.0) * (gam + 1.0))
    jet = (1e-4, 0.0, 0.0, Uz, 1e-4 * 1e2)
    amb = (1.0, 0.0, 0.0, 0.0, 1e-6)
    return np.array([amb, jet])


def jet_patch_list(n_patch=400_000, n_base=256, fractions=(0.05, 0.10, 0.25, 0.60),
                   seed=1005, r_jet=0.02, z_jet=0.04):
    """Multi-level patch list around a jet along +z from the z = 0 face.

    Level l has the patch lattice of a (n_base 2^l)^3 grid; its patches are the ones whose
    centres lie nearest (in a seeded jittered distance) to the jet axis segment.  Returns a dict
    with corner [P][3] (integer cell coordinates of the patch origin on its level), level [P]
    (int8) and dh_lev [4]."""
    rng = np.random.default_rng(seed)
    counts = [int(round(f * n_patch)) for f in fractions]
    counts[-1] = n_patch - sum(counts[:-1])
    corners, levels = [], []
    for lv, cnt in enumerate(counts):
        npl = (n_base << lv) // PS            # patches per side on this level
        # candidate patches in a cylinder around the axis; enough of them to choose from
        r_need = np.sqrt(cnt / (np.pi * npl)) / npl * 1.6 + 2.0 / npl
        r_need = min(r_need, 0.5)
        lo = max(0, int(np.floor((0.5 - r_need) * npl)))
        hi = min(npl, int(np.ceil((0.5 + r_need) * npl)))
        ix = np.arange(lo, hi)
        gx, gy = np.meshgrid(ix, ix, indexing="ij")
        cx = (gx + 0.5) / npl - 0.5
        cy = (gy + 0.5) / npl - 0.5
        rr = np.sqrt(cx * cx + cy * cy).ravel()
        gx, gy = gx.ravel(), gy.ravel()
        nzp = npl
        # all (x, y, z) candidates: distance to axis plus a z penalty favouring the nozzle end
        zz = np.arange(nzp)
        score = rr[:, None] + 0.25 * (zz[None, :] + 0.5) / nzp
        score = score + 0.02 * rng.random(score.shape) / npl
        if score.size < cnt:
            raise ValueError("level %d holds %d candidate patches, %d requested" % (lv, score.size, cnt))
        flat = np.argsort(score, axis=None, kind="stable")[:cnt]
        a, b = np.unravel_index(flat, score.shape)
        c = np.stack([gx[a], gy[a], zz[b]], axis=1) * PS
        corners.append(c.astype(np.int64))
        levels.append(np.full(cnt, lv, dtype=np.int8))
    corner = np.concatenate(corners)
    level = np.concatenate(levels)
    dh0 = 1.0 / n_base
    dh_lev = dh0 / (2.0 ** np.arange(len(fractions)))
    return {"corner": corner, "level": level, "dh_lev": dh_lev, "n_base": n_base,
            "r_jet": r_jet, "z_jet": z_jet}


def jet_labels(pl, patches=None, ghost=3):
    """Label of every padded cell (0 ambient, 1 nozzle) of the selected patches [p][N][N][N].

    Membership uses the cell centre: r < r_jet and z < z_jet."""
    corner, level = pl["corner"], pl["level"]
    idx = np.arange(corner.shape[0]) if patches is None else np.asarray(patches)
    N = PS + 2 * ghost
    o = np.arange(-ghost, PS + ghost)
    out = np.empty((idx.size, N, N, N), dtype=np.uint8)
    for s in range(0, idx.size, 4096):
        sel = idx[s:s + 4096]
        dh = pl["dh_lev"][level[sel]][:, None]
        cx = (corner[sel, 0][:, None] + o[None, :] + 0.5) * dh - 0.5
        cy = (corner[sel, 1][:, None] + o[None, :] + 0.5) * dh - 0.5
        cz = (corner[sel, 2][:, None] + o[None, :] + 0.5) * dh
        r2 = cx[:, None, None, :] * cx[:, None, None, :] + cy[:, None, :, None] * cy[:, None, :, None]
        inside = (r2 < pl["r_jet"] * pl["r_jet"]) & (cz[:, :, None, None] < pl["z_jet"])
        out[s:s + sel.size] = inside
    return out


def jet_labels_torch(pl, device, ghost=3, chunk=16384):
    """jet_labels of every patch, computed on a torch device with the same IEEE operations in
    the same order (so the labels equal jet_labels' bit for bit)."""
    import torch
    corner = torch.as_tensor(pl["corner"], device=device)
    level = torch.as_tensor(pl["level"].astype(np.int64), device=device)
    dh_lev = torch.as_tensor(pl["dh_lev"], dtype=torch.float64, device=device)
    P = corner.shape[0]
    N = PS + 2 * ghost
    o = torch.arange(-ghost, PS + ghost, device=device)
    r2max = pl["r_jet"] * pl["r_jet"]
    out = torch.empty((P, N, N, N), dtype=torch.uint8, device=device)
    for s in range(0, P, chunk):
        sl = slice(s, min(P, s + chunk))
        dh = dh_lev[level[sl]][:, None]
        cx = ((corner[sl, 0][:, None] + o[None, :]).double() + 0.5) * dh - 0.5
        cy = ((corner[sl, 1][:, None] + o[None, :]).double() + 0.5) * dh - 0.5
        cz = ((corner[sl, 2][:, None] + o[None, :]).double() + 0.5) * dh
        r2 = cx[:, None, None, :] * cx[:, None, None, :] + cy[:, None, :, None] * cy[:, None, :, None]
        out[sl] = ((r2 < r2max) & (cz[:, :, None, None] < pl["z_jet"])).to(torch.uint8)
    return out


def assemble_labeled(labels, states):
    """Padded patches [p][5][N][N][N] whose cell c holds states[labels[c]] (states [k][5]).

    Works on numpy arrays or torch tensors (labels uint8, states float64); a pure selection."""
    if isinstance(labels, np.ndarray):
        st = np.asarray(states, dtype=np.float64)
        return np.ascontiguousarray(np.moveaxis(st[labels.astype(np.int64)], -1, 1))
    import torch
    st = torch.as_tensor(np.asarray(states, dtype=np.float64), device=labels.device)
    P = labels.shape[0]
    out = torch.empty((P, 5) + tuple(labels.shape[1:]), dtype=torch.float64, device=labels.device)
    chunk = 8192
    for s in range(0, P, chunk):
        lab = labels[s:s + chunk].long()
        for f in range(5):
            out[s:s + chunk, f] = st[:, f][lab]
    return out
