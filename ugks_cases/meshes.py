"""Unstructured meshes stored as face lists.

A mesh is the input the scheme's finite-volume partition needs (the control
volumes Omega_i, the interface areas S_ij, unit normals n_ij and neighbour
sets N(i) of Sec. 2.1, Eqs. (physical_partition) and (fv_micro_update)):

* ``cell_volume[i]``, ``cell_centroid[i]``
* ``face_cells[f] = (L, R)`` with ``R = -1`` on a physical boundary
* ``face_area[f]``, ``face_normal[f]`` (unit, pointing from L to R, i.e.
  outward from L on a boundary), ``face_centroid[f]`` (as seen from L)
* ``face_shift[f]``: for a periodic face, the translation that carries R's
  centroid next to L (R's image is ``cell_centroid[R] + face_shift[f]``)
* ``face_bc[f]`` (0 interior/periodic, 1 wall, 2 far field, 3 outflow) and
  ``face_bc_id[f]`` (row of the boundary-condition table, -1 for interior)

Everything here is geometry of the input; none of it is the scheme.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

BC_INTERIOR, BC_WALL, BC_FARFIELD, BC_OUTFLOW = 0, 1, 2, 3


@dataclass
class Mesh:
    dim: int
    cell_volume: np.ndarray
    cell_centroid: np.ndarray
    face_cells: np.ndarray
    face_area: np.ndarray
    face_normal: np.ndarray
    face_centroid: np.ndarray
    face_shift: np.ndarray
    face_bc: np.ndarray
    face_bc_id: np.ndarray
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cell_volume.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_area.shape[0])

    def contiguous(self) -> "Mesh":
        """Return the same mesh with every array C-contiguous and typed."""
        f8 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        return Mesh(
            dim=int(self.dim),
            cell_volume=f8(self.cell_volume),
            cell_centroid=f8(self.cell_centroid.reshape(-1, self.dim)),
            face_cells=np.ascontiguousarray(self.face_cells, dtype=np.int64).reshape(-1, 2),
            face_area=f8(self.face_area),
            face_normal=f8(self.face_normal.reshape(-1, self.dim)),
            face_centroid=f8(self.face_centroid.reshape(-1, self.dim)),
            face_shift=f8(self.face_shift.reshape(-1, self.dim)),
            face_bc=np.ascontiguousarray(self.face_bc, dtype=np.int32),
            face_bc_id=np.ascontiguousarray(self.face_bc_id, dtype=np.int32),
            name=self.name,
            extra=dict(self.extra),
        )

    def validate(self, tol: float = 1e-12) -> None:
        """Raise ValueError unless the face list describes a closed, oriented mesh.

        Checks: positive volumes and areas; unit normals; valid cell indices;
        interior faces join two distinct cells with the normal pointing from L
        towards R's (possibly shifted) centroid; boundary normals point out of
        L; and every cell is closed, sum_j sigma_ij S_j n_j = 0.
        """
        d = self.dim
        nc, nf = self.n_cells, self.n_faces
        if d not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if np.any(self.cell_volume <= 0):
            raise ValueError("non-positive cell volume")
        if np.any(self.face_area <= 0):
            raise ValueError("non-positive face area")
        if np.max(np.abs(np.linalg.norm(self.face_normal, axis=1) - 1.0)) > 1e-12:
            raise ValueError("face normals must be unit vectors")
        L = self.face_cells[:, 0]
        R = self.face_cells[:, 1]
        if np.any(L < 0) or np.any(L >= nc) or np.any(R >= nc) or np.any(R < -1):
            raise ValueError("face_cells out of range")
        interior = self.face_bc == BC_INTERIOR
        if np.any((R < 0) & interior) or np.any((R >= 0) & ~interior):
            raise ValueError("interior faces need R >= 0, boundary faces R = -1")
        if np.any(L[interior] == R[interior]):
            raise ValueError("interior face joins a cell to itself")
        xl = self.cell_centroid[L]
        dn = np.where(
            interior[:, None],
            self.cell_centroid[np.maximum(R, 0)] + self.face_shift - xl,
            self.face_centroid - xl,
        )
        if np.any(np.einsum("fd,fd->f", dn, self.face_normal) <= 0):
            raise ValueError("face normal not oriented from L to R / outward")
        closure = np.zeros((nc, d))
        sn = self.face_area[:, None] * self.face_normal
        np.add.at(closure, L, sn)
        np.add.at(closure, R[interior], -sn[interior])
        scale = np.zeros(nc)
        np.add.at(scale, L, self.face_area)
        np.add.at(scale, R[interior], self.face_area[interior])
        if np.max(np.linalg.norm(closure, axis=1) / scale) > tol * 100:
            raise ValueError("mesh cells are not closed")


def quad_mesh(nx: int, ny: int | None = None, *, lx: float = 1.0, ly: float = 1.0,
              periodic_x: bool = False, periodic_y: bool = False, wall_ids=(0, 1, 2, 3),
              name: str = "") -> Mesh:
    """Uniform nx x ny quadrilateral mesh of [0,lx]x[0,ly] as a face list.

    Cell (i, j) has index i + nx*j.  Boundary tags: ``wall_ids`` gives the BC
    table row of the (bottom y=0, right x=lx, top y=ly, left x=0) sides.  With
    ``periodic_x`` the left/right sides become one periodic seam of interior
    faces (L = last column, R = first column, shift = (+lx, 0)); likewise
    ``periodic_y`` for the bottom/top sides.
    """
    ny = nx if ny is None else ny
    hx, hy = lx / nx, ly / ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    cid = (ii + nx * jj).ravel()
    cen = np.zeros((nx * ny, 2))
    cen[cid, 0] = ((ii + 0.5) * hx).ravel()
    cen[cid, 1] = ((jj + 0.5) * hy).ravel()
    vol = np.full(nx * ny, hx * hy)
    fc, fa, fn, fx, fs, fb, fi = [], [], [], [], [], [], []

    def add(L, R, area, n, x, s=(0.0, 0.0), bc=BC_INTERIOR, bid=-1):
        fc.append((L, R)); fa.append(area); fn.append(n); fx.append(x)
        fs.append(s); fb.append(bc); fi.append(bid)

    c = lambda i, j: i + nx * j  # noqa: E731
    bottom, right, top, left = wall_ids
    for j in range(ny):
        y = (j + 0.5) * hy
        if periodic_x:
            add(c(nx - 1, j), c(0, j), hy, (1.0, 0.0), (lx, y), s=(lx, 0.0))
        else:
            add(c(0, j), -1, hy, (-1.0, 0.0), (0.0, y), bc=BC_WALL, bid=left)
        for i in range(1, nx):
            add(c(i - 1, j), c(i, j), hy, (1.0, 0.0), (i * hx, y))
        if not periodic_x:
            add(c(nx - 1, j), -1, hy, (1.0, 0.0), (lx, y), bc=BC_WALL, bid=right)
    for i in range(nx):
        x = (i + 0.5) * hx
        if periodic_y:
            add(c(i, ny - 1), c(i, 0), hx, (0.0, 1.0), (x, ly), s=(0.0, ly))
        else:
            add(c(i, 0), -1, hx, (0.0, -1.0), (x, 0.0), bc=BC_WALL, bid=bottom)
        for j in range(1, ny):
            add(c(i, j - 1), c(i, j), hx, (0.0, 1.0), (x, j * hy))
        if not periodic_y:
            add(c(i, ny - 1), -1, hx, (0.0, 1.0), (x, ly), bc=BC_WALL, bid=top)
    m = Mesh(2, vol, cen, np.array(fc), np.array(fa), np.array(fn), np.array(fx),
             np.array(fs), np.array(fb), np.array(fi), name=name or f"quad{nx}x{ny}")
    m = m.contiguous()
    m.validate()
    return m


def hex_box(nx: int, ny: int | None = None, nz: int | None = None, *, grading: float = 0.0,
            seed: int = 0, periodic_x: bool = False, name: str = "") -> Mesh:
    """Rectilinear hexahedral mesh of the unit cube, stored as a face list.

    Each axis is cut at nodes 0 < x_1 < ... < 1 whose spacings are
    (1 + grading * U(-1, 1)) times uniform, renormalised (numpy
    ``default_rng(seed)``), so cell volumes differ.  Every cell has six faces
    (rectangles).  Walls get boundary-table rows 0..5 for the sides x=0,
    x=1, y=0, y=1, z=0, z=1, as in kuhn_tet_cube; with ``periodic_x`` the
    sides x=0 and x=1 are instead one periodic seam of interior faces
    (L = last layer, R = first layer, shift (1, 0, 0)).  Cell (i, j, k) has
    index i + nx (j + ny k).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)

    def nodes(n):
        w = 1.0 + grading * rng.uniform(-1.0, 1.0, n)
        return np.concatenate([[0.0], np.cumsum(w / w.sum())[:-1], [1.0]])

    ax = [nodes(nx), nodes(ny), nodes(nz)]
    nn = (nx, ny, nz)
    cid = lambda i, j, k: i + nx * (j + ny * k)  # noqa: E731
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    order = np.argsort(cid(I, J, K).ravel())
    lo = [ax[d][g.ravel()[order]] for d, g in enumerate((I, J, K))]
    hi = [ax[d][g.ravel()[order] + 1] for d, g in enumerate((I, J, K))]
    cen = np.stack([(lo[d] + hi[d]) / 2.0 for d in range(3)], axis=1)
    vol = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
    fc, fa, fn, fx, fs, fb, fi = [], [], [], [], [], [], []
    for d in range(3):
        e1, e2 = [a for a in range(3) if a != d]
        for t in range(nn[d] + 1):
            for b in range(nn[e2]):
                for a in range(nn[e1]):
                    ijk_l = [0, 0, 0]
                    ijk_l[d] = t - 1
                    ijk_l[e1] = a
                    ijk_l[e2] = b
                    ijk_r = list(ijk_l)
                    ijk_r[d] = t
                    x = np.zeros(3)
                    x[d] = ax[d][t]
                    x[e1] = 0.5 * (ax[e1][a] + ax[e1][a + 1])
                    x[e2] = 0.5 * (ax[e2][b] + ax[e2][b + 1])
                    area = (ax[e1][a + 1] - ax[e1][a]) * (ax[e2][b + 1] - ax[e2][b])
                    n = np.zeros(3)
                    shift = np.zeros(3)
                    if periodic_x and d == 0 and t == 0:
                        continue  # the seam is the face at x = 1
                    if periodic_x and d == 0 and t == nn[d]:
                        n[d] = 1.0
                        shift[0] = 1.0
                        ijk_r[0] = 0
                        fc.append((cid(*ijk_l), cid(*ijk_r))); fb.append(BC_INTERIOR); fi.append(-1)
                    elif t == 0:
                        n[d] = -1.0
                        fc.append((cid(*ijk_r), -1)); fb.append(BC_WALL); fi.append(2 * d)
                    elif t == nn[d]:
                        n[d] = 1.0
                        fc.append((cid(*ijk_l), -1)); fb.append(BC_WALL); fi.append(2 * d + 1)
                    else:
                        n[d] = 1.0
                        fc.append((cid(*ijk_l), cid(*ijk_r))); fb.append(BC_INTERIOR); fi.append(-1)
                    fa.append(area); fn.append(n); fx.append(x); fs.append(shift)
    m = Mesh(3, vol, cen, np.array(fc), np.array(fa), np.array(fn), np.array(fx),
             np.array(fs), np.array(fb), np.array(fi),
             name=name or f"hex{nx}x{ny}x{nz}_g{grading}_s{seed}")
    m = m.contiguous()
    m.validate()
    return m


def cylinder_ogrid(n_theta: int = 64, n_r: int = 24, *, r0: float = 1.0, r1: float = 6.0,
                   first: float = 0.05, name: str = "") -> Mesh:
    """2-D O-grid of quadrilaterals around a circular cylinder of radius r0.

    Nodes sit at (r_j cos t_i, r_j sin t_i) with n_theta equal angles and
    n_r radial layers whose thickness grows geometrically from ``first`` so
    the layers end at r1; cells are the straight-edged quads between them.
    The ring closes on itself (cells of angle n_theta-1 and 0 share an
    ordinary interior face).  Boundary tags: row 0 for the wall at r0, row 1
    for the far field at r1.  Cell (i, j) has index i + n_theta j.
    """
    # growth ratio q with first * (q^n - 1)/(q - 1) = r1 - r0
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        tot = first * (q ** n_r - 1.0) / (q - 1.0)
        lo, hi = (q, hi) if tot < r1 - r0 else (lo, q)
    q = 0.5 * (lo + hi)
    rad = np.concatenate([[r0], r0 + first * (q ** np.arange(1, n_r + 1) - 1.0) / (q - 1.0)])
    rad[-1] = r1
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    P = np.stack([np.outer(rad, np.cos(th)), np.outer(rad, np.sin(th))], axis=-1)  # [j, i, 2]
    cid = lambda i, j: (i % n_theta) + n_theta * j  # noqa: E731
    nc = n_theta * n_r
    vol = np.zeros(nc)
    cen = np.zeros((nc, 2))
    for j in range(n_r):
        for i in range(n_theta):
            poly = [P[j, i], P[j + 1, i], P[j + 1, (i + 1) % n_theta], P[j, (i + 1) % n_theta]]
            a = 0.0
            cx = cy = 0.0
            for k in range(4):
                x0, y0 = poly[k]
                x1, y1 = poly[(k + 1) % 4]
                cr = x0 * y1 - x1 * y0
                a += cr
                cx += (x0 + x1) * cr
                cy += (y0 + y1) * cr
            a *= 0.5
            vol[cid(i, j)] = a
            cen[cid(i, j)] = (cx / (6.0 * a), cy / (6.0 * a))
    fc, fa, fn, fx, fb, fi = [], [], [], [], [], []

    def add(L, R, p, q_, bc, bid):
        e = q_ - p
        length = float(np.hypot(e[0], e[1]))
        n = np.array([e[1], -e[0]]) / length  # right-hand normal of p -> q
        x = 0.5 * (p + q_)
        ref = cen[R] if R >= 0 else x
        if np.dot(ref - cen[L], n) < 0:
            n = -n
        fc.append((L, R)); fa.append(length); fn.append(n); fx.append(x); fb.append(bc); fi.append(bid)

    for j in range(n_r):          # radial edges between angular neighbours
        for i in range(n_theta):
            add(cid(i, j), cid(i + 1, j), P[j, (i + 1) % n_theta], P[j + 1, (i + 1) % n_theta],
                BC_INTERIOR, -1)
    for j in range(n_r + 1):      # rings
        for i in range(n_theta):
            p, q_ = P[j, i], P[j, (i + 1) % n_theta]
            if j == 0:
                add(cid(i, 0), -1, p, q_, BC_WALL, 0)
            elif j == n_r:
                add(cid(i, n_r - 1), -1, p, q_, BC_FARFIELD, 1)
            else:
                add(cid(i, j - 1), cid(i, j), p, q_, BC_INTERIOR, -1)
    m = Mesh(2, vol, cen, np.array(fc), np.array(fa), np.array(fn), np.array(fx),
             np.zeros((len(fa), 2)), np.array(fb), np.array(fi),
             name=name or f"cyl{n_theta}x{n_r}_f{first}")
    m = m.contiguous()
    m.validate()
    return m


def _tri_geometry(a, b, c):
    cr = np.cross(b - a, c - a)
    area2 = np.linalg.norm(cr, axis=1)
    return 0.5 * area2, cr / area2[:, None], (a + b + c) / 3.0


def _faces_from_simplices(verts: np.ndarray, tets: np.ndarray):
    """Match the triangular faces of a conforming tet mesh.

    Returns (L, R, tri) with R = -1 for boundary faces, and tri the three vertex
    ids of each face.
    """
    nt = tets.shape[0]
    opp = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tri = tets[:, opp].reshape(-1, 3)
    owner = np.repeat(np.arange(nt), 4)
    key = np.sort(tri, axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("a face is shared by more than two tets")
    Ls, Rs, Ts = [], [], []
    i = 0
    n = ks.shape[0]
    pair_start = np.zeros(n, dtype=bool)
    pair_start[:-1] = same
    is_second = np.zeros(n, dtype=bool)
    is_second[1:] = same
    firsts = np.where(pair_start)[0]
    singles = np.where(~pair_start & ~is_second)[0]
    Ls.append(owner[order[firsts]]); Rs.append(owner[order[firsts + 1]])
    Ts.append(tri[order[firsts]])
    Ls.append(owner[order[singles]]); Rs.append(np.full(singles.size, -1))
    Ts.append(tri[order[singles]])
    del i
    L = np.concatenate(Ls); R = np.concatenate(Rs); T = np.concatenate(Ts)
    # deterministic face order: sort by (min(L,R) for interior, L) then vertex key
    srt = np.lexsort((np.sort(T, axis=1)[:, 2], np.sort(T, axis=1)[:, 1],
                      np.sort(T, axis=1)[:, 0], L))
    return L[srt], R[srt], T[srt]


def _tet_mesh_from_vertices(verts, tets, side_of_face, name, extra=None) -> Mesh:
    """Build a Mesh from tet connectivity; ``side_of_face(centroids)`` tags walls."""
    p = verts[tets]
    vol6 = np.einsum("ti,ti->t", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    if np.any(vol6 <= 0):
        raise ValueError("inverted or degenerate tetrahedron")
    vol = vol6 / 6.0
    cen = p.mean(axis=1)
    L, R, T = _faces_from_simplices(verts, tets)
    area, nrm, fcen = _tri_geometry(verts[T[:, 0]], verts[T[:, 1]], verts[T[:, 2]])
    interior = R >= 0
    d = np.where(interior[:, None], cen[np.maximum(R, 0)] - cen[L], fcen - cen[L])
    flip = np.einsum("fd,fd->f", d, nrm) < 0
    nrm[flip] *= -1.0
    bc = np.where(interior, BC_INTERIOR, BC_WALL).astype(np.int32)
    bid = np.full(L.size, -1, dtype=np.int32)
    if np.any(~interior):
        kind, ids = side_of_face(fcen[~interior])
        bc[~interior] = kind
        bid[~interior] = ids
    m = Mesh(3, vol, cen, np.stack([L, R], axis=1), area, nrm, fcen,
             np.zeros_like(fcen), bc, bid, name=name, extra=extra or {})
    m = m.contiguous()
    m.validate()
    return m


def kuhn_tet_cube(n: int, *, jitter: float = 0.15, seed: int = 0, name: str = "") -> Mesh:
    """Unit cube of n^3 hexes, each split into 6 Kuhn tets along (0,0,0)-(1,1,1).

    Every vertex is moved by a uniform random offset in [-jitter*h, jitter*h]
    per coordinate (numpy ``default_rng(seed)``); a vertex on a boundary plane
    keeps that coordinate, so boundary vertices move only within their face or
    edge and corners stay fixed.  All six walls get boundary-table rows
    0..5 for the sides x=0, x=1, y=0, y=1, z=0, z=1.
    """
    h = 1.0 / n
    g = np.arange(n + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    ijk = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    verts = ijk * h
    if jitter > 0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=verts.shape)
        on_bnd = (ijk == 0) | (ijk == n)
        off[on_bnd] = 0.0
        verts = verts + off
    vid = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k  # noqa: E731
    tets = []
    base = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"),
                    axis=-1).reshape(-1, 3)
    for perm in itertools.permutations(range(3)):
        e = np.eye(3, dtype=np.int64)
        v0 = base
        v1 = v0 + e[perm[0]]
        v2 = v1 + e[perm[1]]
        v3 = v2 + e[perm[2]]
        t = np.stack([vid(*v.T) for v in (v0, v1, v2, v3)], axis=1)
        # orient positively on the unjittered lattice
        p = ijk[t].astype(np.float64)
        s = np.einsum("ti,ti->t", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
        t[s < 0] = t[s < 0][:, [0, 2, 1, 3]]
        tets.append(t)
    # hex-major cell order: the six tets of one hex are consecutive
    tets = np.stack(tets, axis=1).reshape(-1, 4)

    def sides(fc):
        ids = np.full(fc.shape[0], -1, dtype=np.int32)
        for ax in range(3):
            ids[np.abs(fc[:, ax]) < 1e-12] = 2 * ax
            ids[np.abs(fc[:, ax] - 1.0) < 1e-12] = 2 * ax + 1
        if np.any(ids < 0):
            raise ValueError("boundary face not on a cube side")
        return np.full(fc.shape[0], BC_WALL, dtype=np.int32), ids

    return _tet_mesh_from_vertices(verts, tets, sides, name or f"kuhn{n}_j{jitter}_s{seed}")


def cubed_sphere_shell(n_ang: int = 11, n_rad: int = 23, *, r0: float = 1.0, r1: float = 6.0,
                       first: float = 0.02, name: str = "") -> Mesh:
    """Spherical shell r0 <= r <= r1 around a unit sphere, meshed with tets.

    The sphere is split into the six faces of a cube, each gnomonically
    projected and divided into n_ang x n_ang patches; radially there are n_rad
    layers with first thickness ``first`` and a constant growth ratio chosen so
    the layers end at r1.  Each hexahedral (patch x layer) element gets a
    centroid vertex and 12 tets, one per triangle of its quads, each quad cut
    along the diagonal through its smallest global vertex id, so the tets
    conform: 72 n_ang^2 n_rad cells.  Tags: the inner sphere is BC row 0
    (wall), the outer sphere row 1 (far field).
    """
    # radial distribution with geometric growth
    def total(q):
        return first * (q ** n_rad - 1.0) / (q - 1.0)
    lo, hi = 1.0 + 1e-9, 2.0
    target = r1 - r0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    q = 0.5 * (lo + hi)
    radii = r0 + np.concatenate([[0.0], np.cumsum(first * q ** np.arange(n_rad))])
    radii[-1] = r1
    # unique surface vertices of the cube [-1,1]^3 surface lattice
    m = n_ang
    t = np.tan(np.linspace(-np.pi / 4, np.pi / 4, m + 1))  # equiangular
    pts = {}
    quads = []
    def key(v):
        return tuple(np.round(v, 12))
    def vid(v):
        k = key(v)
        if k not in pts:
            pts[k] = len(pts)
        return pts[k]
    faces_def = []
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            faces_def.append((ax, sgn))
    for ax, sgn in faces_def:
        a1, a2 = [x for x in range(3) if x != ax]
        for i in range(m):
            for j in range(m):
                corner = []
                for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    v = np.zeros(3)
                    v[ax] = sgn
                    v[a1] = t[i + di]
                    v[a2] = t[j + dj]
                    corner.append(vid(v))
                quads.append(corner)
    surf = np.zeros((len(pts), 3))
    for k, i in pts.items():
        surf[i] = k
    surf /= np.linalg.norm(surf, axis=1, keepdims=True)
    ns = surf.shape[0]
    verts = (radii[:, None, None] * surf[None, :, :]).reshape(-1, 3)
    gid = lambda layer, s: layer * ns + s  # noqa: E731
    # each hexahedral (patch x layer) element: a centroid vertex and 12 tets,
    # one per triangle of its six quads, every quad cut along the diagonal
    # through its smallest global vertex id (so both hexes sharing a quad cut
    # it the same way and the tets conform)
    hex_faces = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))
    tets = []
    centroids = []
    nlat = verts.shape[0]
    for quad in quads:
        for layer in range(n_rad):
            hexv = [gid(layer, s) for s in quad] + [gid(layer + 1, s) for s in quad]
            cid = nlat + len(centroids)
            centroids.append(verts[hexv].mean(axis=0))
            for fq in hex_faces:
                q4 = [hexv[x] for x in fq]
                k = int(np.argmin(q4))
                if k % 2 == 0:
                    tris = ((q4[0], q4[1], q4[2]), (q4[0], q4[2], q4[3]))
                else:
                    tris = ((q4[1], q4[2], q4[3]), (q4[1], q4[3], q4[0]))
                for t3 in tris:
                    tets.append([t3[0], t3[1], t3[2], cid])
    verts = np.concatenate([verts, np.array(centroids)])
    tets = np.array(tets, dtype=np.int64)
    p = verts[tets]
    s6 = np.einsum("ti,ti->t", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    tets[s6 < 0] = tets[s6 < 0][:, [0, 2, 1, 3]]

    def sides(fc):
        r = np.linalg.norm(fc, axis=1)
        inner = r < 0.5 * (r0 + radii[1])
        kind = np.where(inner, BC_WALL, BC_FARFIELD).astype(np.int32)
        ids = np.where(inner, 0, 1).astype(np.int32)
        return kind, ids

    return _tet_mesh_from_vertices(verts, tets, sides, name or f"sphere{n_ang}x{n_rad}",
                                   extra={"radii": radii})


def _split_hex_by_global_order(hexv, verts):
    """Split a hexahedron into tets so that shared quads are cut consistently.

    ``hexv`` lists the hex's vertices as bottom quad (a,b,c,d) then top quad
    (e,f,g,h), each quad in cyclic order.  The hex is split into 6 tets along
    the diagonal from its lowest global id through Kuhn paths, using the rule
    that every quad face is cut along the diagonal through its smallest global
    vertex id.  That rule depends only on the quad's own vertices, so the two
    hexes sharing a quad cut it the same way.
    """
    # local lattice coordinates of the 8 vertices (cube corners)
    loc = {0: (0, 0, 0), 1: (1, 0, 0), 2: (1, 1, 0), 3: (0, 1, 0),
           4: (0, 0, 1), 5: (1, 0, 1), 6: (1, 1, 1), 7: (0, 1, 1)}
    inv = {v: k for k, v in loc.items()}
    # choose the corner with the smallest global id as the Kuhn origin, and
    # flip local axes so that it becomes (0,0,0)
    k0 = int(np.argmin(hexv))
    o = loc[k0]
    def g(c):
        cc = tuple((ci ^ oi) for ci, oi in zip(c, o))
        return hexv[inv[cc]]
    out = []
    for perm in itertools.permutations(range(3)):
        c = [0, 0, 0]
        path = [g(tuple(c))]
        for ax in perm:
            c[ax] = 1
            path.append(g(tuple(c)))
        out.append(path)
    return out
