"""Kuhn tetrahedral mesh of the unit cube and its hierarchical-P2 node numbering.

Test infrastructure only (see ``oracle/__init__``).

The paper's cube meshes (Section 4.1, table of mesh sizes) have n^3 cubes for
n = 4, 8, 16, 32 ("#Tet" counts cubes); each cube is split into the 6 Kuhn
tetrahedra, i.e. the monotone lattice paths from corner (i,j,k) to
(i+1,j+1,k+1). Linear nodes are the vertices, quadratic nodes the edges
(midside nodes), Section 2.3.

Numbering (the ordering the method's coarsening depends on):
* vertex (i, j, k) has id i + (n+1) * (j + (n+1) * k);
* linear nodes are the vertices in id order;
* quadratic nodes are the edges sorted by (smaller vertex id, larger vertex id),
  numbered after all vertices.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# Local edge order of the quadratic basis phi_5..phi_10 in Section 2.3:
# phi_5 = 4 l1 l2, phi_6 = 4 l2 l3, phi_7 = 4 l3 l4, phi_8 = 4 l1 l3,
# phi_9 = 4 l1 l4, phi_10 = 4 l2 l4   (0-based vertex pairs below).
LOCAL_EDGES = ((0, 1), (1, 2), (2, 3), (0, 2), (0, 3), (1, 3))


@dataclass
class Mesh:
    n: int
    coords: np.ndarray      # (nv, 3)
    tets: np.ndarray        # (nt, 4) vertex ids, lattice-path order
    edges: np.ndarray       # (ne, 2) vertex ids (a < b), sorted lexicographically
    tet_nodes: np.ndarray   # (nt, 10) global node ids: 4 vertices, 6 edge nodes

    @property
    def nv(self) -> int:
        return self.coords.shape[0]

    @property
    def ne(self) -> int:
        return self.edges.shape[0]

    @property
    def nnodes(self) -> int:
        return self.nv + self.ne

    def node_coords(self) -> np.ndarray:
        """Coordinates of all P2 nodes (vertices, then edge midpoints)."""
        mid = 0.5 * (self.coords[self.edges[:, 0]] + self.coords[self.edges[:, 1]])
        return np.vstack([self.coords, mid])

    def edge_id(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        """Global node id of the edge between vertices a and b (arrays)."""
        lo = np.minimum(a, b).astype(np.int64)
        hi = np.maximum(a, b).astype(np.int64)
        keys = lo * self.nv + hi
        allk = self.edges[:, 0].astype(np.int64) * self.nv + self.edges[:, 1]
        pos = np.searchsorted(allk, keys)
        assert np.all(allk[pos] == keys), "not an edge of the mesh"
        return self.nv + pos


def vid(n: int, i, j, k):
    return i + (n + 1) * (j + (n + 1) * k)


def kuhn_mesh(n: int, mirrored: bool = False) -> Mesh:
    """n^3 cubes, 6 Kuhn tets each.

    With ``mirrored`` the split of every cube in the upper half of an axis
    (cube index >= n/2) is reflected in that axis, so each cube's main
    diagonal points towards the centre of the domain. The mesh stays
    conforming (a shared face's diagonal depends only on the two axes in the
    face, which both cubes treat alike) and has the same vertex and edge
    counts; every tetrahedron then has a vertex off the boundary (n >= 2).
    The all-Dirichlet Stokes cavity needs this: on the plain split, tets with
    all vertices on the boundary carry spurious Taylor-Hood pressure modes.
    """
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64) / n

    c = np.arange(n)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    if mirrored:
        refl = [(ci * 2 >= n).astype(np.int64), (cj * 2 >= n).astype(np.int64),
                (ck * 2 >= n).astype(np.int64)]
    else:
        refl = [np.zeros_like(ci)] * 3
    start = [ci + refl[0], cj + refl[1], ck + refl[2]]
    step = [1 - 2 * r for r in refl]
    tets = []
    for perm in itertools.permutations(range(3)):
        pos = [s.copy() for s in start]
        path = [vid(n, *pos)]
        for axis in perm:
            pos[axis] = pos[axis] + step[axis]
            path.append(vid(n, *pos))
        tets.append(np.stack(path, axis=1))
    # order: cube-major, then the 6 permutations
    tets = np.stack(tets, axis=1).reshape(-1, 4)

    pairs = np.concatenate([np.sort(tets[:, list(e)], axis=1) for e in LOCAL_EDGES])
    keys = np.unique(pairs[:, 0].astype(np.int64) * (m ** 3) + pairs[:, 1])
    edges = np.stack([keys // (m ** 3), keys % (m ** 3)], axis=1).astype(np.int64)

    mesh = Mesh(n, coords, tets.astype(np.int64), edges, np.empty((0, 10), np.int64))
    enodes = np.stack([mesh.edge_id(tets[:, a], tets[:, b]) for a, b in LOCAL_EDGES], axis=1)
    mesh.tet_nodes = np.concatenate([tets, enodes], axis=1).astype(np.int64)
    return mesh


def face_triangles_x1(mesh: Mesh) -> np.ndarray:
    """Boundary triangles of the face x=1 as vertex triples, shape (n, n, 2, 3).

    Triangle t=0 of square (j, k) is (y_j,z_k),(y_j+1,z_k),(y_j+1,z_k+1);
    t=1 is (y_j,z_k),(y_j,z_k+1),(y_j+1,z_k+1). Both are faces of Kuhn tets
    (the square's diagonal runs from (j,k) to (j+1,k+1)).
    """
    n = mesh.n
    j, k = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = vid(n, n, j, k)
    v10 = vid(n, n, j + 1, k)
    v01 = vid(n, n, j, k + 1)
    v11 = vid(n, n, j + 1, k + 1)
    t0 = np.stack([v00, v10, v11], axis=-1)
    t1 = np.stack([v00, v01, v11], axis=-1)
    return np.stack([t0, t1], axis=2)


def boundary_faces(mesh: Mesh) -> np.ndarray:
    """All boundary triangles (faces owned by exactly one tet), sorted vertex triples."""
    faces = np.concatenate([np.sort(mesh.tets[:, list(f)], axis=1)
                            for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))])
    m = mesh.nv
    keys = (faces[:, 0] * m + faces[:, 1]) * m + faces[:, 2]
    uk, cnt = np.unique(keys, return_counts=True)
    b = uk[cnt == 1]
    return np.stack([b // (m * m), (b // m) % m, b % m], axis=1)
