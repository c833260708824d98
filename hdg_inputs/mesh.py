"""Kuhn-split cube meshes: the basic tetrahedral data structure of the paper's
Section 2 ("Data structure": coordinates, elements, Dirichlet and Neumann
triangle lists), generated synthetically.

Conventions (0-based indices):
  * vertex (i, j, l), 0 <= i, j, l <= n, has id i + (n+1) j + (n+1)^2 l and
    coordinates h (i, j, l) with h = 1/n (before jitter);
  * cubes are visited with l outermost, then j, then i; every cube is split into
    six tetrahedra, one per permutation s of the axes (itertools order), with
    vertices o, o + h e_s0, o + h (e_s0 + e_s1), o + h (1, 1, 1); when that order
    has negative orientation the 2nd and 3rd vertices are swapped, so that every
    element is positively oriented as Section 2 requires;
  * boundary triangles are the element faces (in the local face order of eq 2.1)
    lying on a cube side, listed with outward orientation; a triangle is
    Dirichlet or Neumann according to the side it lies on;
  * optional jitter moves interior vertices only, uniformly in
    [-jitter h, jitter h]^3, drawn from numpy's PCG64(seed).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# Local faces of a tetrahedron in the order of eq 2.1 (0-based vertex slots).
LOCAL_FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (3, 1, 2))

SIDES = ("x0", "x1", "y0", "y1", "z0", "z1")


@dataclass
class KuhnMesh:
    n: int
    coordinates: np.ndarray  # float64 (Nver, 3)
    elements: np.ndarray     # int32 (Nelt, 4)
    dirichlet: np.ndarray    # int32 (Ndir, 3)
    neumann: np.ndarray      # int32 (Nneu, 3)

    @property
    def nver(self) -> int:
        return self.coordinates.shape[0]

    @property
    def nelt(self) -> int:
        return self.elements.shape[0]


def _kuhn_elements(n: int) -> np.ndarray:
    N1 = n + 1
    ii, jj, ll = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # cube order: l outermost, then j, then i
    o = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                  ll.transpose(2, 1, 0).ravel()], axis=1)  # (n^3, 3) grid origins
    eye = np.eye(3, dtype=np.int64)
    tets = []
    for s in itertools.permutations(range(3)):
        v1 = o
        v2 = o + eye[s[0]]
        v3 = v2 + eye[s[1]]
        v4 = o + 1
        # orientation of (v1, v2, v3, v4) is the sign of the permutation s
        det = np.linalg.det(np.stack([eye[s[0]], eye[s[0]] + eye[s[1]], np.ones(3, dtype=np.int64)], axis=1))
        if det < 0:
            v2, v3 = v3, v2
        tets.append(np.stack([v1, v2, v3, v4], axis=1))  # (n^3, 4, 3)
    g = np.stack(tets, axis=1).reshape(-1, 4, 3)  # cube-major, then permutation
    ids = g[..., 0] + N1 * g[..., 1] + N1 * N1 * g[..., 2]
    return ids.astype(np.int32), g


def kuhn_mesh(n: int, jitter: float = 0.0, seed: int = 0,
              dirichlet_sides=SIDES, neumann_sides=()) -> KuhnMesh:
    """Kuhn split of the unit cube into 6 n^3 tetrahedra.

    ``dirichlet_sides`` / ``neumann_sides`` partition the six cube sides
    ("x0", "x1", "y0", "y1", "z0", "z1"); every side must be in exactly one.
    """
    if set(dirichlet_sides) | set(neumann_sides) != set(SIDES) or set(dirichlet_sides) & set(neumann_sides):
        raise ValueError("each cube side must be either Dirichlet or Neumann")
    N1 = n + 1
    h = 1.0 / n
    elements, grid = _kuhn_elements(n)
    ii, jj, ll = np.meshgrid(np.arange(N1), np.arange(N1), np.arange(N1), indexing="ij")
    gv = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                   ll.transpose(2, 1, 0).ravel()], axis=1)  # vertex id order i fastest
    coords = gv.astype(np.float64) * h
    if jitter:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        interior = np.all((gv > 0) & (gv < n), axis=1)
        coords = coords + d * interior[:, None]

    # boundary triangles from the integer grid (boundary vertices never move)
    dir_rows, neu_rows = [], []
    side_of = {("x", 0): "x0", ("x", n): "x1", ("y", 0): "y0", ("y", n): "y1", ("z", 0): "z0", ("z", n): "z1"}
    outward = {"x0": (0, -1), "x1": (0, 1), "y0": (1, -1), "y1": (1, 1), "z0": (2, -1), "z1": (2, 1)}
    tri_all = []
    for f, (a, b, c) in enumerate(LOCAL_FACES):
        ga, gb, gc = grid[:, a], grid[:, b], grid[:, c]
        for ax, name in enumerate("xyz"):
            for val in (0, n):
                on = (ga[:, ax] == val) & (gb[:, ax] == val) & (gc[:, ax] == val)
                if not on.any():
                    continue
                K = np.nonzero(on)[0]
                side = side_of[(name, val)]
                w1, w2, w3 = ga[K], gb[K], gc[K]
                nrm = np.cross(w2 - w1, w3 - w1)
                comp, sgn = outward[side]
                flip = (nrm[:, comp] * sgn) < 0
                v = np.stack([elements[K, a], elements[K, b], elements[K, c]], axis=1)
                v[flip] = v[flip][:, [0, 2, 1]]
                tri_all.append((K, f, side, v))
    # list in element order, then local face order
    recs = []
    for K, f, side, v in tri_all:
        for t in range(K.size):
            recs.append((int(K[t]), f, side, v[t]))
    recs.sort(key=lambda r: (r[0], r[1]))
    for K, f, side, v in recs:
        (dir_rows if side in dirichlet_sides else neu_rows).append(v)
    dirichlet = np.array(dir_rows, dtype=np.int32).reshape(-1, 3)
    neumann = np.array(neu_rows, dtype=np.int32).reshape(-1, 3)
    return KuhnMesh(n=n, coordinates=coords, elements=elements, dirichlet=dirichlet, neumann=neumann)


def single_tet_mesh(vertices=None) -> KuhnMesh:
    """One positively oriented tetrahedron with all four faces Dirichlet."""
    if vertices is None:
        vertices = np.array([[0.1, 0.0, 0.05], [1.0, 0.2, 0.0], [0.15, 0.9, 0.1], [0.2, 0.25, 1.1]])
    coords = np.asarray(vertices, dtype=np.float64)
    el = np.array([[0, 1, 2, 3]], dtype=np.int32)
    rows = []
    for (a, b, c) in LOCAL_FACES:
        w1, w2, w3 = coords[a], coords[b], coords[c]
        nrm = np.cross(w2 - w1, w3 - w1)
        other = [i for i in range(4) if i not in (a, b, c)][0]
        if np.dot(nrm, coords[other] - w1) > 0:  # points inward
            rows.append([a, c, b])
        else:
            rows.append([a, b, c])
    return KuhnMesh(n=0, coordinates=coords, elements=el,
                    dirichlet=np.array(rows, dtype=np.int32), neumann=np.zeros((0, 3), dtype=np.int32))


# The twelve even permutations of four vertex slots: reordering an element's vertices by
# one of them keeps det B_K > 0 (Section 2 requires positively oriented elements).
EVEN_PERMUTATIONS = tuple(p for p in itertools.permutations(range(4))
                          if sum(p[i] > p[j] for i in range(4) for j in range(i + 1, 4)) % 2 == 0)


def permute_element_vertices(mesh: KuhnMesh, seed: int = 0) -> KuhnMesh:
    """The same mesh with each element's vertex list reordered by a seeded even permutation
    (numpy PCG64(seed), one of the twelve per element).  The boundary lists are untouched.
    A Kuhn mesh alone meets only a few (local face, face permutation) pairs; reordered this
    way, interior faces are seen from their two elements under every relative orientation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, len(EVEN_PERMUTATIONS), size=mesh.nelt)
    perms = np.array(EVEN_PERMUTATIONS, dtype=np.int64)[pick]            # (nelt, 4)
    el = np.take_along_axis(mesh.elements, perms, axis=1).astype(np.int32)
    return KuhnMesh(n=mesh.n, coordinates=mesh.coordinates, elements=el,
                    dirichlet=mesh.dirichlet, neumann=mesh.neumann)
