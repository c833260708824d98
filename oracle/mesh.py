"""Expansion of the basic mesh into the fields of Section 2 ("Data structure"),
done the plain way with a dictionary keyed by sorted vertex triples (oracle).

Readings where the paper is silent:
  * faces are numbered by ascending lexicographic order of their sorted vertex
    triple;
  * a boundary face keeps the vertex order of its row in the Dirichlet or
    Neumann list (which must be outward); an interior face takes the local
    order (eq 2.1) of the lower-numbered element that contains it;
  * dirfaces/neufaces map rows of the Dirichlet/Neumann lists to face numbers.
All indices are 0-based; perm values are 1..6 as in eq 2.2-2.3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# eq 2.1: local faces (0-based vertex slots)
LOCAL_FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (3, 1, 2))

# eq 2.2: images of (w1, w2, w3) under F_mu, mu = 1..6 (1-based vertex numbers)
F_MU_IMAGES = ((1, 2, 3), (1, 3, 2), (3, 1, 2), (3, 2, 1), (2, 3, 1), (2, 1, 3))


class MeshError(ValueError):
    pass


@dataclass
class Expanded:
    coordinates: np.ndarray
    elements: np.ndarray
    faces: np.ndarray      # (Nfc, 3) vertex numbers, intrinsic order
    ftype: np.ndarray      # (Nfc,) 0 interior, 1 Dirichlet, 2 Neumann
    dirfaces: np.ndarray   # (Ndir,) face of each Dirichlet row
    neufaces: np.ndarray   # (Nneu,)
    facebyele: np.ndarray  # (Nelt, 4)
    perm: np.ndarray       # (Nelt, 4) values 1..6
    volume: np.ndarray     # (Nelt,)
    area: np.ndarray       # (Nfc,)
    normals: np.ndarray    # (Nelt, 4, 3) outward, |n_l| = |e_l|

    @property
    def nelt(self):
        return self.elements.shape[0]

    @property
    def nfc(self):
        return self.faces.shape[0]


def perm_index(local_triple, face_triple) -> int:
    """mu such that phi_e o F_mu = phi_l^K (eq 2.3): the local vertex i equals the
    face vertex F_MU_IMAGES[mu][i]."""
    for mu, img in enumerate(F_MU_IMAGES, start=1):
        if all(local_triple[i] == face_triple[img[i] - 1] for i in range(3)):
            return mu
    raise MeshError("face vertex sets do not match")


def expand(coordinates, elements, dirichlet, neumann) -> Expanded:
    X = np.asarray(coordinates, dtype=np.float64)
    T = np.asarray(elements, dtype=np.int64)
    Nelt = T.shape[0]
    v = X[T]  # (Nelt, 4, 3)
    det = np.einsum("ij,ij->i", np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), v[:, 3] - v[:, 0])
    if np.any(det <= 0):
        raise MeshError("element with non-positive orientation")
    owners = {}
    for K in range(Nelt):
        for l, (a, b, c) in enumerate(LOCAL_FACES):
            key = tuple(sorted((T[K, a], T[K, b], T[K, c])))
            owners.setdefault(key, []).append((K, l))
    keys = sorted(owners)
    fid = {key: i for i, key in enumerate(keys)}
    Nfc = len(keys)
    faces = np.zeros((Nfc, 3), dtype=np.int64)
    ftype = np.zeros(Nfc, dtype=np.int64)
    for key in keys:
        if len(owners[key]) > 2:
            raise MeshError("non-conforming mesh: face shared by more than two elements")
        K, l = min(owners[key])
        a, b, c = LOCAL_FACES[l]
        faces[fid[key]] = (T[K, a], T[K, b], T[K, c])

    def list_rows(rows, code):
        out = np.zeros(len(rows), dtype=np.int64)
        for r, row in enumerate(np.asarray(rows, dtype=np.int64).reshape(-1, 3)):
            key = tuple(sorted(row))
            if key not in fid or len(owners[key]) != 1:
                raise MeshError("listed boundary triangle is not a boundary face")
            f = fid[key]
            if ftype[f] != 0:
                raise MeshError("boundary face listed twice")
            K, _ = owners[key][0]
            w = X[row]
            n = 0.5 * np.cross(w[1] - w[0], w[2] - w[0])
            if np.dot(n, X[T[K]].mean(axis=0) - w.mean(axis=0)) >= 0:
                raise MeshError("boundary triangle listed with inward orientation")
            faces[f] = row
            ftype[f] = code
            out[r] = f
        return out

    dirfaces = list_rows(dirichlet, 1)
    neufaces = list_rows(neumann, 2)
    for key in keys:
        if len(owners[key]) == 1 and ftype[fid[key]] == 0:
            raise MeshError("boundary face missing from the Dirichlet/Neumann lists")

    facebyele = np.zeros((Nelt, 4), dtype=np.int64)
    perm = np.zeros((Nelt, 4), dtype=np.int64)
    normals = np.zeros((Nelt, 4, 3))
    for K in range(Nelt):
        for l, (a, b, c) in enumerate(LOCAL_FACES):
            loc = (T[K, a], T[K, b], T[K, c])
            f = fid[tuple(sorted(loc))]
            facebyele[K, l] = f
            perm[K, l] = perm_index(loc, tuple(faces[f]))
            w = X[list(loc)]
            n = 0.5 * np.cross(w[1] - w[0], w[2] - w[0])
            # Section 2: with the eq 2.1 orientation faces 2 and 4 point out, 1 and 3 in
            normals[K, l] = -n if l in (0, 2) else n
    fw = X[faces]
    area = 0.5 * np.linalg.norm(np.cross(fw[:, 1] - fw[:, 0], fw[:, 2] - fw[:, 0]), axis=1)
    return Expanded(coordinates=X, elements=T, faces=faces, ftype=ftype, dirfaces=dirfaces,
                    neufaces=neufaces, facebyele=facebyele, perm=perm, volume=det / 6.0,
                    area=area, normals=normals)
