"""Brute-force contraction of finite honeycomb patches.

TEST INFRASTRUCTURE ONLY (see ``oracle/ctm.py``).

This is the independent check of the contraction network used by the
CTMRG oracle.  The paper's figures (Fig. 1c,d: pairs of sites mapped onto a
square quadrant inside a 60-degree sector; Fig. 4b: local expectation value)
are not available, so the network is rebuilt here from lattice coordinates
alone and contracted directly, with no reference to corners or edges:

* pointy-top honeycomb, bond length 1, a hexagon centre at the origin;
* sector w (w = 0..5) is the 60-degree wedge bisected by the ray at
  90 + 60 w degrees; in sector 0 the vertical bonds centred at
  (0, 1.5) + m e1 + n e2 (e1, e2 the lattice vectors at 60 and 120 degrees,
  length sqrt(3)), 0 <= m, n < N, are the pairs of the local mapping; the
  other sectors are rotations of sector 0;
* every site carries the double-layer tensor (fully symmetric in its three
  legs for a C3v-symmetric site tensor, so legs need no orientation), bonds
  between two patch sites are contracted, bonds leaving the patch are closed
  by identifying ket and bra (the vector delta_{u u'});
* the two sites of sector 0's apex pair keep their physical legs open.

Contracting gives the bond density matrix of that pair on the 12 N^2-site
patch, which N-1 untruncated CTMRG steps must reproduce.
"""
from __future__ import annotations

import math

import numpy as np

SQ3 = math.sqrt(3.0)
E1 = np.array([SQ3 / 2, 1.5])
E2 = np.array([-SQ3 / 2, 1.5])


def rotation(w: int) -> np.ndarray:
    t = math.pi / 3 * w
    return np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])


def patch_sites(N: int):
    """Coordinates of the 12 N^2 sites; also returns the indices of sector 0's
    apex pair (outer site, inner site)."""
    pts = []
    outer0 = inner0 = None
    for w in range(6):
        R = rotation(w)
        for m in range(N):
            for n in range(N):
                c = np.array([0.0, 1.5]) + m * E1 + n * E2
                inner = R @ (c - np.array([0.0, 0.5]))
                outer = R @ (c + np.array([0.0, 0.5]))
                if w == 0 and m == 0 and n == 0:
                    inner0, outer0 = len(pts), len(pts) + 1
                pts.append(inner)
                pts.append(outer)
    return np.array(pts), outer0, inner0


def bonds(pts: np.ndarray):
    """All nearest-neighbour pairs (distance 1) inside the patch."""
    out = []
    for i in range(len(pts)):
        dist = np.linalg.norm(pts - pts[i], axis=1)
        for j in np.nonzero(np.abs(dist - 1.0) < 1e-9)[0]:
            if j > i:
                out.append((i, int(j)))
    return out


def _contract(tensors, labels, open_labels):
    """Greedy pairwise contraction: repeatedly contract the two connected
    tensors whose product is smallest."""
    tensors = list(tensors)
    labels = [list(l) for l in labels]
    while len(tensors) > 1:
        best = None
        for i in range(len(tensors)):
            li = set(labels[i])
            for j in range(i + 1, len(tensors)):
                shared = li.intersection(labels[j])
                if not shared:
                    continue
                size = 1
                for t, ls in ((i, labels[i]), (j, labels[j])):
                    for ax, l in enumerate(ls):
                        if l not in shared:
                            size *= tensors[t].shape[ax]
                if best is None or size < best[0]:
                    best = (size, i, j, shared)
        if best is None:            # disconnected pieces: outer product
            best = (0, 0, 1, set())
        _, i, j, shared = best
        shared = list(shared)
        ai = [labels[i].index(l) for l in shared]
        aj = [labels[j].index(l) for l in shared]
        t = np.tensordot(tensors[i], tensors[j], axes=(ai, aj))
        nl = [l for l in labels[i] if l not in shared] + [l for l in labels[j] if l not in shared]
        for k in (j, i):
            del tensors[k]
            del labels[k]
        tensors.append(t)
        labels.append(nl)
    t, l = tensors[0], labels[0]
    return np.transpose(t, [l.index(x) for x in open_labels])


def patch_density_matrix(A: np.ndarray, N: int) -> np.ndarray:
    """Bond density matrix rho[(s,t),(s',t')] of sector 0's apex pair on the
    12 N^2-site patch, normalized to unit trace."""
    d, D = A.shape[0], A.shape[1]
    D2 = D * D
    a = np.einsum("suvw,sxyz->uxvywz", A, A).reshape(D2, D2, D2)
    ao = np.einsum("suvw,txyz->uxvywzst", A, A).reshape(D2, D2, D2, d, d)
    closing = np.eye(D).reshape(D2)
    pts, outer0, inner0 = patch_sites(N)
    bl = bonds(pts)
    legs = {i: [] for i in range(len(pts))}
    for b, (i, j) in enumerate(bl):
        legs[i].append(("b", b))
        legs[j].append(("b", b))
    tensors, labels = [], []
    for i in range(len(pts)):
        if i == outer0:
            t, phys = ao, [("p", "s"), ("p", "s'")]
        elif i == inner0:
            t, phys = ao, [("p", "t"), ("p", "t'")]
        else:
            t, phys = a, []
        k = len(legs[i])
        assert k <= 3
        # the tensor is symmetric in its virtual legs: bonds inside the patch
        # take the first k of them, the remaining ones are closed
        for ax in reversed(range(k, 3)):
            t = np.tensordot(t, closing, axes=([ax], [0]))
        tensors.append(t)
        labels.append(list(legs[i]) + phys)
    rho = _contract(tensors, labels, [("p", "s"), ("p", "t"), ("p", "s'"), ("p", "t'")])
    rho = rho.reshape(d * d, d * d)
    return rho / np.trace(rho)


def patch_norm(A: np.ndarray, N: int) -> float:
    """<Psi|Psi> of the 12 N^2-site patch with every leg leaving it closed."""
    D = A.shape[1]
    D2 = D * D
    a = np.einsum("suvw,sxyz->uxvywz", A, A).reshape(D2, D2, D2)
    closing = np.eye(D).reshape(D2)
    pts, _, _ = patch_sites(N)
    bl = bonds(pts)
    legs = {i: [] for i in range(len(pts))}
    for b, (i, j) in enumerate(bl):
        legs[i].append(("b", b))
        legs[j].append(("b", b))
    tensors, labels = [], []
    for i in range(len(pts)):
        t = a
        for ax in reversed(range(len(legs[i]), 3)):
            t = np.tensordot(t, closing, axes=([ax], [0]))
        tensors.append(t)
        labels.append(list(legs[i]))
    return float(_contract(tensors, labels, []))
