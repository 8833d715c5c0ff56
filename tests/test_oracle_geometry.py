"""Pins for the oracle's geometry (CPU only).

The paper fixes: cubes in a 2D layer with at most four neighbours (Results,
Setup, Model), the example network file's neighbour lists (Fig. 2), and that
each face-near molecule belongs to a single face's signalling model.  The
rest (hex lattice, ring order, face slicing, colour classes) is this
project's convention; here it is checked against brute force.
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_example_network_adjacency(oracle_lib):
    net = json.load(open(os.path.join(GOLDEN, "network_2x2.json")))["cells"]
    # lay the printed cells on the lattice by position
    pos = {cid: (round(c["position"][0] / 1e-6), round(c["position"][1] / 1e-6))
           for cid, c in net.items()}
    by_pos = {v: k for k, v in pos.items()}
    for cid, c in net.items():
        x, y = pos[cid]
        cell = y * 2 + x
        xn = oracle_lib.lattice_neighbour(0, 2, 2, cell, 0 if x == 0 else 2)
        yn = oracle_lib.lattice_neighbour(0, 2, 2, cell, 1 if y == 0 else 3)
        want_x, want_y = c["neighbors"]
        assert by_pos[(xn % 2, xn // 2)] == str(want_x)
        assert by_pos[(yn % 2, yn // 2)] == str(want_y)


def _cube(q, r):
    return (q, r, -q - r)


@pytest.mark.parametrize("lattice,nx,ny", [(0, 4, 4), (0, 5, 3), (0, 1, 6), (1, 4, 4),
                                           (1, 7, 5), (1, 1, 3), (1, 6, 1), (0, 1, 1)])
def test_edges_brute_force(oracle_lib, lattice, nx, ny):
    ei, ej, ed, ec = oracle_lib.lattice_edges(lattice, nx, ny)
    pairs = set()
    for i, j in zip(ei, ej):
        assert j > i
        pairs.add((int(i), int(j)))
    assert len(pairs) == len(ei)
    want = set()
    for a, b in itertools.combinations(range(nx * ny), 2):
        xa, ya, xb, yb = a % nx, a // nx, b % nx, b // nx
        if lattice == 0:
            adj = abs(xa - xb) + abs(ya - yb) == 1
        else:
            ca, cb = _cube(xa, ya), _cube(xb, yb)
            adj = max(abs(u - v) for u, v in zip(ca, cb)) == 1
        if adj:
            want.add((a, b))
    assert pairs == want
    # each colour class is a matching; ranking is by (colour, i)
    for col in set(ec.tolist()):
        cells = np.concatenate([ei[ec == col], ej[ec == col]])
        assert len(set(cells.tolist())) == len(cells)
    order = list(zip(ec.tolist(), ei.tolist()))
    assert order == sorted(order)
    # every cell has at most 4 (square) / 6 (hex) neighbours
    deg = np.bincount(np.concatenate([ei, ej]), minlength=nx * ny)
    assert deg.max(initial=0) <= (4 if lattice == 0 else 6)


def test_edge_class_sizes_of_the_two_main_workloads(oracle_lib):
    _, _, _, ec = oracle_lib.lattice_edges(0, 4, 4)
    assert np.bincount(ec).tolist() == [8, 4, 8, 4]
    _, _, _, ec = oracle_lib.lattice_edges(1, 64, 64)
    assert len(ec) == 12033
    assert np.bincount(ec).tolist() == [2048, 1984, 2048, 1984, 2016, 1953]


@pytest.mark.parametrize("w,h", [(w, h) for w in range(1, 9) for h in range(1, 9)])
def test_ring_is_the_boundary_walk(oracle_lib, w, h):
    ring = oracle_lib.ring(w, h)
    boundary = {y * w + x for x in range(w) for y in range(h)
                if x in (0, w - 1) or y in (0, h - 1)}
    assert len(ring) == len(set(ring))
    assert set(ring) == boundary
    assert ring[0] == w - 1  # top-right corner (x = w-1, y = 0)
    # consecutive ring voxels are mesh neighbours (a closed walk)
    if len(ring) > 1:
        for a, b in zip(ring, ring[1:]):
            nb = oracle_lib.voxel_neighbours(w, h, a)
            assert b in nb
    if w == 4 and h == 4:
        assert len(ring) == 12


@pytest.mark.parametrize("w,h", [(w, h) for w in range(1, 9) for h in range(1, 9)])
@pytest.mark.parametrize("nd", [4, 6])
def test_face_groups_single_face(oracle_lib, w, h, nd):
    ring = oracle_lib.ring(w, h)
    M = len(ring)
    groups = [oracle_lib.face_group(w, h, nd, d) for d in range(nd)]
    for g in groups:
        assert len(g) >= 1 and set(g) <= set(ring)
    if M >= nd:
        # groups partition the ring: every membrane voxel in exactly one face
        flat = [v for g in groups for v in g]
        assert sorted(flat) == sorted(ring)
    if (w, h) == (4, 4):
        assert all(len(g) == (3 if nd == 4 else 2) for g in groups)


def test_square_4x4_faces_point_outward(oracle_lib):
    w = h = 4
    # direction 0 +x, 1 +y, 2 -x, 3 -y (y pointing down)
    side = {0: lambda x, y: x == w - 1, 1: lambda x, y: y == h - 1,
            2: lambda x, y: x == 0, 3: lambda x, y: y == 0}
    for d in range(4):
        for v in oracle_lib.face_group(w, h, 4, d):
            assert side[d](v % w, v // w)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 4), (3, 1), (4, 4), (8, 8), (2, 5)])
def test_voxel_neighbours_brute_force(oracle_lib, w, h):
    for v in range(w * h):
        x, y = v % w, v // w
        got = oracle_lib.voxel_neighbours(w, h, v)
        want = []
        for dx, dy in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
            if 0 <= x + dx < w and 0 <= y + dy < h:
                want.append((y + dy) * w + x + dx)
        assert got == want
