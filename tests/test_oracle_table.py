"""Pins of the oracle's cube conventions and marching-cubes polygons.

What fixes them: the paper's six printed regular types and their stated
pairwise Hamming distances (Sec. V-F), its bounds of 5 triangles per cube and
3 owned + 9 neighbouring edges (Sec. IV, V-B), the definition of the MC edge
table (a vertex exists exactly on the edges whose end signs differ, Sec. V-B),
and the geometry of the cube: rotation equivariance, complement symmetry of
the edge table and a crack-free, consistently oriented surface on random
sign fields.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from tests import meshutil

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def printed_regular_types():
    rows = [l.strip() for l in open(os.path.join(GOLDEN, "regular_types.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    return rows


def crossing_edges(t):
    ends = oracle.edge_ends()
    return {e for e in range(12) if ((t >> ends[e][0]) & 1) != ((t >> ends[e][1]) & 1)}


def test_regular_types_match_printed_strings():
    printed = printed_regular_types()
    assert oracle.regular_types() == [int(s, 2) for s in printed]
    # Read least significant bit first the set is the same (the figure that
    # fixed the bit order is missing from the paper's text).
    assert sorted(int(s[::-1], 2) for s in printed) == sorted(int(s, 2) for s in printed)


def test_regular_types_pairwise_hamming_4_or_8():
    reg = [int(s, 2) for s in printed_regular_types()]
    for a, b in itertools.combinations(reg, 2):
        assert bin(a ^ b).count("1") in (4, 8)


def test_regular_types_are_axis_aligned_half_cubes():
    # Under the corner numbering the regular types cut the cube in half
    # along an axis: their inside corners form one face.
    C = oracle.corner_offsets()
    for t in oracle.regular_types():
        inside = [k for k in range(8) if (t >> k) & 1]
        assert len(inside) == 4
        pts = C[inside]
        assert any(len(set(pts[:, a])) == 1 for a in range(3)), t
        # and each regular type meshes as a single flat quad (2 triangles)
        assert oracle.cube_polygon_sizes(t) == [4]


def test_corner_numbering_edges_and_ownership():
    C = oracle.corner_offsets()
    E = oracle.edge_ends()
    # eight distinct unit-cube corners, twelve distinct unit-length edges
    assert len({tuple(c) for c in C}) == 8
    assert len({tuple(sorted(e)) for e in E}) == 12
    for a, b in E:
        assert np.abs(C[a] - C[b]).sum() == 1
    # Sec. V-B: 3 of a cube's edges start at its own anchor corner, 9 belong
    # to adjacent cubes.
    own = [e for e in range(12) if min(tuple(C[E[e][0]]), tuple(C[E[e][1]])) == (0, 0, 0)]
    assert len(own) == 3


@pytest.mark.parametrize("t", range(256))
def test_polygons_cover_exactly_the_crossing_edges(t):
    polys = oracle.cube_polygons(t)
    flat = [e for p in polys for e in p]
    assert len(flat) == len(set(flat))
    assert set(flat) == crossing_edges(t)
    # complement has the same edge set (a vertex per sign change)
    assert crossing_edges(255 - t) == crossing_edges(t)
    tris = oracle.cube_triangles(t)
    assert len(tris) <= 5                       # at most five per cube (Sec. IV)
    assert len(tris) == sum(len(p) - 2 for p in polys)
    assert all(3 <= len(p) <= 7 for p in polys)


def cube_rotations():
    """The 24 proper rotations of the cube as 3x3 integer matrices."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), int)
            for i, (p, s) in enumerate(zip(perm, signs)):
                M[i, p] = s
            if round(np.linalg.det(M)) == 1:
                mats.append(M)
    assert len(mats) == 24
    return mats


def corner_and_edge_permutations(M):
    C = oracle.corner_offsets()
    E = oracle.edge_ends()
    cen = (2 * C - 1)  # corners at +-1
    rot = cen @ M.T
    cperm = [int(np.where((cen == r).all(1))[0][0]) for r in rot]
    edges = {tuple(sorted(e)): i for i, e in enumerate(E.tolist())}
    eperm = [edges[tuple(sorted((cperm[a], cperm[b])))] for a, b in E]
    return cperm, eperm


def rotate_type(t, cperm):
    return sum(1 << cperm[k] for k in range(8) if (t >> k) & 1)


def canon_cycle(p):
    i = p.index(min(p))
    return tuple(p[i:] + p[:i])


def test_rotation_equivariance_of_polygons():
    for M in cube_rotations():
        cperm, eperm = corner_and_edge_permutations(M)
        for t in range(256):
            rt = rotate_type(t, cperm)
            mapped = {canon_cycle([eperm[e] for e in p]) for p in oracle.cube_polygons(t)}
            got = {canon_cycle(p) for p in oracle.cube_polygons(rt)}
            assert mapped == got, (t, rt)


def test_orbit_counts():
    rots = [corner_and_edge_permutations(M)[0] for M in cube_rotations()]
    seen, orbits, orbits_c = set(), 0, set()
    for t in range(256):
        orb = frozenset(rotate_type(t, p) for p in rots)
        if t not in seen:
            orbits += 1
            seen |= orb
        orbits_c.add(frozenset(orb | {255 - x for x in orb}))
    assert orbits == 23          # 22 non-trivial classes + the empty cube ... under rotation
    assert len(orbits_c) == 15   # Lorensen and Cline's 14 cases plus the empty cube


def test_complement_reverses_orientation_without_ambiguous_faces():
    """Where no face has alternating signs, t and its complement give the
    same polygons traversed in the opposite direction."""
    C = oracle.corner_offsets()
    faces = []
    for a in range(3):
        for s in (0, 1):
            faces.append([k for k in range(8) if C[k][a] == s])
    checked = 0
    for t in range(256):
        amb = False
        for f in faces:
            signs = [(t >> k) & 1 for k in f]
            if sum(signs) == 2:
                diag = [k for k in f if (t >> k) & 1]
                if np.abs(C[diag[0]] - C[diag[1]]).sum() == 2:
                    amb = True
        if amb:
            continue
        checked += 1
        a = {canon_cycle(p) for p in oracle.cube_polygons(t)}
        b = {canon_cycle(p[::-1]) for p in oracle.cube_polygons(255 - t)}
        assert a == b, t
    assert checked == 136


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_sign_field_is_crack_free_and_oriented(seed):
    """Marching random sign fields (many ambiguous faces) gives a closed,
    consistently oriented surface: every interior mesh edge is traversed
    equally often in both directions, and only edges lying on the volume's
    outer faces are open.  (A polygon that crosses an ambiguous face twice
    can put a fan diagonal in that face, so an interior edge may carry four
    triangles; it is still balanced.)"""
    rng = np.random.default_rng(seed)
    n = 2  # 2x2x2 blocks -> 15^3 valid cubes
    d = rng.choice([-1.0, 1.0], size=(8 * n, 8 * n, 8 * n)) * rng.uniform(0.1, 1.0, (8 * n,) * 3)
    from scenes import dense_to_blocks
    coords, db = dense_to_blocks(d.astype(np.float32))
    vol = oracle.OracleVolume(0.01)
    vol.import_blocks(coords, db, np.ones_like(db))
    vol.extract(scope_all=True)
    keys = vol.triangles()
    verts = vol.vertices()
    index = {tuple(k): i for i, k in enumerate(verts["keys"].tolist())}
    tris = np.array([[index[tuple(k)] for k in tri] for tri in keys.tolist()])
    de = meshutil.directed_edges(tris)
    ue = meshutil.undirected_edges(tris)
    K = verts["keys"]
    lo, hi = 0, 8 * n - 1
    n_open = 0
    for (u, v), cnt in ue.items():
        fwd, bwd = de.get((u, v), 0), de.get((v, u), 0)
        if fwd == bwd:
            continue
        # an open edge: used once, both vertices on one outer face plane
        assert cnt == 1, (K[u], K[v], fwd, bwd)
        n_open += 1
        pu = K[u, :3] + 0.5 * np.eye(3, dtype=int)[K[u, 3]]
        pv = K[v, :3] + 0.5 * np.eye(3, dtype=int)[K[v, 3]]
        on = [(a, b) for a in range(3) for b in (lo, hi) if pu[a] == b and pv[a] == b]
        assert on, (K[u], K[v])
    assert n_open > 0
    # reference counts equal vertex degrees in triangles (Sec. V-E)
    deg = np.bincount(tris.ravel(), minlength=len(K))
    assert (deg == verts["ref"]).all()
    assert verts["ref"].sum() == 3 * len(tris)
