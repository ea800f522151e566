"""Pins of the Hamming-distance refinement, Eqs. (3)-(5) of Sec. V-F, on
hand-built cubes, and of its use in the oracle's pipeline."""
import numpy as np
import pytest

import oracle
import scenes

EPS = 0.5


def corners_for(t, mag=2.0, small=()):
    """Corner TSDF values realising type t; corners in `small` get |d| = 0.1."""
    d = np.array([(-mag if (t >> k) & 1 else mag) for k in range(8)], np.float32)
    for k in small:
        d[k] = np.float32(-0.1 if (t >> k) & 1 else 0.1)
    return d


@pytest.mark.parametrize("j", range(6))
def test_regular_types_stay(j):
    r = oracle.regular_types()[j]
    for prev in (0, r, 255, 0x5A):
        assert oracle.refine_type(r, prev, corners_for(r), EPS) == r


def test_empty_and_full_cubes_stay():
    # distance 4 from every regular type (Sec. V-F discriminates at 3)
    for t in (0, 255):
        for prev in (0, 255, 0xCC):
            assert oracle.refine_type(t, prev, corners_for(t, small=range(8)), EPS) == t


@pytest.mark.parametrize("j", range(6))
@pytest.mark.parametrize("k", range(8))
def test_one_flipped_near_zero_corner_is_restored(j, k):
    r = oracle.regular_types()[j]
    t = r ^ (1 << k)
    assert oracle.refine_type(t, r, corners_for(t, small=[k]), EPS) == r
    # not restored when the flipped corner is far from the surface (Eq. 5)
    assert oracle.refine_type(t, r, corners_for(t), EPS) == t
    # nor when the previous type is too far away (Eq. 3): the opposite
    # regular type is at Hamming distance 7 from t
    assert oracle.refine_type(t, r ^ 0xFF, corners_for(t, small=[k]), EPS) == t


def test_threshold_is_strict():
    r = oracle.regular_types()[0]
    t = r ^ 1
    d = corners_for(t)
    d[0] = np.float32(EPS)          # |d| == eps is not < eps
    assert oracle.refine_type(t, r, d, EPS) == t
    d[0] = np.nextafter(np.float32(EPS), np.float32(0))
    assert oracle.refine_type(t, r, d, EPS) == r


def test_previous_regular_type_wins_ties():
    # t at distance 2 from two regular types (a perpendicular pair)
    reg = oracle.regular_types()
    a, b = reg[0], reg[4]   # 0xCC and 0xF0 differ in 4 corners
    diff = [k for k in range(8) if ((a ^ b) >> k) & 1]
    t = a ^ (1 << diff[0]) ^ (1 << diff[1])
    assert bin(t ^ b).count("1") == 2
    d = corners_for(t, small=diff)
    assert oracle.refine_type(t, a, d, EPS) == a
    assert oracle.refine_type(t, b, d, EPS) == b
    # with neither as previous, the first listed one is taken
    assert oracle.refine_type(t, t, d, EPS) == a


def test_refine_twice_equals_once_and_regularises():
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.04, holes=True)
    vol = oracle.OracleVolume(seq.voxel_m, 4.0, EPS)
    changed_total = 0
    for k in (0, 10):
        vol.integrate(seq.frame(k), scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        vol.extract()
        changed_total += vol.refine()
        # a second pass changes nothing
        assert vol.refine() == 0
        vol.gc()
    assert changed_total > 0
    cur = vol.blocks()["cur"]
    reg = set(oracle.regular_types())
    frac_regular = np.isin(cur[cur > 0], list(reg)).mean()
    assert frac_regular > 0.3
    # the mesh stays consistent: reference counts equal triangle degrees
    vv = vol.vertices(live_only=False)
    assert (vv["ref"] > 0).all()
    assert vv["ref"].sum() == 3 * len(vol.triangles())


def test_refining_extraction_equals_extract_then_refine():
    """Sec. V-F applies the regular type before marching cubes: extraction
    with the refinement folded in ends with the types, vertices, t, counts
    and triangles of a plain extraction followed by a refinement pass, and
    differs from the plain extraction alone."""
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.04, holes=True)
    fused = oracle.OracleVolume(seq.voxel_m, 4.0, EPS)
    two = oracle.OracleVolume(seq.voxel_m, 4.0, EPS)
    plain = oracle.OracleVolume(seq.voxel_m, 4.0, EPS)
    differs = False
    for k in (0, 4, 8, 12, 16, 20):
        for v in (fused, two, plain):
            v.integrate(seq.frame(k), scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        fused.extract(refine=True)
        two.extract()
        two.refine()
        plain.extract()
        bf, bt, bp = fused.blocks(), two.blocks(), plain.blocks()
        assert np.array_equal(bf["coords"], bt["coords"])
        assert np.array_equal(bf["cur"], bt["cur"]) and np.array_equal(bf["prev"], bt["prev"])
        differs |= not np.array_equal(bf["cur"], bp["cur"])
        vf, vt = fused.vertices(), two.vertices()
        assert np.array_equal(vf["keys"], vt["keys"])
        assert np.array_equal(vf["t"], vt["t"]) and np.array_equal(vf["ref"], vt["ref"])
        tf, tt = fused.triangles(), two.triangles()
        assert len(tf) == len(tt)
        assert sorted(map(bytes, tf)) == sorted(map(bytes, tt))
        # a vertex the unrefined types drop and the refined ones keep is
        # re-born by the two passes but never dropped by the fused one
        nf, nt = fused.births(), two.births()
        assert (nf <= nt).all()
        for v in (fused, two, plain):
            v.gc()
    assert differs
