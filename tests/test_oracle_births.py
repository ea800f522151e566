"""The oracle's vertex birth frames, pinned by set algebra over from-scratch
extractions (CPU only).

Reading (the paper visualises how long each vertex has been held, Fig. 1,
without defining it): frames count integrations and imports from 1; at the
end of every extraction or refinement a vertex whose count is positive, but
was not at the end of the previous pass, is stamped with the current frame.
From-scratch vertex sets are pinned elsewhere (incremental == from scratch),
so the expected stamps follow from which sets a vertex's edge belongs to."""
import numpy as np

import oracle
import scenes


def sphere(seed, radius):
    sv = scenes.sphere_volume(seed=seed, dims_blocks=(4, 4, 4), voxel_m=0.008, radius=radius,
                              center=np.full(3, 0.128), jitter=0.0)
    return sv.blocks()


def keyset(o):
    return {tuple(k) for k in o.vertices()["keys"].tolist()}


def scratch(fields):
    o = oracle.OracleVolume(0.008)
    o.import_blocks(*fields)
    o.extract(scope_all=True)
    return keyset(o)


def births_by_key(o):
    return dict(zip(map(tuple, o.vertices()["keys"].tolist()), o.births().tolist()))


A, B = sphere(1, 0.100), sphere(1, 0.104)


def test_one_import_all_born_in_frame_one():
    o = oracle.OracleVolume(0.008)
    o.import_blocks(*A)
    o.extract(scope_all=True)
    b = o.births()
    assert len(b) > 1000 and (b == 1).all()


def test_second_field_births_follow_set_membership():
    sa, sb = scratch(A), scratch(B)
    assert sa & sb and sb - sa  # both kinds occur
    o = oracle.OracleVolume(0.008)
    o.import_blocks(*A)
    o.extract(scope_all=True)
    o.gc()
    o.import_blocks(*B)
    o.extract(scope_all=True)
    o.gc()
    got = births_by_key(o)
    assert set(got) == sb
    assert all(got[k] == (1 if k in sa else 2) for k in got)


def test_vertices_lost_and_regained_are_reborn():
    sa, sb = scratch(A), scratch(B)
    o = oracle.OracleVolume(0.008)
    for fields in (A, B, A):
        o.import_blocks(*fields)
        o.extract(scope_all=True)
        o.gc()
    got = births_by_key(o)
    assert set(got) == sa
    assert all(got[k] == (1 if k in sb else 3) for k in got)
    assert any(v == 3 for v in got.values())


def test_a_frame_without_extraction_stamps_nothing():
    o = oracle.OracleVolume(0.008)
    o.import_blocks(*A)          # frame 1, not extracted
    o.import_blocks(*A)          # frame 2
    o.extract(scope_all=True)
    assert (o.births() == 2).all()
