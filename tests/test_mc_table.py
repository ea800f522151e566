"""The library's marching-cubes tables (built on the host when a volume is
created) against the oracle's per-cube polygons, for all 256 types: the same
triangles with the same orientation, and per-edge use counts that match
them.  The two sides build their polygons independently (an entry/exit walk
round each face here, a geometric orientation test in the oracle)."""
import os
import subprocess

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLES = os.path.join(ROOT, "paper_1803_03949_amd", "csrc", "vm_tables.hip")

PROBE = r"""
#include <stdio.h>
#include "TABLES"
int main() {
  static uint8_t tri[256 * 16], uses[256 * 12];
  vm::build_mc_tables(tri, uses);
  for (int t = 0; t < 256; ++t) {
    for (int k = 0; k < 16; ++k) printf("%d ", tri[t * 16 + k]);
    for (int e = 0; e < 12; ++e) printf("%d ", uses[t * 12 + e]);
    printf("\n");
  }
  return 0;
}
"""


def canonical(tris):
    """Triangles as rotations starting at their smallest edge (orientation
    kept), sorted."""
    out = []
    for a, b, c in np.asarray(tris).reshape(-1, 3).tolist():
        r = [(a, b, c), (b, c, a), (c, a, b)]
        out.append(min(r, key=lambda x: x[0]))
    return sorted(out)


def test_library_tables_equal_the_oracle_polygons(tmp_path):
    src = tmp_path / "probe.cpp"
    src.write_text(PROBE.replace("TABLES", TABLES))
    exe = tmp_path / "probe"
    r = subprocess.run(["g++", "-std=c++17", "-x", "c++", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines()
    assert len(rows) == 256
    for t, row in enumerate(rows):
        v = [int(x) for x in row.split()]
        tri, uses = v[:16], v[16:]
        n = tri[0]
        lib_tris = np.array(tri[1:1 + 3 * n]).reshape(n, 3)
        assert all(x == 255 for x in tri[1 + 3 * n:]), t
        want = oracle.cube_triangles(t)
        assert canonical(lib_tris) == canonical(want), t
        counts = np.bincount(lib_tris.ravel(), minlength=12) if n else np.zeros(12, int)
        assert list(counts) == uses, t
