"""The library's refinement (per-type candidate tables and a byte-wise test
of the flipped corners, shared by its kernels and compiled here for the
host) against the oracle's Eqs. (3)-(5) on every input: all 2^8 types, all
2^8 previous types and all 2^8 patterns of near-zero corners."""
import os
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1803_03949_amd", "csrc")

PROBE = r"""
#include <dlfcn.h>
#include <stdio.h>
#include "vm_internal.h"
typedef int (*orc_refine_type_t)(int, int, const float*, float);
int main(int argc, char** argv) {
  void* h = dlopen(argv[1], RTLD_NOW);
  if (!h) { printf("dlopen failed\n"); return 2; }
  orc_refine_type_t ref = (orc_refine_type_t)dlsym(h, "orc_refine_type");
  if (!ref) { printf("no orc_refine_type\n"); return 2; }
  uint64_t cand[256];
  int regular = 0;
  for (uint32_t t = 0; t < 256; ++t) cand[t] = vm::refine_candidates(t), regular += (int)(cand[t] >> 63);
  long bad = 0, refined = 0;
  const float eps = 0.5f;
  for (uint32_t near8 = 0; near8 < 256; ++near8) {
    float d[8];
    for (int k = 0; k < 8; ++k) d[k] = ((near8 >> k) & 1u) ? 0.25f : 2.0f;
    for (uint32_t t = 0; t < 256; ++t)
      for (uint32_t p = 0; p < 256; ++p) {
        const uint32_t got = vm::refine_type(t, p, (cand[p] >> 63) != 0, near8, cand[t]);
        const uint32_t want = (uint32_t)ref((int)t, (int)p, d, eps);
        bad += got != want;
        refined += want != t;
      }
  }
  printf("%d %ld %ld\n", regular, refined, bad);
  return 0;
}
"""


def test_library_refinement_equals_the_oracle_on_every_input(tmp_path):
    lib = oracle.build(force=False)
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC, str(src), "-o", str(exe),
                        "-ldl"], capture_output=True, text=True)
    if r.returncode != 0 and "not found" in r.stderr:
        pytest.skip("hipcc not available")
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe), lib], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    regular, refined, bad = (int(x) for x in out.stdout.split())
    assert regular == 6          # the six printed regular types flag themselves
    assert refined > 1_000_000   # the search is not vacuous
    assert bad == 0
