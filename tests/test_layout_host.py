"""Workspace layout invariants of the header the kernels and the host runtime
share (compiled for the host with g++; CPU only)."""
import subprocess
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]

PROG = r"""
#include <cstdio>
#include <cstdlib>
#include "sift_internal.h"
using namespace sift;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s line %d h=%d w=%d\n", #c, __LINE__, h, w); ++fails; } } while (0)
int main() {
  unsigned seed = 12345;
  auto rnd = [&](int lo, int hi) { seed = seed * 1103515245u + 12345u; return lo + (int)((seed >> 8) % (unsigned)(hi - lo + 1)); };
  for (int trial = 0; trial < 3000; ++trial) {
    int up = rnd(0, 1), s = rnd(1, kMaxScales), border = rnd(1, 8);
    int n_oct = rnd(1, 6);
    int need = 2 * border + 3;
    int minside = need << (n_oct - 1);
    if (up) minside = (minside + 1) / 2;
    int h = rnd(minside, minside + 900), w = rnd(minside, minside + 900);
    LayoutCfg c{n_oct + up, up, s, border, rnd(1, 5000), rnd(1, 70000)};
    RegionTail t = region_tail(h, w, c);
    int64_t prev_end = 256;
    int bands = 0;
    for (int k = 0; k < c.n_oct; ++k) {
      OctView v = octave_view(h, w, c, k);
      int eh = up ? 2 * h : h, ew = up ? 2 * w : w;
      for (int j = 0; j < k; ++j) { eh = (eh + 1) / 2; ew = (ew + 1) / 2; }
      CHECK(v.h == eh && v.w == ew);
      CHECK(v.pitch >= v.w && v.pitch % 64 == 0);
      CHECK(v.level0 % 256 == 0 && v.plane % 256 == 0);
      CHECK(v.plane >= (int64_t)v.pitch * v.h * 4);
      CHECK(v.level0 == prev_end);
      prev_end = v.level0 + v.plane * (s + 3);
      CHECK(v.band_base == bands);
      CHECK(v.nband * kBand >= v.h - 2 * border && (v.nband - 1) * kBand < v.h - 2 * border);
      CHECK(v.nseg * kSeg >= v.w - 2 * border && (v.nseg - 1) * kSeg < v.w - 2 * border);
      bands += v.nband;
      for (int lb = v.band_base; lb < v.band_base + v.nband; ++lb) {
        int kk, bb;
        band_owner(h, w, c, lb, &kk, &bb);
        CHECK(kk == k && bb == lb - v.band_base);
      }
    }
    int64_t mend = prev_end;
    for (int k = 0; k < c.n_oct; ++k) {
      OctView v = octave_view(h, w, c, k);
      CHECK(v.masks >= mend && v.masks % 256 == 0);
      mend = v.masks + (int64_t)s * v.h * v.nseg * 8;
    }
    CHECK(t.total_bands == bands);
    CHECK(t.band_cnt >= mend && t.band_off >= t.band_cnt + (int64_t)bands * s * 4);
    CHECK(t.cands >= t.band_off + (int64_t)bands * s * 4 && t.cands % 256 == 0);
    CHECK(t.refined >= t.cands + (int64_t)c.max_cand * 16);
    CHECK(t.n_ori >= t.refined + (int64_t)c.max_cand * 48);
    CHECK(t.angles >= t.n_ori + (int64_t)c.max_cand * 4);
    CHECK(t.kp_off >= t.angles + (int64_t)c.max_cand * kMaxPeaks * 4);
    CHECK(t.kp_src >= t.kp_off + (int64_t)c.max_cand * 4);
    CHECK(t.bytes >= t.kp_src + (int64_t)c.max_kp * 4);
  }
  for (int n = 1; n < 300; n += 37) {
    Header hd; make_header(n, &hd); int h = n, w = 0;
    CHECK(hd.tile_prefix >= (int64_t)n * (int64_t)sizeof(ImgEntry));
    CHECK(hd.band_prefix >= hd.tile_prefix + (int64_t)kNumTileH * kMaxOct * (n + 1) * 4);
    CHECK(hd.cand_prefix >= hd.band_prefix + (n + 1) * 4);
    CHECK(hd.kp_prefix >= hd.cand_prefix + (n + 1) * 4);
    CHECK(hd.queue >= hd.kp_prefix + (n + 1) * 4);
    CHECK(hd.bytes >= hd.queue + kQueues * 4 && hd.bytes % 256 == 0);
  }
  { int h = 0, w = 0; CHECK(sizeof(RefinedKp) == 48); CHECK(sizeof(ImgEntry) == 80); }
  printf("fails=%d\n", fails);
  return fails != 0;
}
"""


def test_layout_invariants(tmp_path):
    src = tmp_path / "layout.cpp"
    src.write_text(PROG)
    exe = tmp_path / "layout"
    subprocess.run(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined",
                    "-I", str(ROOT / "paper_2605_17869_amd" / "csrc"), "-I", str(ROOT / "include"),
                    str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "fails=0" in r.stdout
