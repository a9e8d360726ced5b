"""The serving scheduler on the CPU: the arena allocator and the batch former
of the continuous-batching server, driven against a simulated device (batches
finish in a seeded random order after random delays), built with AddressSanitizer
and UndefinedBehaviorSanitizer; and the arena bytes the server reserves per
batch against what the batched call needs (through the C ABI, host arithmetic
only)."""
import subprocess
from pathlib import Path

import numpy as np

from paper_2605_17869_amd import sift as S

ROOT = Path(__file__).resolve().parents[1]

SIM = r"""
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <vector>
#include "sift_sched.h"
using namespace sift;

struct Req { long id; int64_t region; };
struct Run { int64_t off, bytes; long first, n; int left; };

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s line %d trial %d\n", #c, __LINE__, trial); ++fails; } } while (0)

int main() {
  unsigned seed = 2024;
  auto rnd = [&](int lo, int hi) {
    seed = seed * 1103515245u + 12345u;
    return lo + (int)((seed >> 8) % (unsigned)(hi - lo + 1));
  };
  for (int trial = 0; trial < 400; ++trial) {
    const int max_batch = rnd(1, 64), max_inflight = rnd(1, 8);
    const long n_req = rnd(1, 300);
    // request regions: 1..40 MiB in 256-byte units
    std::vector<int64_t> region(n_req);
    int64_t biggest = 0;
    for (long i = 0; i < n_req; ++i) {
      region[i] = (int64_t)rnd(1, 40 * 4096) * 256;
      if (region[i] > biggest) biggest = region[i];
    }
    // any arena that holds the largest single request (as admission demands)
    const int64_t arena_size = batch_bytes(1, biggest) + (int64_t)rnd(0, 200) * (1 << 20);
    Arena a;
    a.reset(arena_size);
    std::deque<Req> pending;
    std::vector<Run> flying;
    long next_arrival = 0, served = 0, expect_next = 0;
    int64_t in_use = 0;
    int steps = 0;
    while (served < n_req) {
      CHECK(++steps < 100000);
      if (steps >= 100000) break;
      // arrivals
      for (int k = rnd(0, 5); k > 0 && next_arrival < n_req; --k, ++next_arrival)
        pending.push_back(Req{next_arrival, region[next_arrival]});
      // the worker: launch while a stream is free and the head fits
      while (!pending.empty() && (int)flying.size() < max_inflight) {
        int64_t bytes = 0;
        const int n = next_batch(pending, max_batch, a.largest(), &bytes);
        if (n == 0) break;
        CHECK(n <= max_batch && bytes <= a.largest());
        int64_t regs = 0;
        for (int i = 0; i < n; ++i) regs += pending[i].region;
        CHECK(bytes == batch_bytes(n, regs));
        // the prefix is maximal: one more request would not fit or exceeds max_batch
        if (n < max_batch && n < (int)pending.size())
          CHECK(batch_bytes(n + 1, regs + pending[n].region) > a.largest());
        const int64_t off = a.take(bytes);
        CHECK(off >= 0 && off % 256 == 0 && off + bytes <= arena_size);
        for (const Run& r : flying)   // disjoint from every range in use
          CHECK(off + bytes <= r.off || r.off + r.bytes <= off);
        // arrival order: batches start at the oldest pending request
        CHECK(pending.front().id == expect_next);
        expect_next += n;
        flying.push_back(Run{off, bytes, pending.front().id, n, rnd(1, 6)});
        in_use += align_up256(bytes);
        pending.erase(pending.begin(), pending.begin() + n);
      }
      CHECK(in_use + a.free_bytes() == a.size());
      // an idle device always admits the head (the arena is whole again)
      if (flying.empty() && !pending.empty()) CHECK(a.largest() == a.size());
      // the simulated device: batches finish in random order
      for (size_t i = 0; i < flying.size();) {
        if (--flying[i].left <= 0 || rnd(0, 3) == 0) {
          a.give(flying[i].off, flying[i].bytes);
          in_use -= align_up256(flying[i].bytes);
          served += flying[i].n;
          flying.erase(flying.begin() + i);
        } else {
          ++i;
        }
      }
    }
    CHECK(served == n_req && pending.empty() && flying.empty());
    CHECK(a.largest() == a.size() && a.free_bytes() == a.size());
  }
  printf("fails=%d\n", fails);
  return fails != 0;
}
"""


def test_scheduler_against_a_simulated_device(tmp_path):
    src = tmp_path / "sim.cpp"
    src.write_text(SIM)
    exe = tmp_path / "sim"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined",
                    "-I", str(ROOT / "paper_2605_17869_amd" / "csrc"), "-I", str(ROOT / "include"),
                    str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "fails=0" in r.stdout


def test_server_batch_bytes_cover_the_batched_call():
    """The arena bytes the server reserves for a batch are at least what
    sift_extract_batch needs for it, however the call splits it into
    sub-batches (n_streams 0..8)."""
    rng = np.random.default_rng(5)
    for upsample in (0, 1):
        base = dict(n_octaves=3, upsample=upsample)
        for n in list(range(1, 17)) + [23, 40, 64]:
            sizes = [(int(rng.integers(60, 900)), int(rng.integers(60, 900))) for _ in range(n)]
            srv = S.server_batch_bytes(base, sizes)
            for streams in range(0, 9):
                need = S.Extractor(dict(base, n_streams=streams)).batch_workspace_size(sizes)
                assert srv >= need, (n, streams, srv, need)
            assert srv % 256 == 0
