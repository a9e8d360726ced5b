"""The host runtime (csrc/sift_api.cpp, sift_graph.cpp, sift_server.cpp,
sift_match.cpp, sift_verify.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side and driven through the C ABI on
the CPU: parameter validation, workspace and arena sizing, and the argument
errors every entry point reports before it enqueues anything.  The kernel
launchers are replaced by stubs (no GPU here; nothing in the driver reaches a
launch)."""
import os
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2605_17869_amd" / "csrc"

STUB = r"""
#include "sift_launch.h"
#include "sift_match.h"
#include "sift_verify.h"
namespace sift {
hipError_t launch_setup(const HdrPtrs&, const SetupChunk&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_finalize(const HdrPtrs&, int, const DevParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_blur(const BlurArgs&, int, int, hipStream_t) { return hipErrorNotSupported; }
bool chain_supported(int, int, int, const int*) { return false; }
hipError_t launch_chain(const ChainArgs&, int, int, int, const int*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_detect(char*, const HdrPtrs&, int, const DevParams&, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_band_scan(char*, const HdrPtrs&, int, const DevParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_emit(char*, const HdrPtrs&, int, const DevParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_img_prefix(char*, const HdrPtrs&, int, const DevParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_refine(char*, const HdrPtrs&, int, const DevParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_orient(char*, const HdrPtrs&, int, const DevParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_ori_scan(char*, const HdrPtrs&, int, const DevParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_describe(char*, const HdrPtrs&, int, const DevParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_match_setup(const MatchHdr&, const MatchSetupChunk&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_match_rows(const MatchHdr&, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_match_cols(const MatchHdr&, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_match_emit(const MatchHdr&, int, float, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_verify_setup(const VerifyHdr&, const VerifySetupChunk&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_verify_prep(const VerifyHdr&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_verify_models(const VerifyHdr&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_verify_hyp(const VerifyHdr&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_verify_refine(const VerifyHdr&, int, hipStream_t) { return hipErrorNotSupported; }
}  // namespace sift
"""

DRIVER = r"""
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>
#include "sift.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s line %d\n", #c, __LINE__); ++fails; } } while (0)

int main() {
  sift_params p;
  CHECK(sift_params_default(&p) == SIFT_OK);
  CHECK(sift_params_default(nullptr) == SIFT_ERR_INVALID_ARG);
  CHECK(std::strlen(sift_status_string(SIFT_ERR_HIP)) > 0);
  // bad settings are refused with a message
  const int bad_chain[2] = {-1, 5};
  for (int b : bad_chain) {
    sift_params q = p;
    q.blur_chain = b;
    sift_handle* h = nullptr;
    CHECK(sift_create(&q, &h) == SIFT_ERR_INVALID_ARG && h == nullptr);
    CHECK(std::strlen(sift_last_error()) > 0);
  }
  const int bad_waves[3] = {2, 16, -4};
  for (int b : bad_waves) {
    sift_params q = p;
    q.detect_waves = b;
    sift_handle* h = nullptr;
    CHECK(sift_create(&q, &h) == SIFT_ERR_INVALID_ARG && h == nullptr);
  }
  sift_params q0 = p;
  q0.n_scales = 0;
  sift_handle* h0 = nullptr;
  CHECK(sift_create(&q0, &h0) != SIFT_OK);
  CHECK(sift_create(nullptr, &h0) == SIFT_ERR_INVALID_ARG);

  const int32_t hs[6] = {480, 768, 333, 97, 1066, 61};
  const int32_t ws[6] = {640, 1024, 70, 129, 1600, 53};
  for (int up = 0; up < 2; ++up)
    for (int f16 = 0; f16 < 2; ++f16)
      for (int chain = 0; chain <= 4; ++chain) {
        sift_params q = p;
        q.upsample = up;
        q.pyramid_fp16 = f16;
        q.blur_chain = chain;
        q.detect_waves = chain % 2 ? 8 : 4;
        q.n_octaves = 3;
        sift_handle* h = nullptr;
        CHECK(sift_create(&q, &h) == SIFT_OK && h != nullptr);
        if (!h) continue;
        sift_params back;
        CHECK(sift_get_params(h, &back) == SIFT_OK && back.blur_chain == chain &&
              back.detect_waves == q.detect_waves);
        size_t a = 0, b = 0;
        CHECK(sift_workspace_size(h, 480, 640, &a) == SIFT_OK && a > 0);
        CHECK(sift_workspace_size(h, 960, 1280, &b) == SIFT_OK && b > a);
        CHECK(sift_workspace_size(h, 20, 20, &a) == SIFT_ERR_IMAGE_TOO_SMALL);
        CHECK(sift_workspace_size(h, 0, 640, &a) != SIFT_OK);
        CHECK(sift_workspace_size(h, 40000, 640, &a) != SIFT_OK);
        CHECK(sift_workspace_size(h, 480, 640, nullptr) == SIFT_ERR_INVALID_ARG);
        // a batch's workspace holds every image's region
        size_t batch = 0;
        CHECK(sift_batch_workspace_size(h, 6, hs, ws, &batch) == SIFT_OK);
        size_t largest = 0;
        for (int i = 0; i < 6; ++i) {
          size_t one = 0;
          CHECK(sift_workspace_size(h, hs[i], ws[i], &one) == SIFT_OK);
          largest = one > largest ? one : largest;
        }
        CHECK(batch > largest);
        // the serving arena reserves at least what the batched call needs
        for (int n = 1; n <= 6; ++n) {
          size_t need = 0, arena = 0;
          CHECK(sift_batch_workspace_size(h, n, hs, ws, &need) == SIFT_OK);
          CHECK(sift_server_batch_bytes(&q, n, hs, ws, &arena) == SIFT_OK && arena >= need);
        }
        // the tuner's workspace holds every candidate split
        size_t tune = 0;
        CHECK(sift_autotune_workspace_size(&q, 6, hs, ws, &tune) == SIFT_OK && tune >= batch);
        size_t bucket = 0;
        CHECK(sift_bucket_workspace_size(h, 8, 1024, 1024, &bucket) == SIFT_OK && bucket > 0);
        // argument errors come back before anything is enqueued
        sift_output out;
        std::memset(&out, 0, sizeof out);
        alignas(256) static char fake_ws[1024];
        const float* img = reinterpret_cast<const float*>(0x100000);
        CHECK(sift_extract(h, nullptr, 480, 640, 640, fake_ws, sizeof fake_ws, &out, nullptr) ==
              SIFT_ERR_INVALID_ARG);
        CHECK(sift_extract(h, img, 480, 640, 640, fake_ws, sizeof fake_ws, &out, nullptr) ==
              SIFT_ERR_INVALID_ARG);   // null output pointers
        out.keypoints = reinterpret_cast<sift_keypoint*>(0x200000);
        out.descriptors = reinterpret_cast<float*>(0x300000);
        out.count = reinterpret_cast<int32_t*>(0x400000);
        out.capacity = 16;
        CHECK(sift_extract(h, img, 480, 640, 600, fake_ws, sizeof fake_ws, &out, nullptr) ==
              SIFT_ERR_INVALID_ARG);   // pitch < width
        CHECK(sift_extract(h, img, 480, 640, 640, fake_ws + 8, sizeof fake_ws - 8, &out, nullptr) ==
              SIFT_ERR_INVALID_ARG);   // misaligned workspace
        CHECK(sift_extract(h, img, 480, 640, 640, fake_ws, sizeof fake_ws, &out, nullptr) ==
              SIFT_ERR_WORKSPACE_TOO_SMALL);
        sift_destroy(h);
      }

  // matcher and verifier sizing and argument checks (host arithmetic only)
  std::vector<sift_match_pair> mp(3);
  std::memset(mp.data(), 0, sizeof(sift_match_pair) * mp.size());
  for (int i = 0; i < 3; ++i) {
    mp[i].desc_a = reinterpret_cast<const float*>(0x100000);
    mp[i].desc_b = reinterpret_cast<const float*>(0x200000);
    mp[i].cap_a = 1000 + 500 * i;
    mp[i].cap_b = 2000;
    mp[i].matches = reinterpret_cast<sift_match*>(0x300000);
    mp[i].n_matches = reinterpret_cast<int32_t*>(0x400000);
    mp[i].capacity = 1000 + 500 * i;
  }
  size_t mbytes = 0;
  CHECK(sift_match_workspace_size(3, mp.data(), &mbytes) == SIFT_OK && mbytes > 0);
  CHECK(sift_match_workspace_size(0, mp.data(), &mbytes) != SIFT_OK);
  mp[1].cap_a = SIFT_MATCH_MAX_ROWS + 1;
  CHECK(sift_match_workspace_size(3, mp.data(), &mbytes) == SIFT_ERR_INVALID_ARG);
  std::vector<sift_verify_pair> vp(2);
  std::memset(vp.data(), 0, sizeof(sift_verify_pair) * vp.size());
  for (int i = 0; i < 2; ++i) {
    vp[i].kp_a = reinterpret_cast<const sift_keypoint*>(0x100000);
    vp[i].kp_b = reinterpret_cast<const sift_keypoint*>(0x200000);
    vp[i].matches = reinterpret_cast<const sift_match*>(0x300000);
    vp[i].cap = 500 + 700 * i;
    vp[i].H = reinterpret_cast<double*>(0x400000);
    vp[i].score = reinterpret_cast<double*>(0x500000);
    vp[i].n_inliers = reinterpret_cast<int32_t*>(0x600000);
  }
  size_t vbytes = 0;
  CHECK(sift_verify_workspace_size(2, vp.data(), 1500, &vbytes) == SIFT_OK && vbytes > 0);
  CHECK(sift_verify_workspace_size(2, vp.data(), SIFT_VERIFY_MAX_HYPOTHESES + 1, &vbytes) ==
        SIFT_ERR_INVALID_ARG);
  alignas(256) static char vws[256];
  CHECK(sift_verify_batch(2, vp.data(), reinterpret_cast<const float*>(0x700000), 1500, 0.0f, 5,
                          vws, sizeof vws, nullptr) == SIFT_ERR_INVALID_ARG);   // sigma_max <= 0
  CHECK(sift_verify_batch(2, vp.data(), reinterpret_cast<const float*>(0x700000), 1500, 2.0f, 5,
                          vws, sizeof vws, nullptr) == SIFT_ERR_WORKSPACE_TOO_SMALL);
  if (fails == 0) std::printf("OK\n");
  return fails == 0 ? 0 : 1;
}
"""

SOURCES = ["sift_api.cpp", "sift_graph.cpp", "sift_server.cpp", "sift_match.cpp", "sift_verify.cpp"]


def hipcc():
    root = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = Path(root) / "bin" / "hipcc"
    return str(cand) if cand.exists() else "hipcc"


def test_host_runtime_under_sanitizers(tmp_path):
    if subprocess.run([hipcc(), "--version"], capture_output=True).returncode != 0:
        pytest.skip("hipcc not available")
    drv = tmp_path / "driver.cpp"
    stub = tmp_path / "stub.cpp"
    drv.write_text(DRIVER)
    stub.write_text(STUB)
    flags = ["-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
             "-I", str(CSRC), "-I", str(ROOT / "include"),
             "-Xarch_host", "-fsanitize=address,undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w"]
    objs, procs = [], []
    for src in [*(CSRC / s for s in SOURCES), stub, drv]:
        obj = tmp_path / (src.name + ".o")
        procs.append(subprocess.Popen([hipcc(), *flags, "-c", str(src), "-o", str(obj)],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for pr in procs:
        out, _ = pr.communicate()
        assert pr.returncode == 0, out.decode(errors="replace")[-3000:]
    exe = tmp_path / "runtime_asan"
    link = subprocess.run([hipcc(), "--offload-arch=gfx950", "-Xarch_host",
                           "-fsanitize=address,undefined", "-o", str(exe), *map(str, objs)],
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stdout[-2000:] + link.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and "OK" in run.stdout, run.stdout[-3000:] + run.stderr[-3000:]
