// Driver of the host-only self-tests, built with AddressSanitizer and
// UndefinedBehaviorSanitizer over the library's host sources (see
// build.py: build_sanitized).  Needs no GPU: it runs the pool / index stress
// test, the BF16 launch planner on random row groups, the per-layer
// readiness segments against a brute-force count, the setup orchestrator
// with stand-in stages, and argument errors.  Exit status 0 when every check
// passed; a sanitizer report aborts the process.
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/sage.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s (%s)\n", what, sage_last_error());
    failures++;
  }
}

int main() {
  // pool and fingerprint index
  for (uint64_t seed = 0; seed < 24; seed++)
    for (uint32_t budget : {1u, 3u, 17u, 64u, 300u}) {
      uint32_t at = 0;
      expect(sage_selftest_pool(seed, 4000, budget, &at) == SAGE_OK && at == 4000, "pool stress");
    }
  uint32_t at = 0;
  expect(sage_selftest_pool(0, 10, 0, &at) == SAGE_EINVAL, "pool stress rejects a zero budget");
  expect(sage_selftest_pool(0, 10, 4, nullptr) == SAGE_EINVAL, "pool stress rejects a null output");

  // planner on random groups
  std::mt19937_64 rng(7);
  const char* shapes[] = {"ggemm6p_bf16_256x256", "ggemm6_bf16_256x128", "ggemm_bf16_128x128",
                          "ggemm3t_bf16_32x32", "ggemm3t_bf16_16x16", "ggemm3g4_bf16_32x64"};
  const double wave[] = {0.125, 0.07, 0.05, 0.019, 0.012, 0.03};
  for (int t = 0; t < 400; t++) {
    const size_t ng = 1 + rng() % 40;
    std::vector<uint32_t> rows(ng);
    for (auto& r : rows) r = 1 + (uint32_t)(rng() % 1200);
    const size_t ns = 1 + rng() % 6;
    char out[256];
    const sage_status st = sage_selftest_plan(4096, rows.data(), ng, shapes, wave, ns, 256, out, sizeof out);
    expect(st == SAGE_OK && std::strchr(out, ':') != nullptr, "planner");
  }
  const char* bad[] = {"no_such_shape"};
  char small[4];
  uint32_t one = 5;
  expect(sage_selftest_plan(4096, &one, 1, bad, wave, 1, 256, small, sizeof small) == SAGE_EINVAL,
         "planner rejects an unknown shape");

  // readiness segments against brute force
  for (int t = 0; t < 300; t++) {
    const uint32_t layers = 1 + (uint32_t)(rng() % 9);
    const uint64_t layer_bytes = (uint64_t)65536 * (1 + rng() % 6);
    const uint32_t nblk = (uint32_t)(layers * layer_bytes / 65536);
    std::vector<uint32_t> first;
    for (uint32_t b = 0; b < nblk; b++)
      if (rng() % 3) first.push_back(b);
    if (first.empty()) first.push_back(0);
    std::vector<size_t> seg(layers);
    expect(sage_selftest_segments(first.data(), first.size(), layers, layer_bytes, seg.data()) == SAGE_OK,
           "segments");
    for (uint32_t l = 0; l < layers; l++) {
      const uint64_t end_block = (l + 1) * layer_bytes / 65536;  // blocks of layers 0..l
      size_t want = 0;
      while (want < first.size() && first[want] < end_block) want++;
      expect(seg[l] == want, "segments against brute force");
    }
  }
  uint32_t dec[] = {3, 1};
  size_t seg2[2];
  expect(sage_selftest_segments(dec, 2, 2, 65536, seg2) == SAGE_EINVAL, "segments reject a decreasing order");

  // setup orchestrator: overlapped branches take about the longer one
  double ms = 0;
  expect(sage_selftest_setup_overlap(20, 5, 10, 0, &ms) == SAGE_OK && ms < 32, "overlapped setup");
  expect(sage_selftest_setup_overlap(20, 5, 10, 1, &ms) == SAGE_OK && ms >= 34, "serial setup");

  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("host self-tests passed\n");
  return 0;
}
