// Driver of the host validation path of libeg (eg_check) for sanitizer builds:
// every rejection cause, the overflow guard of the bound, and seeded random
// games of every size class, each with its expected status.  Exits 0 when
// every status is as expected; the sanitizers abort on any memory or
// undefined-behaviour error.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "eg.h"

namespace {

int failures = 0;

struct Arena {
  std::vector<int64_t> off;
  std::vector<int32_t> tgt, w;
  std::vector<uint8_t> own;
  int32_t W = 0;
  eg_game_desc desc() {
    return eg_game_desc{(int32_t)off.size() - 1, off.back(), off.data(), tgt.empty() ? nullptr : tgt.data(),
                        w.empty() ? nullptr : w.data(), own.data(), W, EG_MEM_HOST};
  }
};

// SplitMix64 (Vigna), for reproducible inputs
uint64_t mix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

Arena random_arena(uint64_t seed, int32_t n, int32_t max_deg, int32_t wlim) {
  Arena a;
  uint64_t s = seed;
  a.off.push_back(0);
  for (int32_t v = 0; v < n; v++) {
    const int32_t d = 1 + (int32_t)(mix(s) % (uint64_t)max_deg);
    for (int32_t k = 0; k < d; k++) {
      a.tgt.push_back((int32_t)(mix(s) % (uint64_t)n));
      a.w.push_back((int32_t)(mix(s) % (uint64_t)(2 * wlim + 1)) - wlim);
    }
    a.off.push_back((int64_t)a.tgt.size());
  }
  a.own.assign(((size_t)n + 7) / 8, 0);
  for (int32_t v = 0; v < n; v++)
    if (mix(s) & 1) a.own[(size_t)v / 8] |= (uint8_t)(1u << (v % 8));
  a.W = wlim;
  return a;
}

void expect(const char* what, const eg_game_desc* d, int bound_mode, int want) {
  eg_game_info info;
  char msg[256];
  const int rc = eg_check(d, bound_mode, &info, msg, sizeof msg);
  if (rc != want) {
    printf("FAIL %s: status %d, expected %d (%s)\n", what, rc, want, msg);
    failures++;
  }
}

}  // namespace

int main() {
  // valid games of several size classes, both bound modes
  for (uint64_t seed = 1; seed <= 40; seed++) {
    Arena a = random_arena(seed, 1 + (int32_t)(seed * 37 % 3000), 1 + (int32_t)(seed % 17), 1 + (int32_t)(seed * 13));
    eg_game_desc d = a.desc();
    expect("random valid", &d, EG_BOUND_NW, EG_OK);
    expect("random valid, M_G", &d, EG_BOUND_MG, EG_OK);
  }
  Arena base = random_arena(99, 50, 4, 10);
  {
    eg_game_desc d = base.desc();
    expect("null descriptor", nullptr, EG_BOUND_NW, EG_EINVAL);
    d.n = 0;
    expect("n = 0", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    d.m = -1;
    expect("m < 0", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    d.m = (int64_t)1 << 31;
    expect("m = 2^31", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    d.offsets = nullptr;
    expect("null offsets", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    d.targets = nullptr;
    expect("null targets", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    d.W = -1;
    expect("W < 0", &d, EG_BOUND_NW, EG_EINVAL);
    d = base.desc();
    expect("unknown bound mode", &d, 7, EG_EINVAL);
    d.mem = EG_MEM_DEVICE;
    expect("device pointers", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    Arena a = base;
    a.off[0] = 1;
    eg_game_desc d = a.desc();
    d.m = base.off.back();
    expect("offsets[0] != 0", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    Arena a = base;
    eg_game_desc d = a.desc();
    d.m = base.off.back() - 1;
    expect("offsets[n] != m", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    Arena a = base;
    std::swap(a.off[10], a.off[11]);
    if (a.off[10] == a.off[11]) a.off[10]++;
    eg_game_desc d = a.desc();
    expect("decreasing or empty rows", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    Arena a = base;
    a.tgt[5] = 50;
    eg_game_desc d = a.desc();
    expect("target = n", &d, EG_BOUND_NW, EG_EINVAL);
    a.tgt[5] = -1;
    d = a.desc();
    expect("target < 0", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    // vertex 1 without out-edges: the arena is not total
    Arena a;
    a.off = {0, 1, 1, 2};
    a.tgt = {1, 0};
    a.w = {0, 0};
    a.own = {0};
    eg_game_desc d = a.desc();
    expect("out-degree 0", &d, EG_BOUND_NW, EG_EINVAL);
  }
  {
    Arena a = base;
    a.w[3] = -11;
    eg_game_desc d = a.desc();
    expect("W below the largest negative magnitude", &d, EG_BOUND_NW, EG_EINVAL);
    a.W = 11;
    d = a.desc();
    expect("W at it", &d, EG_BOUND_NW, EG_OK);
  }
  {
    // (n - 1) * W + P + 1 + W beyond int64: rejected; n large with W = INT32_MAX fits
    Arena a;
    a.off = {0, 1, 2};
    a.tgt = {1, 0};
    a.w = {INT32_MIN + 1, INT32_MAX};
    a.own = {1};
    a.W = INT32_MAX;
    eg_game_desc d = a.desc();
    expect("extreme weights, 2 vertices", &d, EG_BOUND_NW, EG_OK);
    Arena b = random_arena(7, 3000, 3, 5);
    b.W = INT32_MAX;
    d = b.desc();
    expect("W = INT32_MAX, 3000 vertices", &d, EG_BOUND_NW, EG_OK);
  }
  printf("%s: %d failures\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
