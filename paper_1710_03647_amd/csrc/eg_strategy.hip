// Player 0's positional strategy read off the least progress measure.
//
// Def. 5 asks of a progress measure f that every player-0 vertex v have an
// out-edge (v, u) with f(v) >= f(u) (-) w(v, u).  Following such an edge from
// each player-0 vertex with finite f(v) is a winning positional strategy with
// initial credit f(v): along the edge f(v) + w >= f(u), so a play that starts
// with credit f(v) keeps its energy >= f of its current vertex >= 0, and no
// play leaves the finite part of f (Lemma 1 then holds for the strategy's
// graph).  The choice is the first such edge of the row, so it is unique.
//
// In the device encoding (TOP = B + P + 1, stored weights <= P) the condition
// for a finite f(v) <= B is f(u) - w <= f(v): a TOP successor gives at least
// B + 1, and the floor of (-) at 0 never decides since f(v) >= 0.  A weight
// clamped to P = B + 1 decides as the original one would: below 0 for a
// finite f(u), above B for TOP.
//
// One lane per vertex scans a row of at most SHORT_ROW edges and stops at the
// first witness; longer rows are handed to the whole wave, 64 edges per step,
// so that a hub costs deg / 64 steps.
#include "eg_internal.h"

namespace eg {
namespace {

constexpr int SWAVE = 64;
constexpr int SBLOCK = 256;
constexpr uint32_t SHORT_ROW = 32;

template <typename V>
__global__ __launch_bounds__(SBLOCK) void k_strategy(DevGame g, int32_t* choice, uint32_t* missing) {
  const V* f = (const V*)g.f;
  const V top = (V)g.top;
  const uint32_t n = (uint32_t)g.n;
  const uint32_t lane = __lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  // c0 is the wave's first vertex: the same in every lane, so ballots see the whole wave
  for (uint32_t c0 = blockIdx.x * blockDim.x + threadIdx.x - lane; c0 < n; c0 += stride) {
    const uint32_t c = c0 + lane;
    bool need = false;
    uint32_t beg = 0, deg = 0;
    V fv = 0;
    if (c < n) {
      const uint32_t v = g.perm ? (uint32_t)g.perm[c] : c;
      const uint32_t raw = g.rs[v];
      fv = f[v];
      if (!(raw & OWNER_BIT) && fv != top) {
        beg = raw & ROW_MASK;
        deg = (g.rs[v + 1] & ROW_MASK) - beg;
        need = true;
      }
    }
    int32_t pick = -1;
    if (need && deg <= SHORT_ROW) {
      for (uint32_t k = 0; k < deg; k++) {
        const int2 e = g.edges[beg + k];
        if ((V)f[e.x] - (V)e.y <= fv) {
          pick = (int32_t)k;
          break;
        }
      }
    }
    unsigned long long longs = __ballot(need && deg > SHORT_ROW);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(beg, (int)src, SWAVE);
      const uint32_t d = __shfl(deg, (int)src, SWAVE);
      const V x = __shfl(fv, (int)src, SWAVE);
      int32_t found = -1;  // wave-uniform: it comes from a ballot
      for (uint32_t k0 = 0; k0 < d && found < 0; k0 += SWAVE) {
        const uint32_t k = k0 + lane;
        bool hit = false;
        if (k < d) {
          const int2 e = g.edges[b + k];
          hit = (V)f[e.x] - (V)e.y <= x;
        }
        const unsigned long long hits = __ballot(hit);
        if (hits) found = (int32_t)(k0 + (uint32_t)__ffsll((long long)hits) - 1);
      }
      if (lane == src) pick = found;
    }
    if (c < n) {
      choice[c] = pick;
      if (need && pick < 0) atomicAdd(missing, 1u);
    }
  }
}

}  // namespace

hipError_t launch_strategy(const DevGame& g, int vbits, int32_t* choice, uint32_t* missing, hipStream_t s) {
  const uint32_t blocks = std::min<uint32_t>(((uint32_t)g.n + SBLOCK - 1) / SBLOCK, 1u << 16);
  if (vbits == 32) hipLaunchKernelGGL(k_strategy<int32_t>, dim3(blocks), dim3(SBLOCK), 0, s, g, choice, missing);
  else hipLaunchKernelGGL(k_strategy<int64_t>, dim3(blocks), dim3(SBLOCK), 0, s, g, choice, missing);
  return hipGetLastError();
}

}  // namespace eg
