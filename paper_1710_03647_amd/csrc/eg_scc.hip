// Strongly connected components of the game graph and the levels of its
// condensation, for the component schedule of eg_solve (the refinement the
// paper proposes after its results, Sec. 6: solve components in topological
// order).
//
// A vertex's value depends only on its successors, so the vertices of a
// component whose successors outside it all lie in components already solved
// reach their least-fixpoint values by iterating inside the component alone.
// Level 0 holds the components with no edge leaving them (sink components); a
// component's level is one more than the largest level of the components its
// edges reach.  The schedule solves level 0, then level 1 with level 0 fixed,
// and so on; every edge leaving a level ends in a lower one.
//
// Components are found by repeated phases over the vertices not yet assigned:
//  trim:   a vertex with no unassigned successor or no unassigned predecessor
//          other than itself is a component of its own;
//  colour: every vertex takes the largest id of the unassigned vertices that
//          reach it (a max over predecessors, iterated to a fixpoint);
//  mark:   from every root (a vertex whose colour is its own id) the vertices
//          of its colour that reach it, walking predecessor-wise (a vertex
//          joins when one of its successors of the same colour has joined);
//          they form the root's component (every vertex of that colour that
//          reaches the root is also reached from it, by the colouring).
// Each phase assigns at least the component of the largest unassigned id.
// Component labels are vertex ids: the root (or the trimmed vertex) itself.
//
// Rows of up to SCC_SHORT entries are scanned by their vertex's lane, longer
// ones by the whole wave, and in the colouring and level sweeps rows above
// SCC_LONG by a whole block.
#include "eg_internal.h"

namespace eg {

namespace {
constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr uint32_t SCC_SHORT = 32;
// Rows longer than this are listed once and folded by a whole block each in
// the colouring and level sweeps: the hubs of power-law games sit next to
// each other after renumbering, and one wave would take them in turn.
constexpr uint32_t SCC_LONG = 2048;
constexpr int SCC_LONG_GRID = 1024;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// barrier that first waits for this wave's LDS operations (atomics included)
__device__ __forceinline__ void block_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __syncthreads();
}

// Reductions over a row [b, e) of `idx` (out-edge targets or predecessor ids):
// any_of stops at the first hit, max_of folds the whole row.  The row belongs
// to the vertex of lane `src`; every lane of the wave calls these together.
template <typename Pred>
__device__ __forceinline__ bool wave_any(uint32_t b, uint32_t e, Pred pred) {
  const uint32_t lane = lane_id();
  for (uint32_t k0 = b; k0 < e; k0 += WAVE) {
    const uint32_t k = k0 + lane;
    const bool hit = k < e && pred(k);
    if (__ballot(hit)) return true;
  }
  return false;
}

template <typename Val>
__device__ __forceinline__ int32_t wave_max(uint32_t b, uint32_t e, int32_t acc, Val val) {
  const uint32_t lane = lane_id();
  for (uint32_t k = b + lane; k < e; k += WAVE) {
    const int32_t x = val(k);
    acc = x > acc ? x : acc;
  }
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t y = __shfl_xor(acc, o, WAVE);
    acc = y > acc ? y : acc;
  }
  return acc;
}

__device__ __forceinline__ uint32_t out_begin(const DevGame& g, uint32_t v) { return g.rs[v] & ROW_MASK; }
__device__ __forceinline__ uint32_t out_end(const DevGame& g, uint32_t v) { return g.rs[v + 1] & ROW_MASK; }

// trim: comp[v] = v for an unassigned v without an unassigned successor or
// predecessor other than itself
__global__ __launch_bounds__(BLOCK) void k_scc_trim(DevGame g, SccBuf sc) {
  const uint32_t n = (uint32_t)g.n, lane = lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t hits = 0;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane; v0 < n; v0 += stride) {
    const uint32_t v = v0 + lane;
    const bool live = v < n && sc.comp[v] < 0;
    uint32_t ob = 0, oe = 0, pb = 0, pe = 0;
    if (live) {
      ob = out_begin(g, v);
      oe = out_end(g, v);
      pb = g.rev_off[v];
      pe = g.rev_off[v + 1];
    }
    auto out_live = [&](uint32_t k, uint32_t self) {
      const int32_t u = g.edges[k].x;
      return (uint32_t)u != self && sc.comp[u] < 0;
    };
    auto in_live = [&](uint32_t k, uint32_t self) {
      const int32_t p = g.rev_src[k];
      return (uint32_t)p != self && sc.comp[p] < 0;
    };
    bool has_out = false, has_in = false;
    if (live && oe - ob <= SCC_SHORT)
      for (uint32_t k = ob; k < oe && !has_out; k++) has_out = out_live(k, v);
    if (live && pe - pb <= SCC_SHORT)
      for (uint32_t k = pb; k < pe && !has_in; k++) has_in = in_live(k, v);
    unsigned long long longs = __ballot(live && oe - ob > SCC_SHORT);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(ob, (int)src, WAVE), e = __shfl(oe, (int)src, WAVE), self = v0 + src;
      const bool any = wave_any(b, e, [&](uint32_t k) { return out_live(k, self); });
      if (lane == src) has_out = any;
    }
    longs = __ballot(live && pe - pb > SCC_SHORT);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(pb, (int)src, WAVE), e = __shfl(pe, (int)src, WAVE), self = v0 + src;
      const bool any = wave_any(b, e, [&](uint32_t k) { return in_live(k, self); });
      if (lane == src) has_in = any;
    }
    if (live && !(has_out && has_in)) {
      sc.comp[v] = (int32_t)v;
      hits++;
    }
  }
  if (hits) atomicAdd(sc.flag, hits);
}

// colour: color[v] = max(color[v], color[p]) over unassigned predecessors p
__global__ __launch_bounds__(BLOCK) void k_scc_color(DevGame g, SccBuf sc) {
  const uint32_t n = (uint32_t)g.n, lane = lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t hits = 0;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane; v0 < n; v0 += stride) {
    const uint32_t v = v0 + lane;
    const bool live = v < n && sc.comp[v] < 0;
    uint32_t pb = 0, pe = 0;
    int32_t c = -1;
    if (live) {
      pb = g.rev_off[v];
      pe = g.rev_off[v + 1];
      c = sc.color[v];
    }
    auto val = [&](uint32_t k) {
      const int32_t p = g.rev_src[k];
      return sc.comp[p] < 0 ? sc.color[p] : -1;
    };
    int32_t best = c;
    if (live && pe - pb <= SCC_SHORT)
      for (uint32_t k = pb; k < pe; k++) {
        const int32_t x = val(k);
        best = x > best ? x : best;
      }
    unsigned long long longs = __ballot(live && pe - pb > SCC_SHORT && pe - pb <= SCC_LONG);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(pb, (int)src, WAVE), e = __shfl(pe, (int)src, WAVE);
      const int32_t m = wave_max(b, e, -1, val);
      if (lane == src) best = m > best ? m : best;
    }
    if (live && best > c) {
      sc.color[v] = best;
      hits++;
    }
  }
  if (hits) atomicAdd(sc.flag, hits);
}

// mark: an unassigned, unmarked v joins when a successor of its colour has
__global__ __launch_bounds__(BLOCK) void k_scc_mark(DevGame g, SccBuf sc) {
  const uint32_t n = (uint32_t)g.n, lane = lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t hits = 0;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane; v0 < n; v0 += stride) {
    const uint32_t v = v0 + lane;
    const bool live = v < n && sc.comp[v] < 0 && !sc.mark[v];
    uint32_t ob = 0, oe = 0;
    int32_t c = -1;
    if (live) {
      ob = out_begin(g, v);
      oe = out_end(g, v);
      c = sc.color[v];
    }
    auto joins = [&](uint32_t k, int32_t col) {
      const int32_t u = g.edges[k].x;
      return sc.mark[u] != 0 && sc.comp[u] < 0 && sc.color[u] == col;
    };
    bool hit = false;
    if (live && oe - ob <= SCC_SHORT)
      for (uint32_t k = ob; k < oe && !hit; k++) hit = joins(k, c);
    unsigned long long longs = __ballot(live && oe - ob > SCC_SHORT);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(ob, (int)src, WAVE), e = __shfl(oe, (int)src, WAVE);
      const int32_t col = __shfl(c, (int)src, WAVE);
      const bool any = wave_any(b, e, [&](uint32_t k) { return joins(k, col); });
      if (lane == src) hit = any;
    }
    if (hit) {
      sc.mark[v] = 1;
      hits++;
    }
  }
  if (hits) atomicAdd(sc.flag, hits);
}

// Block-wide max of one value per thread (every thread gets it).
__device__ __forceinline__ int32_t block_max(int32_t x, int32_t* wred) {
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t y = __shfl_xor(x, o, WAVE);
    x = y > x ? y : x;
  }
  if (lane == 0) wred[wid] = x;
  block_sync();
  int32_t m = wred[0];
  for (uint32_t w = 1; w < BLOCK / WAVE; w++) m = wred[w] > m ? wred[w] : m;
  block_sync();  // wred may be rewritten by the next call
  return m;
}

// the vertices whose rows the block kernels below take (once per game)
__global__ __launch_bounds__(BLOCK) void k_scc_long_lists(DevGame g, SccBuf sc) {
  const uint32_t n = (uint32_t)g.n;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane_id(); v0 < n; v0 += gridDim.x * blockDim.x) {
    const uint32_t v = v0 + lane_id();
    const bool in = v < n;
    const bool li = in && g.rev_off[v + 1] - g.rev_off[v] > SCC_LONG;
    const bool lo = in && out_end(g, v) - out_begin(g, v) > SCC_LONG;
    unsigned long long m = __ballot(li);
    if (m) {
      const uint32_t leader = __ffsll((long long)m) - 1;
      uint32_t base = 0;
      if (lane_id() == leader) base = atomicAdd(&sc.nlong[0], (uint32_t)__popcll(m));
      base = __shfl(base, (int)leader, WAVE);
      if (li) sc.long_in[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (int32_t)v;
    }
    m = __ballot(lo);
    if (m) {
      const uint32_t leader = __ffsll((long long)m) - 1;
      uint32_t base = 0;
      if (lane_id() == leader) base = atomicAdd(&sc.nlong[1], (uint32_t)__popcll(m));
      base = __shfl(base, (int)leader, WAVE);
      if (lo) sc.long_out[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (int32_t)v;
    }
  }
}

// colour of the long predecessor lists: one block per listed vertex
__global__ __launch_bounds__(BLOCK) void k_scc_color_long(DevGame g, SccBuf sc) {
  __shared__ int32_t wred[BLOCK / WAVE];
  const uint32_t cnt = sc.nlong[0];
  uint32_t hits = 0;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int32_t v = sc.long_in[i];
    if (sc.comp[v] >= 0) continue;  // block-uniform
    int32_t best = -1;
    for (uint32_t k = g.rev_off[v] + threadIdx.x; k < g.rev_off[v + 1]; k += BLOCK) {
      const int32_t p = g.rev_src[k];
      const int32_t x = sc.comp[p] < 0 ? sc.color[p] : -1;
      best = x > best ? x : best;
    }
    best = block_max(best, wred);
    if (threadIdx.x == 0 && best > sc.color[v]) {
      sc.color[v] = best;
      hits++;
    }
  }
  if (hits) atomicAdd(sc.flag, hits);
}

// level of the long out-rows: one block per listed vertex
__global__ __launch_bounds__(BLOCK) void k_scc_level_long(DevGame g, SccBuf sc) {
  __shared__ int32_t wred[BLOCK / WAVE];
  const uint32_t cnt = sc.nlong[1];
  uint32_t hits = 0;
  int32_t top = 0;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int32_t v = sc.long_out[i];
    const int32_t cv = sc.comp[v];
    int32_t best = 0;
    for (uint32_t k = out_begin(g, v) + threadIdx.x; k < out_end(g, v); k += BLOCK) {
      const int32_t u = g.edges[k].x;
      const int32_t x = sc.lev[u] + (sc.comp[u] != cv ? 1 : 0);
      best = x > best ? x : best;
    }
    best = block_max(best, wred);
    if (threadIdx.x == 0 && best > sc.lev[v]) {
      sc.lev[v] = best;
      hits++;
    }
    top = best > top ? best : top;
  }
  if (hits) atomicAdd(sc.flag, hits);
  if (threadIdx.x == 0 && top) atomicMax(sc.max_level, top);
}

// start of a colour phase: every unassigned vertex takes its own id
__global__ void k_scc_color_init(int32_t n, SccBuf sc) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x)
    if (sc.comp[v] < 0) sc.color[v] = (int32_t)v;
}

// after the colouring: the roots are marked
__global__ void k_scc_roots(int32_t n, SccBuf sc) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x)
    sc.mark[v] = sc.comp[v] < 0 && sc.color[v] == (int32_t)v ? 1 : 0;
}

// after the marking: marked vertices join their root's component; flag counts
// the vertices still unassigned
__global__ void k_scc_assign(int32_t n, SccBuf sc) {
  uint32_t left = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x) {
    if (sc.comp[v] >= 0) continue;
    if (sc.mark[v]) {
      sc.comp[v] = sc.color[v];
      sc.mark[v] = 0;
    } else {
      left++;
    }
  }
  if (left) atomicAdd(sc.flag, left);
}

// level: lev[v] = max over successors u of lev[u] (+1 when u is in another
// component), iterated to the least fixpoint (the condensation is acyclic)
__global__ __launch_bounds__(BLOCK) void k_scc_level(DevGame g, SccBuf sc) {
  const uint32_t n = (uint32_t)g.n, lane = lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t hits = 0;
  int32_t top = 0;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane; v0 < n; v0 += stride) {
    const uint32_t v = v0 + lane;
    const bool in = v < n;
    uint32_t ob = 0, oe = 0;
    int32_t cv = 0, l = 0;
    if (in) {
      ob = out_begin(g, v);
      oe = out_end(g, v);
      cv = sc.comp[v];
      l = sc.lev[v];
    }
    auto val = [&](uint32_t k, int32_t comp) {
      const int32_t u = g.edges[k].x;
      return sc.lev[u] + (sc.comp[u] != comp ? 1 : 0);
    };
    int32_t best = l;
    if (in && oe - ob <= SCC_SHORT)
      for (uint32_t k = ob; k < oe; k++) {
        const int32_t x = val(k, cv);
        best = x > best ? x : best;
      }
    unsigned long long longs = __ballot(in && oe - ob > SCC_SHORT && oe - ob <= SCC_LONG);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(ob, (int)src, WAVE), e = __shfl(oe, (int)src, WAVE);
      const int32_t comp = __shfl(cv, (int)src, WAVE);
      const int32_t m = wave_max(b, e, 0, [&](uint32_t k) { return val(k, comp); });
      if (lane == src) best = m > best ? m : best;
    }
    if (in && best > l) {
      sc.lev[v] = best;
      hits++;
    }
    top = best > top ? best : top;
  }
  if (hits) atomicAdd(sc.flag, hits);
  if (top) atomicMax(sc.max_level, top);
}

__global__ void k_scc_reset(int32_t n, SccBuf sc) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x) {
    sc.comp[v] = -1;
    sc.lev[v] = 0;
    sc.mark[v] = 0;
  }
}

// count of components: vertices that are their component's label
__global__ void k_scc_count(int32_t n, SccBuf sc) {
  uint32_t c = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x)
    c += sc.comp[v] == (int32_t)v;
  if (c) atomicAdd(sc.flag, c);
}

// L_r of level `level`: the flags (round parity r) of its vertices, the
// per-block counts and the round r-1 "raised" word that lets round r run
__global__ __launch_bounds__(BLOCK) void k_level_activate(DevGame g, const int32_t* lev, int32_t level, uint32_t r) {
  __shared__ uint32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  block_sync();
  uint8_t* act = (r & 1) ? g.act1 : g.act0;
  uint32_t mine = 0;
  for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * BLOCK) {
    const bool a = lev[v] == level;
    act[v] = a ? 1 : 0;
    mine += a;
  }
  atomicAdd(&s_cnt, mine);
  block_sync();
  if (threadIdx.x == 0) {
    g.blk_chg[blockIdx.x] = s_cnt;
    if (s_cnt) g.ctrl[C_ANY0 + (r - 1) % 3] = 1;
  }
}

__global__ void k_scc_output(DevGame g, SccBuf sc, int32_t* comp_out, int32_t* lev_out) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const uint32_t i = g.perm ? (uint32_t)g.perm[v] : v;
    comp_out[v] = sc.comp[i];
    lev_out[v] = sc.lev[i];
  }
}

int grid_for(int32_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n + BLOCK - 1) / BLOCK, 8192)); }

// Runs `launch` in batches of up to 16 sweeps until a batch changes nothing;
// the flag word is cleared before each batch.  Every sweep family here is
// monotone and reaches its fixpoint within n + 1 changing sweeps; more than
// `cap` sweeps means a broken invariant and returns an error.
template <typename F>
hipError_t until_stable(const SccBuf& sc, uint32_t* h_flag, hipStream_t s, F launch, uint64_t* sweeps, uint64_t cap) {
  uint64_t done = 0;
  for (uint32_t batch = 1;; batch = batch < 16 ? batch * 2 : 16) {
    if (done > cap) return hipErrorUnknown;
    done += batch;
    hipError_t e = hipMemsetAsync(sc.flag, 0, 4, s);
    if (e != hipSuccess) return e;
    for (uint32_t i = 0; i < batch; i++) {
      launch();
      (*sweeps)++;
    }
    if ((e = hipMemcpyAsync(h_flag, sc.flag, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (*h_flag == 0) return hipGetLastError();
  }
}
}  // namespace

size_t scc_bytes(int32_t n) {
  const size_t nn = (size_t)n;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return 5 * up(4 * nn) + up(nn) + up(16);
}

void bind_scc(SccBuf& sc, void* base, int32_t n) {
  const size_t nn = (size_t)n;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* b = (char*)base;
  sc.comp = (int32_t*)b;
  b += up(4 * nn);
  sc.lev = (int32_t*)b;
  b += up(4 * nn);
  sc.color = (int32_t*)b;
  b += up(4 * nn);
  sc.mark = (uint8_t*)b;
  b += up(nn);
  sc.flag = (uint32_t*)b;
  sc.max_level = (int32_t*)(b + 4);
  sc.nlong = (uint32_t*)(b + 8);
  b += up(16);
  sc.long_in = (int32_t*)b;
  b += up(4 * nn);
  sc.long_out = (int32_t*)b;
}

hipError_t compute_scc(const DevGame& g, const SccBuf& sc, uint32_t* h_word, hipStream_t s, SccInfo* info) {
  const int32_t n = g.n;
  const int grid = grid_for(n);
  hipError_t e;
  uint64_t sweeps = 0, phases = 0;
  const uint64_t cap = 2 * (uint64_t)n + 64;
  hipLaunchKernelGGL(k_scc_reset, dim3(grid), dim3(BLOCK), 0, s, n, sc);
  if ((e = hipMemsetAsync(sc.nlong, 0, 8, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scc_long_lists, dim3(grid), dim3(BLOCK), 0, s, g, sc);
  for (;;) {
    if (phases > (uint64_t)n) return hipErrorUnknown;  // each phase assigns a component
    e = until_stable(sc, h_word, s, [&] { hipLaunchKernelGGL(k_scc_trim, dim3(grid), dim3(BLOCK), 0, s, g, sc); },
                     &sweeps, cap);
    if (e != hipSuccess) return e;
    // anything left?
    if ((e = hipMemsetAsync(sc.flag, 0, 4, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scc_assign, dim3(grid), dim3(BLOCK), 0, s, n, sc);  // marks are all clear here
    if ((e = hipMemcpyAsync(h_word, sc.flag, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (*h_word == 0) break;
    phases++;
    hipLaunchKernelGGL(k_scc_color_init, dim3(grid), dim3(BLOCK), 0, s, n, sc);
    e = until_stable(sc, h_word, s,
                     [&] {
                       hipLaunchKernelGGL(k_scc_color, dim3(grid), dim3(BLOCK), 0, s, g, sc);
                       hipLaunchKernelGGL(k_scc_color_long, dim3(SCC_LONG_GRID), dim3(BLOCK), 0, s, g, sc);
                     },
                     &sweeps, cap);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scc_roots, dim3(grid), dim3(BLOCK), 0, s, n, sc);
    e = until_stable(sc, h_word, s, [&] { hipLaunchKernelGGL(k_scc_mark, dim3(grid), dim3(BLOCK), 0, s, g, sc); },
                     &sweeps, cap);
    if (e != hipSuccess) return e;
    if ((e = hipMemsetAsync(sc.flag, 0, 4, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scc_assign, dim3(grid), dim3(BLOCK), 0, s, n, sc);
  }
  if ((e = hipMemsetAsync(sc.max_level, 0, 4, s)) != hipSuccess) return e;
  e = until_stable(sc, h_word, s,
                   [&] {
                     hipLaunchKernelGGL(k_scc_level, dim3(grid), dim3(BLOCK), 0, s, g, sc);
                     hipLaunchKernelGGL(k_scc_level_long, dim3(SCC_LONG_GRID), dim3(BLOCK), 0, s, g, sc);
                   },
                   &sweeps, cap);
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(sc.flag, 0, 4, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scc_count, dim3(grid), dim3(BLOCK), 0, s, n, sc);
  if ((e = hipMemcpyAsync(h_word, sc.flag, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;  // flag, max_level
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  info->components = h_word[0];
  info->levels = (uint32_t)((int32_t)h_word[1] + 1);
  info->sweeps = sweeps;
  info->phases = phases;
  return hipGetLastError();
}

hipError_t launch_scc_output(const DevGame& g, const SccBuf& sc, int32_t* comp_out, int32_t* lev_out, hipStream_t s) {
  hipLaunchKernelGGL(k_scc_output, dim3(grid_for(g.n)), dim3(BLOCK), 0, s, g, sc, comp_out, lev_out);
  return hipGetLastError();
}

hipError_t launch_level_activate(const DevGame& g, const int32_t* lev, int32_t level, uint32_t r, int grid,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_level_activate, dim3(grid), dim3(BLOCK), 0, s, g, lev, level, r);
  return hipGetLastError();
}

}  // namespace eg
