// Device kernels of libeg for gfx950 (wave64).
//
// Layout:   rs[v] = row start of v | owner bit,  edges[e] = {target, weight}
// Reverse:  rev_off / rev_src = predecessor lists, one entry per edge (the
//           paper's redundant CSC of Sec. 5), built by histogram + scan + scatter.
// Solve:    f values of width V (int32 when TOP + W < 2^31, else int64);
//           stored weights are at most P = min(max weight, B + 1) and TOP is
//           encoded as B + P + 1, so for any edge f(u) - w(v,u) > B exactly
//           when f(u) is TOP or the finite term leaves C_G.
#include <limits>

#include "eg_internal.h"

namespace eg {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of mask in lanes below this one
__device__ __forceinline__ uint32_t mbcnt(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Append `item` for every active lane with want = true: one atomic per wave.
__device__ __forceinline__ void wave_append(bool want, int32_t item, int32_t* out, uint32_t* count) {
  unsigned long long m = __ballot(want);
  if (m == 0) return;
  const uint32_t leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, leader, WAVE);
  if (want) out[base + mbcnt(m)] = item;
}

// ---------------------------------------------------------------- layout
__global__ void k_layout_rows(const int64_t* off, const uint8_t* owner_bits, int32_t n, uint32_t m,
                              uint32_t* rs) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (v == n) {
      rs[n] = m;
    } else {
      const uint32_t own = (owner_bits[v >> 3] >> (v & 7)) & 1u;
      rs[v] = (uint32_t)off[v] | (own << 31);
    }
  }
}

// Weights above `wclamp` (>= the bound + 1 or the largest weight) are stored as
// wclamp: for a finite f(u) <= B both give the term 0.
__global__ void k_layout_edges(const int32_t* tgt, const int32_t* w, uint32_t m, int32_t wclamp,
                               int2* edges) {
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x)
    edges[e] = make_int2(tgt[e], min(w[e], wclamp));
}

hipError_t launch_layout(const int64_t* off, const uint8_t* owner_bits, const int32_t* tgt,
                         const int32_t* w, int32_t n, uint32_t m, int32_t wclamp, uint32_t* rs,
                         int2* edges, hipStream_t s) {
  const int grid_v = (int)std::min<int64_t>(((int64_t)n + BLOCK) / BLOCK, 8192);
  hipLaunchKernelGGL(k_layout_rows, dim3(grid_v), dim3(BLOCK), 0, s, off, owner_bits, n, m, rs);
  if (m > 0) {
    const int grid_e = (int)std::min<int64_t>(((int64_t)m + BLOCK - 1) / BLOCK, 16384);
    hipLaunchKernelGGL(k_layout_edges, dim3(grid_e), dim3(BLOCK), 0, s, tgt, w, m, wclamp, edges);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- scan
constexpr int SCAN_BLOCK = 1024;

__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t x) {
  __shared__ uint32_t wsum[SCAN_BLOCK / WAVE];
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    uint32_t y = __shfl_up(x, o, WAVE);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == WAVE - 1) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t t = lane < SCAN_BLOCK / WAVE ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < SCAN_BLOCK / WAVE; o <<= 1) {
      uint32_t y = __shfl_up(t, o, WAVE);
      if (lane >= (uint32_t)o) t += y;
    }
    if (lane < SCAN_BLOCK / WAVE) wsum[lane] = t;
  }
  __syncthreads();
  return x + (wid > 0 ? wsum[wid - 1] : 0u);
}

// exclusive scan of each SCAN_BLOCK tile; tile totals to sums[]
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const uint32_t* in, uint32_t* out,
                                                           uint32_t* sums, size_t count) {
  const size_t i = (size_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  const uint32_t x = i < count ? in[i] : 0u;
  const uint32_t incl = block_inclusive_scan(x);
  if (i < count) out[i] = incl - x;
  if (threadIdx.x == SCAN_BLOCK - 1) sums[blockIdx.x] = incl;
}

__global__ void k_scan_add(uint32_t* out, const uint32_t* sums, size_t count) {
  const size_t i = (size_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  if (i < count) out[i] += sums[blockIdx.x];
}

size_t scan_tmp_words(size_t count) {
  size_t words = 0;
  while (count > 1) {
    count = (count + SCAN_BLOCK - 1) / SCAN_BLOCK;
    words += count + 1;
  }
  return words + 1;
}

// in-place-capable exclusive scan of `count` words (recursive over tile sums)
static hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, size_t count, uint32_t* tmp,
                                 hipStream_t s) {
  const size_t tiles = (count + SCAN_BLOCK - 1) / SCAN_BLOCK;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, out, tmp,
                     count);
  if (tiles > 1) {
    hipError_t e = exclusive_scan(tmp, tmp, tiles, tmp + tiles + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, out, tmp, count);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- reverse CSR
__global__ void k_indegree(const int2* edges, uint32_t m, uint32_t* deg) {
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x)
    atomicAdd(&deg[edges[e].x], 1u);
}

// source vertex of edge e: the v with rs[v] <= e < rs[v+1] (row starts masked)
__device__ __forceinline__ int32_t source_of(const uint32_t* rs, int32_t n, uint32_t e) {
  int32_t lo = 0, hi = n;  // invariant: start(lo) <= e < start(hi)
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((rs[mid] & ROW_MASK) <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Each thread walks edges e = first, first + stride, ...; its source index only
// moves forward, so after one binary search it advances by scanning.
__global__ void k_scatter_preds(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                                uint32_t* cursor, int32_t* rev_src) {
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t v = source_of(rs, n, e);
  for (; e < m; e += stride) {
    while ((rs[v + 1] & ROW_MASK) <= e) v++;
    const uint32_t slot = atomicAdd(&cursor[edges[e].x], 1u);
    rev_src[slot] = v;
  }
}

hipError_t launch_reverse_csr(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                              uint32_t* rev_off, int32_t* rev_src, uint32_t* cursor,
                              uint32_t* scan_tmp, size_t scan_tmp_words_avail, hipStream_t s) {
  if (scan_tmp_words_avail < scan_tmp_words((size_t)n + 1)) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(cursor, 0, sizeof(uint32_t) * ((size_t)n + 1), s);
  if (e != hipSuccess) return e;
  const int grid_e = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)m + BLOCK - 1) / BLOCK, 16384));
  if (m > 0) hipLaunchKernelGGL(k_indegree, dim3(grid_e), dim3(BLOCK), 0, s, edges, m, cursor);
  e = exclusive_scan(cursor, rev_off, (size_t)n + 1, scan_tmp, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(cursor, rev_off, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if (m > 0)
    hipLaunchKernelGGL(k_scatter_preds, dim3(grid_e), dim3(BLOCK), 0, s, rs, edges, n, m, cursor,
                       rev_src);
  return hipGetLastError();
}

// ---------------------------------------------------------------- solve
// Initial active set of Alg. 3 (and Alg. 1): player-0 vertices whose out-edges
// all have negative weight, player-1 vertices with some negative out-edge.
// Equivalently, the vertices whose lift from f = 0 is positive.  With resume,
// f is kept and every vertex is active.
template <int H, typename V>
__global__ __launch_bounds__(BLOCK) void k_init(DevGame g, int resume) {
  V* f = (V*)g.f;
  const uint32_t sub = threadIdx.x & (H - 1);
  const uint32_t group = (blockIdx.x * blockDim.x + threadIdx.x) / H;
  const uint32_t ngroups = gridDim.x * blockDim.x / H;
  uint32_t* count = &g.ctrl[C_CNT0 + 1];
  for (uint32_t v = group; v < (uint32_t)g.n; v += ngroups) {
    bool active = true;
    if (!resume) {
      const uint32_t a = g.rs[v], b = g.rs[v + 1];
      const bool p1 = (a & OWNER_BIT) != 0;
      int any_neg = 0, all_neg = 1;
      for (uint32_t e = (a & ROW_MASK) + sub; e < (b & ROW_MASK); e += H) {
        const int neg = g.edges[e].y < 0;
        any_neg |= neg;
        all_neg &= neg;
      }
#pragma unroll
      for (int o = H / 2; o > 0; o >>= 1) {
        any_neg |= __shfl_xor(any_neg, o, H);
        all_neg &= __shfl_xor(all_neg, o, H);
      }
      active = p1 ? any_neg != 0 : all_neg != 0;
    }
    if (sub == 0) {
      if (!resume) f[v] = 0;
      g.stamp[v] = active ? 1u : 0u;
    }
    wave_append(sub == 0 && active, (int32_t)v, g.wl1, count);
  }
}

// One round of Alg. 3 over the active list of round r, fused: each group of H
// lanes lifts one vertex v (Def. 6) from a coalesced read of its out-edges and
// a gather of f at the targets, combines the lanes by shuffles, stores f(v) in
// place if it rose, and then scans pre(v) to activate every predecessor for
// round r+1 exactly once (stamp test-and-set, wave-aggregated append).
template <int H, typename V>
__global__ __launch_bounds__(BLOCK) void k_round(DevGame g, uint32_t r) {
  __shared__ unsigned long long s_stats[S_WORDS];
  if (threadIdx.x < S_WORDS) s_stats[threadIdx.x] = 0;
  const uint32_t n_in = g.ctrl[C_CNT0 + r % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g.ctrl[C_CNT0 + (r + 2) % 3] = 0;  // the list of round r-1, recycled for round r+2
    if (n_in) g.ctrl[C_ROUNDS] += 1;
  }
  __syncthreads();
  if (n_in == 0) return;

  V* f = (V*)g.f;
  const int32_t* wl_in = (r & 1) ? g.wl1 : g.wl0;
  int32_t* wl_out = (r & 1) ? g.wl0 : g.wl1;
  uint32_t* cnt_out = &g.ctrl[C_CNT0 + (r + 1) % 3];
  const uint32_t next = r + 1;
  const V bound = (V)g.bound, top = (V)g.top;

  const uint32_t sub = threadIdx.x & (H - 1);
  const uint32_t leader = lane_id() & ~(uint32_t)(H - 1);
  const uint32_t group = (blockIdx.x * blockDim.x + threadIdx.x) / H;
  const uint32_t ngroups = gridDim.x * blockDim.x / H;
  unsigned long long lifts = 0, edges_read = 0, changes = 0, pushes = 0;

  for (uint32_t i = group; i < n_in; i += ngroups) {
    const int32_t v = wl_in[i];
    const uint32_t a = g.rs[v], b = g.rs[v + 1];
    const uint32_t beg = a & ROW_MASK, end = b & ROW_MASK;
    const bool p1 = (a & OWNER_BIT) != 0;
    V acc = p1 ? V(0) : std::numeric_limits<V>::max();
    for (uint32_t e = beg + sub; e < end; e += H) {
      const int2 ed = g.edges[e];
      V t = f[ed.x] - (V)ed.y;
      t = t > V(0) ? t : V(0);
      acc = p1 ? (t > acc ? t : acc) : (t < acc ? t : acc);
    }
#pragma unroll
    for (int o = H / 2; o > 0; o >>= 1) {
      const V other = __shfl_xor(acc, o, H);
      acc = p1 ? (other > acc ? other : acc) : (other < acc ? other : acc);
    }
    if (acc > bound) acc = top;
    int changed = 0;
    if (sub == 0) {
      const V old = f[v];
      lifts++;
      edges_read += end - beg;
      if (acc != old) {
        f[v] = acc;
        changed = 1;
        changes++;
      }
    }
    changed = __shfl(changed, leader, WAVE);
    if (changed) {
      const uint32_t pb = g.rev_off[v], pe = g.rev_off[v + 1];
      for (uint32_t k = pb + sub; k < pe; k += H) {
        const int32_t p = g.rev_src[k];
        bool want = false;
        if (g.stamp[p] != next) want = atomicExch(&g.stamp[p], next) != next;
        pushes += want;
        wave_append(want, p, wl_out, cnt_out);
      }
    }
  }
  atomicAdd(&s_stats[S_LIFTS], lifts);
  atomicAdd(&s_stats[S_EDGES], edges_read);
  atomicAdd(&s_stats[S_CHANGES], changes);
  atomicAdd(&s_stats[S_PUSHES], pushes);
  __syncthreads();
  if (threadIdx.x < S_WORDS && s_stats[threadIdx.x]) atomicAdd(&g.stats[threadIdx.x], s_stats[threadIdx.x]);
}

template <typename V>
__global__ void k_output(DevGame g, int64_t* out) {
  const V* f = (const V*)g.f;
  const V top = (V)g.top;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const V x = f[v];
    out[v] = x == top ? INT64_MAX : (int64_t)x;
  }
}

template <typename V>
__global__ void k_input(DevGame g, const int64_t* in) {
  V* f = (V*)g.f;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const int64_t x = in[v];
    f[v] = x == INT64_MAX ? (V)g.top : (V)x;
  }
}

int pick_h(double avg_deg) {
  int h = 1;
  while (h < 64 && h < avg_deg) h <<= 1;
  return h;
}

int round_grid(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    cus = 256;
  return cus * 8;
}

template <typename V>
static hipError_t init_v(const DevGame& g, int h, int resume, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n * h + BLOCK - 1) / BLOCK, 16384));
  switch (h) {
#define EG_CASE(H) \
  case H: hipLaunchKernelGGL((k_init<H, V>), dim3(grid), dim3(BLOCK), 0, s, g, resume); break;
    EG_CASE(1) EG_CASE(2) EG_CASE(4) EG_CASE(8) EG_CASE(16) EG_CASE(32) EG_CASE(64)
#undef EG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename V>
static hipError_t round_v(const DevGame& g, int h, uint32_t r, int grid, hipStream_t s) {
  switch (h) {
#define EG_CASE(H) \
  case H: hipLaunchKernelGGL((k_round<H, V>), dim3(grid), dim3(BLOCK), 0, s, g, r); break;
    EG_CASE(1) EG_CASE(2) EG_CASE(4) EG_CASE(8) EG_CASE(16) EG_CASE(32) EG_CASE(64)
#undef EG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(const DevGame& g, int vbits, int h, int resume, hipStream_t s) {
  return vbits == 32 ? init_v<int32_t>(g, h, resume, s) : init_v<int64_t>(g, h, resume, s);
}

hipError_t launch_round(const DevGame& g, int vbits, int h, uint32_t r, int grid, hipStream_t s) {
  return vbits == 32 ? round_v<int32_t>(g, h, r, grid, s) : round_v<int64_t>(g, h, r, grid, s);
}

hipError_t launch_output(const DevGame& g, int vbits, int64_t* out, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + BLOCK - 1) / BLOCK, 8192));
  if (vbits == 32) hipLaunchKernelGGL(k_output<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, out);
  else hipLaunchKernelGGL(k_output<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, out);
  return hipGetLastError();
}

hipError_t launch_input(const DevGame& g, int vbits, const int64_t* in, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + BLOCK - 1) / BLOCK, 8192));
  if (vbits == 32) hipLaunchKernelGGL(k_input<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, in);
  else hipLaunchKernelGGL(k_input<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, in);
  return hipGetLastError();
}

}  // namespace eg
