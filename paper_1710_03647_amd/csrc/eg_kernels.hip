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

// Block barrier that first waits until this wave's LDS operations, atomics
// included, have completed (s_waitcnt lgkmcnt(0)).  The workgroup fence of
// __syncthreads() may leave that wait out, and then an LDS atomic issued
// before the barrier can land after another wave's read that follows it.
__device__ __forceinline__ void block_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt = 0; vmcnt, expcnt unconstrained
  __syncthreads();
}

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
  block_sync();
  if (wid == 0) {
    uint32_t t = lane < SCAN_BLOCK / WAVE ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < SCAN_BLOCK / WAVE; o <<= 1) {
      uint32_t y = __shfl_up(t, o, WAVE);
      if (lane >= (uint32_t)o) t += y;
    }
    if (lane < SCAN_BLOCK / WAVE) wsum[lane] = t;
  }
  block_sync();
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
//
// The predecessor lists (one entry per edge, grouped by target) are built by
// two partition passes, so that no counter is shared by the many edges of a
// hub (in-degrees of power-law games reach 10^5 and more), and every write
// lands in a short run of consecutive words:
//  1. by bucket of targets (2^shift consecutive targets, at most RB_BUCKETS
//     buckets): each block counts the buckets of its chunk of edges in LDS and
//     adds the non-zero counts to the bucket totals; after a scan of the totals
//     it counts again, reserves one range per non-empty bucket with one atomic
//     and writes its entries {source, target} (and weight) there;
//  2. by target, over the bucketed entries cut into pieces of RP_PIECE: each
//     piece counts the targets of an LDS window (RP_WIN targets from the base
//     of its first entry's bucket) and adds the non-zero counts to the
//     in-degrees; after the scan of the in-degrees (rev_off) it reserves one
//     range per non-empty target and writes the sources.  The entries of a
//     piece come from a few consecutive buckets, so the window holds nearly
//     all of them; an entry outside it takes a global atomic of its own.
// The order inside a predecessor list is not fixed (it does not matter).

constexpr uint32_t RB_MIN_SHIFT = 10;   // at least 1024 targets per bucket
constexpr uint32_t RB_CHUNK = 32768;    // edges per block in pass 1
constexpr uint32_t RB_SUB = 4096;       // edges whose sources one block step resolves
constexpr uint32_t RP_PIECE = 8192;     // bucketed entries per piece in pass 2
constexpr uint32_t RP_WIN = 4096;       // targets counted in LDS per piece
constexpr uint32_t RP_BIG = 32768;      // buckets with more entries are written piece by piece

// A bucket written piece by piece (k_rp_scatter) rather than by one block
// (k_rp_bucket): more than RP_BIG entries, or more targets than LDS holds.
__device__ __forceinline__ bool rp_big(const uint32_t* bstart, uint32_t b, uint32_t shift) {
  return (1u << shift) > RP_WIN || bstart[b + 1] - bstart[b] > RP_BIG;
}

uint32_t rb_shift(int32_t n) {
  uint32_t bits = 0;
  while (bits < 31 && (1u << bits) < (uint32_t)n) bits++;
  return bits > 12 + RB_MIN_SHIFT ? bits - 12 : RB_MIN_SHIFT;
}

// Bucket totals of pass 1.
__global__ __launch_bounds__(BLOCK) void k_rb_count(const int2* edges, uint32_t m, uint32_t shift, uint32_t* bcnt) {
  __shared__ uint32_t hist[RB_BUCKETS];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < RB_BUCKETS; i += BLOCK) hist[i] = 0;
  block_sync();
  const uint32_t e0 = blockIdx.x * RB_CHUNK, e1 = min(m, e0 + RB_CHUNK);
#pragma unroll 8
  for (uint32_t e = e0 + tid; e < e1; e += BLOCK) atomicAdd(&hist[(uint32_t)edges[e].x >> shift], 1u);
  block_sync();
  for (uint32_t i = tid; i < RB_BUCKETS; i += BLOCK)
    if (hist[i]) atomicAdd(&bcnt[i], hist[i]);
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

// source of edge sub + x for x < len, into srcl: the row ids of the row starts
// inside (sub, sub + len) are written at their positions, the row holding
// edge sub at position 0, and an inclusive max-scan spreads each row id over
// its edges (row starts rise with the row id, every row has an edge).
__device__ __forceinline__ void chunk_sources(const uint32_t* rs, int32_t n, uint32_t sub, uint32_t len,
                                              uint32_t* srcl, uint32_t* wmax, uint32_t* s_va, uint32_t* s_more) {
  static_assert(RB_SUB % BLOCK == 0, "whole positions per thread");
  constexpr uint32_t PER = RB_SUB / BLOCK;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid / WAVE;
  if (tid == 0) *s_va = (uint32_t)source_of(rs, n, sub);
  for (uint32_t x = tid; x < RB_SUB; x += BLOCK) srcl[x] = 0;
  block_sync();
  const uint32_t va = *s_va, s1 = sub + len;
  for (uint32_t r0 = va + 1, it = 0;; r0 += BLOCK, it++) {
    const uint32_t r = r0 + tid;
    bool in = false;
    if (r < (uint32_t)n) {
      const uint32_t st = rs[r] & ROW_MASK;  // > sub: row va holds edge sub
      if (st < s1) {
        srcl[st - sub] = r;
        in = true;
      }
    }
    if (tid == BLOCK - 1) s_more[it & 1] = in;  // rows start in increasing order
    block_sync();
    if (!s_more[it & 1]) break;
  }
  if (tid == 0) srcl[0] = va;
  block_sync();
  uint32_t loc[PER];
  uint32_t run = 0;
#pragma unroll
  for (uint32_t j = 0; j < PER; j++) {
    const uint32_t y = srcl[tid * PER + j];
    run = y > run ? y : run;
    loc[j] = run;
  }
  uint32_t incl = run;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, WAVE);
    if (lane >= (uint32_t)o) incl = y > incl ? y : incl;
  }
  if (lane == WAVE - 1) wmax[wid] = incl;
  uint32_t excl = __shfl_up(incl, 1, WAVE);
  if (lane == 0) excl = 0;
  block_sync();
  for (uint32_t w = 0; w < wid; w++) excl = wmax[w] > excl ? wmax[w] : excl;
#pragma unroll
  for (uint32_t j = 0; j < PER; j++) srcl[tid * PER + j] = loc[j] > excl ? loc[j] : excl;
  block_sync();
}

// Pass 1: the block's chunk of edges into the ranges of their buckets.
__global__ __launch_bounds__(BLOCK) void k_rb_scatter(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                                                      uint32_t shift, uint32_t* bcur, int2* ent, int32_t* entw) {
  __shared__ uint32_t base[RB_BUCKETS];  // counts, then the first slot of the block's range per bucket
  __shared__ uint32_t lcur[RB_BUCKETS];
  __shared__ uint32_t srcl[RB_SUB];
  __shared__ uint32_t wmax[BLOCK / WAVE];
  __shared__ uint32_t s_va, s_more[2];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < RB_BUCKETS; i += BLOCK) {
    base[i] = 0;
    lcur[i] = 0;
  }
  block_sync();
  const uint32_t e0 = blockIdx.x * RB_CHUNK, e1 = min(m, e0 + RB_CHUNK);
#pragma unroll 8
  for (uint32_t e = e0 + tid; e < e1; e += BLOCK) atomicAdd(&base[(uint32_t)edges[e].x >> shift], 1u);
  block_sync();
  for (uint32_t i = tid; i < RB_BUCKETS; i += BLOCK)
    if (base[i]) base[i] = atomicAdd(&bcur[i], base[i]);
  block_sync();
  for (uint32_t sub = e0; sub < e1; sub += RB_SUB) {
    const uint32_t len = min(e1 - sub, RB_SUB);
    chunk_sources(rs, n, sub, len, srcl, wmax, &s_va, s_more);
    for (uint32_t x = tid; x < len; x += BLOCK) {
      const int2 ed = edges[sub + x];
      const uint32_t b = (uint32_t)ed.x >> shift;
      const uint32_t slot = base[b] + atomicAdd(&lcur[b], 1u);
      ent[slot] = make_int2((int32_t)srcl[x], ed.x);
      if (entw) entw[slot] = ed.y;
    }
    block_sync();  // srcl is rewritten by the next step
  }
}

// Pass 2, counting: in-degrees.
__global__ __launch_bounds__(BLOCK) void k_rp_count(const int2* ent, uint32_t m, uint32_t shift, uint32_t* deg) {
  __shared__ uint32_t hist[RP_WIN];
  const uint32_t tid = threadIdx.x;
  for (uint32_t p0 = blockIdx.x * RP_PIECE; p0 < m; p0 += gridDim.x * RP_PIECE) {
    const uint32_t p1 = min(m, p0 + RP_PIECE);
    block_sync();  // the previous piece is done with hist
    for (uint32_t i = tid; i < RP_WIN; i += BLOCK) hist[i] = 0;
    const uint32_t tmin = ((uint32_t)ent[p0].y >> shift) << shift;
    block_sync();
#pragma unroll 8
    for (uint32_t x = p0 + tid; x < p1; x += BLOCK) {
      const uint32_t t = (uint32_t)ent[x].y, d = t - tmin;
      if (d < RP_WIN) atomicAdd(&hist[d], 1u);
      else atomicAdd(&deg[t], 1u);
    }
    block_sync();
    for (uint32_t i = tid; i < RP_WIN; i += BLOCK)
      if (hist[i]) atomicAdd(&deg[tmin + i], hist[i]);
  }
}

// Pass 2, writing, buckets of at most RP_BIG entries: one block per bucket.
// The bucket's entries fill exactly the predecessor lists of its targets, one
// range of the reverse CSR, which the block writes while its lines are in L2.
__global__ __launch_bounds__(BLOCK) void k_rp_bucket(const int2* ent, const int32_t* entw, const uint32_t* bstart,
                                                     uint32_t nb, uint32_t shift, int32_t n, const uint32_t* rev_off,
                                                     int32_t* rev_src, int32_t* rev_w) {
  __shared__ uint32_t roff[RP_WIN];
  __shared__ uint32_t lcur[RP_WIN];
  const uint32_t tid = threadIdx.x;
  const uint32_t width = 1u << shift;
  for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint32_t x0 = bstart[b], x1 = bstart[b + 1];
    if (x1 == x0 || rp_big(bstart, b, shift)) continue;  // block-uniform
    const uint32_t t0 = b << shift;
    block_sync();  // the previous bucket is done with the LDS arrays
    for (uint32_t i = tid; i < width; i += BLOCK) {
      roff[i] = t0 + i < (uint32_t)n ? rev_off[t0 + i] : 0u;
      lcur[i] = 0;
    }
    block_sync();
    for (uint32_t x = x0 + tid; x < x1; x += BLOCK) {
      const int2 en = ent[x];
      const uint32_t d = (uint32_t)en.y - t0;
      const uint32_t slot = roff[d] + atomicAdd(&lcur[d], 1u);
      rev_src[slot] = en.x;
      if (rev_w) rev_w[slot] = entw[x];
    }
  }
}

// Pass 2, writing, the entries of the other buckets: each piece's sources into
// the ranges it reserves.
__global__ __launch_bounds__(BLOCK) void k_rp_scatter(const int2* ent, const int32_t* entw, uint32_t m,
                                                      uint32_t shift, const uint32_t* bstart, uint32_t* cursor,
                                                      int32_t* rev_src, int32_t* rev_w) {
  __shared__ uint32_t base[RP_WIN];
  __shared__ uint32_t lcur[RP_WIN];
  const uint32_t tid = threadIdx.x;
  for (uint32_t p0 = blockIdx.x * RP_PIECE; p0 < m; p0 += gridDim.x * RP_PIECE) {
    const uint32_t p1 = min(m, p0 + RP_PIECE);
    block_sync();
    for (uint32_t i = tid; i < RP_WIN; i += BLOCK) {
      base[i] = 0;
      lcur[i] = 0;
    }
    const uint32_t tmin = ((uint32_t)ent[p0].y >> shift) << shift;
    block_sync();
#pragma unroll 8
    for (uint32_t x = p0 + tid; x < p1; x += BLOCK) {
      const uint32_t t = (uint32_t)ent[x].y, d = t - tmin;
      if (d < RP_WIN && rp_big(bstart, t >> shift, shift)) atomicAdd(&base[d], 1u);
    }
    block_sync();
    for (uint32_t i = tid; i < RP_WIN; i += BLOCK)
      if (base[i]) base[i] = atomicAdd(&cursor[tmin + i], base[i]);
    block_sync();
    for (uint32_t x = p0 + tid; x < p1; x += BLOCK) {
      const int2 en = ent[x];
      const uint32_t t = (uint32_t)en.y, d = t - tmin;
      if (!rp_big(bstart, t >> shift, shift)) continue;  // written by k_rp_bucket
      const uint32_t slot = d < RP_WIN ? base[d] + atomicAdd(&lcur[d], 1u) : atomicAdd(&cursor[t], 1u);
      rev_src[slot] = en.x;
      if (rev_w) rev_w[slot] = entw[x];
    }
  }
}

// ---------------------------------------------------------------- target-partitioned edge copy
// For dense rounds of large games the gathers of f are confined per XCD: the
// vertex range is cut into `nparts` slices, and a second copy of the edges is
// grouped by (tile of PTILE source vertices, target slice).  Each record keeps
// its target and its tile-local source index (10 bits above the 22 target
// bits), so a chunk is reduced without knowing row boundaries.

__device__ __forceinline__ uint32_t chunk_of(uint32_t v, uint32_t tgt, uint32_t nparts, uint32_t part_size) {
  return (v / PTILE) * nparts + tgt / part_size;
}

// The copy is built like the buckets of the reverse CSR: each block takes
// PT_CHUNK consecutive edges (whose sources lie in at most PT_TILES tiles,
// since every vertex has an out-edge), counts its (tile, slice) chunks in LDS
// and adds the non-zero counts to the chunk totals; after a scan of the
// totals it counts again, reserves one range per non-empty chunk with one
// atomic and writes its records there.  The sources come from chunk_sources.
constexpr uint32_t PT_CHUNK = 4 * RB_SUB;              // edges per block
constexpr uint32_t PT_TILES = PT_CHUNK / PTILE + 2;    // tiles a block's edges can touch
constexpr uint32_t PT_KEYS = PT_TILES * 64;            // (tile, slice) counters, at most 64 slices

template <bool SCATTER>
__global__ __launch_bounds__(BLOCK) void k_part_edges(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                                                      uint32_t nparts, uint32_t part_size, uint32_t* cnt,
                                                      int2* pedges) {
  __shared__ uint32_t lcnt[PT_KEYS];  // counts, then the first slot of the block's range per chunk
  __shared__ uint32_t lcur[SCATTER ? PT_KEYS : 1];
  __shared__ uint32_t srcl[RB_SUB];
  __shared__ uint32_t wmax[BLOCK / WAVE];
  __shared__ uint32_t s_va, s_more[2], s_t0;
  const uint32_t tid = threadIdx.x;
  const uint32_t e0 = blockIdx.x * PT_CHUNK, e1 = min(m, e0 + PT_CHUNK);
  for (uint32_t i = tid; i < PT_KEYS; i += BLOCK) {
    lcnt[i] = 0;
    if (SCATTER) lcur[i] = 0;
  }
  // the tile of the block's first edge (every later edge is in it or after it)
  if (tid == 0) s_t0 = (uint32_t)source_of(rs, n, e0) / PTILE;
  block_sync();
  const uint32_t t0 = s_t0;
  for (int pass = 0; pass < (SCATTER ? 2 : 1); pass++) {
    for (uint32_t sub = e0; sub < e1; sub += RB_SUB) {
      const uint32_t len = min(e1 - sub, RB_SUB);
      chunk_sources(rs, n, sub, len, srcl, wmax, &s_va, s_more);
      for (uint32_t x = tid; x < len; x += BLOCK) {
        const int2 ed = edges[sub + x];
        const uint32_t src = srcl[x];
        const uint32_t key = (src / PTILE - t0) * nparts + (uint32_t)ed.x / part_size;
        if (pass == 0) {
          atomicAdd(&lcnt[key], 1u);
        } else {
          const uint32_t slot = lcnt[key] + atomicAdd(&lcur[key], 1u);
          pedges[slot] = make_int2((int32_t)((uint32_t)ed.x | ((src % PTILE) << PTILE_SHIFT)), ed.y);
        }
      }
      block_sync();  // srcl is rewritten by the next step
    }
    const uint32_t nkeys = PT_TILES * nparts;
    for (uint32_t k = tid; k < nkeys; k += BLOCK) {
      if (!lcnt[k]) continue;
      const uint32_t c = (t0 + k / nparts) * nparts + k % nparts;
      if (!SCATTER) atomicAdd(&cnt[c], lcnt[k]);
      else if (pass == 0) lcnt[k] = atomicAdd(&cnt[c], lcnt[k]);
    }
    block_sync();
  }
}

__global__ void k_owner_words(const uint32_t* rs, int32_t n, uint32_t* own) {
  const uint32_t words = ((uint32_t)n + 31) / 32;
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
    uint32_t x = 0;
    for (uint32_t i = 0; i < 32 && w * 32 + i < (uint32_t)n; i++) x |= (rs[w * 32 + i] >> 31) << i;
    own[w] = x;
  }
}

size_t partition_scratch_words(int32_t n, uint32_t nparts) {
  return (size_t)(((uint32_t)n + PTILE - 1) / PTILE) * nparts + 1;
}

hipError_t launch_partition(const DevGame& dg, const uint8_t*, uint32_t* cursor, uint32_t* scan_tmp,
                            size_t scan_words, hipStream_t s) {
  const uint32_t nchunks = (uint32_t)partition_scratch_words(dg.n, dg.nparts) - 1;
  // the chunk counters reuse the n + 1 words of the predecessor-list cursor
  if (nchunks > (uint32_t)dg.n || scan_words < scan_tmp_words((size_t)nchunks + 1)) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(cursor, 0, 4 * ((size_t)nchunks + 1), s);
  if (e != hipSuccess) return e;
  if (dg.nparts > 64) return hipErrorInvalidValue;
  const int grid_s = (int)std::max<uint64_t>(1, ((uint64_t)dg.m + PT_CHUNK - 1) / PT_CHUNK);
  hipLaunchKernelGGL(k_part_edges<false>, dim3(grid_s), dim3(BLOCK), 0, s, dg.rs, dg.edges, dg.n, dg.m, dg.nparts,
                     dg.part_size, cursor, (int2*)nullptr);
  e = exclusive_scan(cursor, (uint32_t*)dg.poff, (size_t)nchunks + 1, scan_tmp, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(cursor, dg.poff, 4 * (size_t)nchunks, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_edges<true>, dim3(grid_s), dim3(BLOCK), 0, s, dg.rs, dg.edges, dg.n, dg.m, dg.nparts,
                     dg.part_size, cursor, (int2*)dg.pedges);
  const int grid_w = (int)std::max<int64_t>(1, std::min<int64_t>((((int64_t)dg.n + 31) / 32 + BLOCK - 1) / BLOCK, 4096));
  hipLaunchKernelGGL(k_owner_words, dim3(grid_w), dim3(BLOCK), 0, s, dg.rs, dg.n, (uint32_t*)dg.own_bits);
  return hipGetLastError();
}

hipError_t launch_reverse_csr(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                              uint32_t* rev_off, int32_t* rev_src, int32_t* rev_w, uint32_t* cursor,
                              uint32_t* scan_tmp, size_t scan_tmp_words_avail, const RcsrScratch& rx,
                              hipStream_t s) {
  if (scan_tmp_words_avail < scan_tmp_words((size_t)n + 1)) return hipErrorInvalidValue;
  const uint32_t shift = rb_shift(n);
  const uint32_t nb = (((uint32_t)n - 1) >> shift) + 1;
  if (nb > RB_BUCKETS || (rev_w && !rx.entw)) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(cursor, 0, sizeof(uint32_t) * ((size_t)n + 1), s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    if ((e = hipMemsetAsync(rx.bcnt, 0, sizeof(uint32_t) * ((size_t)nb + 1), s)) != hipSuccess) return e;
    const uint32_t chunks = (m + RB_CHUNK - 1) / RB_CHUNK;
    hipLaunchKernelGGL(k_rb_count, dim3(chunks), dim3(BLOCK), 0, s, edges, m, shift, rx.bcnt);
    if ((e = exclusive_scan(rx.bcnt, rx.bcnt, (size_t)nb + 1, scan_tmp, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(rx.bcur, rx.bcnt, sizeof(uint32_t) * nb, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_rb_scatter, dim3(chunks), dim3(BLOCK), 0, s, rs, edges, n, m, shift, rx.bcur, rx.ent,
                       rev_w ? rx.entw : (int32_t*)nullptr);
    const int grid_p = (int)std::min<uint32_t>((m + RP_PIECE - 1) / RP_PIECE, 8192u);
    hipLaunchKernelGGL(k_rp_count, dim3(grid_p), dim3(BLOCK), 0, s, (const int2*)rx.ent, m, shift, cursor);
  }
  if ((e = exclusive_scan(cursor, rev_off, (size_t)n + 1, scan_tmp, s)) != hipSuccess) return e;
  if (m > 0) {
    if ((e = hipMemcpyAsync(cursor, rev_off, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s)) !=
        hipSuccess)
      return e;
    const int grid_p = (int)std::min<uint32_t>((m + RP_PIECE - 1) / RP_PIECE, 8192u);
    hipLaunchKernelGGL(k_rp_bucket, dim3(std::min<uint32_t>(nb, 4096u)), dim3(BLOCK), 0, s, (const int2*)rx.ent,
                       (const int32_t*)rx.entw, (const uint32_t*)rx.bcnt, nb, shift, n, (const uint32_t*)rev_off,
                       rev_src, rev_w);
    hipLaunchKernelGGL(k_rp_scatter, dim3(grid_p), dim3(BLOCK), 0, s, (const int2*)rx.ent,
                       (const int32_t*)rx.entw, m, shift, (const uint32_t*)rx.bcnt, cursor, rev_src, rev_w);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- solve
//
// Active sets.  Byte flags act[r & 1][v] != 0 mark v as a member of the active
// set L_r of round r (Alg. 3); round r clears the flags it consumes and sets
// flags in act[(r+1) & 1] for L_{r+1}, so the two sets never interfere.  A
// round runs in one of two representations:
//   sparse: L_r is also a list (wl[r & 1], length ctrl[C_CNT0 + r % 3]); a
//           predecessor p joins L_{r+1} through an atomic OR on the word that
//           holds its flag (the old value tells whether it was already in),
//           is staged in LDS, and one global atomic per block appends the
//           block's entries;
//   dense:  only the flags; each block sweeps tiles of V and a predecessor
//           joins L_{r+1} by a plain byte store (every writer stores the same
//           value, so no atomic is needed).
// The flag arrays are n bytes each, small enough to stay in L2.
//
// Per round each block writes its own counters (stats slots, changes), so no
// counter is shared between blocks except the list length of sparse rounds.

constexpr int TILE = TILE_VERTICES;  // list entries / vertices per tile
static_assert(TILE == BLOCK, "one tile entry per thread");
static_assert(BLOCK / WAVE == 4, "four waves per block (wbig)");
constexpr int UNROLL = 4;           // edges (or predecessor entries) per thread in flight (4: measured
                                    // 5% faster than 8 on uniform rounds, 4% on the R-MAT lift)
constexpr int PUSH_CAP = 2048;      // staged list entries per block (sparse rounds)

// Append `item` for the lanes with want = true to an LDS array: one LDS atomic per wave.
__device__ __forceinline__ void lds_append(bool want, int32_t item, int32_t* buf, uint32_t* count) {
  const unsigned long long m = __ballot(want);
  if (m == 0) return;
  const uint32_t leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, leader, WAVE);
  if (want) buf[base + mbcnt(m)] = item;
}

// Exclusive scan over the BLOCK threads; *total receives the sum.  Contains a
// barrier; wsum (BLOCK/WAVE words of LDS) may be reused after the next barrier.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* wsum, uint32_t* total) {
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, WAVE);
    if (lane >= (uint32_t)o) incl += y;
  }
  if (lane == WAVE - 1) wsum[wid] = incl;
  block_sync();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / WAVE; w++) {
    const uint32_t sw = wsum[w];
    off += (uint32_t)w < wid ? sw : 0u;
    tot += sw;
  }
  *total = tot;
  return off + incl - x;
}

// Largest i in [0, BLOCK) with pre[i] <= x, given pre[0] = 0 <= x < pre[BLOCK]:
// the thread whose (non-empty) range [pre[i], pre[i+1]) holds x.
__device__ __forceinline__ uint32_t find_range(const uint32_t* pre, uint32_t x) {
  uint32_t lo = 0, hi = BLOCK;
#pragma unroll
  for (int step = 0; step < 8; step++) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Terms of one chunk of UNROLL * BLOCK edges in the contiguous-row lift: the
// term of chunk position q sits at (q % UNROLL) * (BLOCK + 1) + q / UNROLL, so
// that the fold (thread t reads positions t * UNROLL + j) and the stream (lane
// i writes positions j * BLOCK + i) both touch consecutive words per lane
// group; the pad word per row staggers the banks of the groups.
constexpr int TERM_ROW = BLOCK + 1;
__device__ __forceinline__ uint32_t term_slot(uint32_t q) { return (q % UNROLL) * TERM_ROW + q / UNROLL; }

template <typename V>
struct RoundShared {
  uint32_t epre[BLOCK + 1];  // exclusive prefix of out-degrees of the tile's active vertices
  uint32_t ebeg[BLOCK];      // their row starts with the owner bit
  V key[BLOCK];              // running min of the per-edge keys (negated terms for player 1)
  uint32_t wsum[BLOCK / WAVE];
  uint32_t wbig[BLOCK / WAVE];  // per wave: some active vertex has more than LANE_DEG out-edges
  // The terms of the contiguous-row lift live only during a tile's lift, and
  // only dense and all-vertex rounds take that lift; the predecessor phase
  // comes after the lift, and push stages list entries across the tiles of
  // sparse rounds only.  So the two never overlap in time.
  union {
    V term[2][UNROLL * TERM_ROW];  // contiguous-row lift: the terms of two consecutive chunks
    struct {
      uint32_t ppre[BLOCK + 1];    // exclusive prefix of in-degrees of the tile's changed vertices
      uint32_t pbeg[BLOCK];        // their predecessor-list starts
      V pval[BLOCK];               // their new values (player-1 frontier filter)
      int32_t push[PUSH_CAP];      // sparse: staged entries of L_{r+1}
    };
  };
  unsigned long long st[S_WORDS];
  uint32_t n_push, base;
  uint32_t cbase;  // contiguous-row lift: first edge of the tile's rows, or NO_CONTIG
};
constexpr uint32_t NO_CONTIG = 0xFFFFFFFFu;

// Reads of data used once per round (plain loads measured faster than
// non-temporal ones on gfx950 here).
__device__ __forceinline__ int2 load_edge(const int2* edges, uint32_t e) { return edges[e]; }
// A streamed edge that should not displace the gathered values from L2.
__device__ __forceinline__ int2 load_edge_nt(const int2* edges, uint32_t e) {
  const unsigned long long x = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(edges + e));
  return make_int2((int32_t)(uint32_t)x, (int32_t)(uint32_t)(x >> 32));
}
template <typename T>
__device__ __forceinline__ T load_stream(const T* p) {
  return *p;
}

// Lanes with want = true activate p for L_{r+1} (flag array act_next).
template <bool DENSE, typename V>
__device__ __forceinline__ void activate(const DevGame& g, RoundShared<V>& sh, bool want, int32_t p,
                                         uint8_t* act_next, int32_t* wl_out, uint32_t* cnt_out,
                                         unsigned long long& pushes) {
  // component schedule: a predecessor on a higher level waits for its level
  if (g.level && want && g.level[p] != g.cur_level) want = false;
  if (DENSE) {
    if (want) act_next[p] = 1;  // every writer stores the same value
  } else {
    bool ins = false;
    if (want && act_next[p] == 0) {
      const uint32_t bit = 1u << (8 * (p & 3));
      ins = (atomicOr((uint32_t*)(act_next + (p & ~3)), bit) & bit) == 0;
    }
    pushes += ins;
    const unsigned long long m = __ballot(ins);
    if (m == 0) return;
    const uint32_t leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&sh.n_push, (uint32_t)__popcll(m));
    base = __shfl(base, leader, WAVE);
    if (ins) {
      const uint32_t slot = base + mbcnt(m);
      if (slot < (uint32_t)PUSH_CAP) sh.push[slot] = p;
      else wl_out[atomicAdd(cnt_out, 1u)] = p;  // stage full: append directly
    }
  }
}

// Edges [x0, x0 + J * BLOCK) of the tile's flattened edge range (lanes past E
// re-read the last edge and contribute nothing).  Every lane issues its J edge
// loads and then its J gathers of f with no branch in between, so the gathers
// of a lane overlap instead of each waiting for the one before.
template <typename V, int J>
__device__ __forceinline__ void lift_edges(const DevGame& g, RoundShared<V>& sh, const V* f, uint32_t x0,
                                           uint32_t E, const V* hub = nullptr, uint32_t hub_n = 0) {
  const uint32_t tid = threadIdx.x;
  uint32_t slot[J];
  bool neg[J];
  int2 ed[J];
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t x = x0 + j * BLOCK + tid;
    const uint32_t xc = x < E ? x : E - 1;
    const uint32_t s = find_range(sh.epre, xc);
    const uint32_t beg = sh.ebeg[s];
    slot[j] = x < E ? s : (uint32_t)BLOCK;
    neg[j] = (beg & OWNER_BIT) != 0;
    ed[j] = load_edge(g.edges, (beg & ROW_MASK) + (xc - sh.epre[s]));
  }
  V fu[J];
#pragma unroll
  for (int j = 0; j < J; j++) fu[j] = (uint32_t)ed[j].x < hub_n ? hub[ed[j].x] : f[ed[j].x];
  const uint32_t lane = lane_id();
#pragma unroll
  for (int j = 0; j < J; j++) {
    V tm = fu[j] - (V)ed[j].y;
    tm = tm > V(0) ? tm : V(0);
    // Lanes hold consecutive edges, so lanes of one vertex are contiguous and
    // its keys are folded across the wave first: one LDS atomic per vertex
    // and wave instead of one per edge (the edges of a vertex would all hit
    // the same LDS word).
    V k = neg[j] ? -tm : tm;
    const uint32_t sl = slot[j];
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const V ko = __shfl_down(k, o, WAVE);
      const uint32_t so = __shfl_down(sl, o, WAVE);
      if (lane + o < (uint32_t)WAVE && so == sl) k = ko < k ? ko : k;
    }
    const uint32_t sprev = __shfl_up(sl, 1, WAVE);
    if (sl < BLOCK && (lane == 0 || sprev != sl))
      __hip_atomic_fetch_min(&sh.key[sl], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Edges [x0, min(x0 + J * BLOCK, E)) of a tile whose active rows are one
// contiguous run of edges from `base` (every vertex of the tile active): the
// edge of position x is edges[base + x], so no search is needed to load it.
// The block streams the chunk coalesced (lane i takes positions j * BLOCK + i),
// gathers f of every target with J gathers in flight per lane, and writes the
// unsigned terms max(0, f(u) - w) to LDS.  Then thread t folds the contiguous
// positions [t * J, t * J + J): one search finds the vertex of its first
// edge, the thread walks forward across row boundaries, keeps the running key
// of the current vertex in a register and folds it into the vertex's LDS key
// (one atomic min per vertex and thread) when the row or the run ends.  Ends
// with a barrier: the next chunk rewrites the terms.
// Fold of one chunk of the contiguous-row lift: thread t takes the chunk's
// positions [x0 + t * UNROLL, + UNROLL) below E, finds the vertex of the first
// with one search, walks forward across row ends keeping the running key of
// the current vertex in a register, and folds it into the vertex's LDS key
// (one atomic min per vertex and thread) when the row or the run ends.
template <typename V>
__device__ __forceinline__ void fold_contig(RoundShared<V>& sh, const V* term, uint32_t x0, uint32_t E) {
  const uint32_t tid = threadIdx.x;
  const uint32_t a = x0 + tid * UNROLL;
  if (a >= E) return;
  uint32_t sl = find_range(sh.epre, a);
  uint32_t next = sh.epre[sl + 1];
  bool neg = (sh.ebeg[sl] & OWNER_BIT) != 0;
  V acc = std::numeric_limits<V>::max();
#pragma unroll
  for (int j = 0; j < UNROLL; j++) {
    const uint32_t x = a + j;
    if (x < E) {
      if (x >= next) {  // a row ends inside the run: its vertices have degree >= 1
        __hip_atomic_fetch_min(&sh.key[sl], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        do {
          sl++;
          next = sh.epre[sl + 1];
        } while (x >= next);
        neg = (sh.ebeg[sl] & OWNER_BIT) != 0;
        acc = std::numeric_limits<V>::max();
      }
      const V tm = term[j * TERM_ROW + tid];
      const V k = neg ? -tm : tm;
      acc = k < acc ? k : acc;
    }
  }
  __hip_atomic_fetch_min(&sh.key[sl], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Edges [x0, min(x0 + J * BLOCK, E)) of a tile whose active rows are one
// contiguous run of edges from `base` (every vertex of the tile active): the
// edge of position x is edges[base + x], so no search is needed to load it.
// The block streams the chunk coalesced (lane i takes positions j * BLOCK + i),
// gathers f of every target with J gathers in flight per lane (the values of
// the first hub_n vertices from their LDS copy), writes the unsigned terms
// max(0, f(u) - w) to LDS, and folds them (fold_contig).  Ends with a barrier.
template <typename V, int J>
__device__ __forceinline__ void lift_contig(const DevGame& g, RoundShared<V>& sh, const V* f, uint32_t base,
                                            uint32_t x0, uint32_t E, const V* hub = nullptr, uint32_t hub_n = 0) {
  static_assert(J <= UNROLL, "a chunk holds at most UNROLL * BLOCK terms");
  const uint32_t tid = threadIdx.x;
  int2 ed[J];
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t x = x0 + j * BLOCK + tid;
    ed[j] = load_edge_nt(g.edges, base + (x < E ? x : E - 1));
  }
  V fu[J];
#pragma unroll
  for (int j = 0; j < J; j++) fu[j] = (uint32_t)ed[j].x < hub_n ? hub[ed[j].x] : f[ed[j].x];
#pragma unroll
  for (int j = 0; j < J; j++) {
    V tm = fu[j] - (V)ed[j].y;
    sh.term[0][term_slot(j * BLOCK + tid)] = tm > V(0) ? tm : V(0);
  }
  block_sync();
  fold_contig<V>(sh, sh.term[0], x0, E);
  block_sync();
}

static_assert(UNROLL == 4, "lift_contig_range dispatches chunk widths 1 to 4");

// Positions [lo, hi) of a contiguous tile (block-uniform).  A range of one
// chunk goes to lift_contig with as many edges per lane as it needs.  Longer
// ranges are software-pipelined: the edges of chunk k + 1 are loaded before
// chunk k's terms are published and its gathers issued before chunk k is
// folded, the terms of consecutive chunks alternate between the two LDS
// buffers, and a chunk costs one barrier (the writes of chunk k + 2 into a
// buffer follow, in every thread, the barrier that follows the fold of chunk
// k).  Lanes past hi re-read the last edge and their terms are not folded.
template <typename V>
__device__ __forceinline__ void lift_contig_range(const DevGame& g, RoundShared<V>& sh, const V* f, uint32_t base,
                                                  uint32_t lo, uint32_t hi, const V* hub = nullptr,
                                                  uint32_t hub_n = 0) {
  constexpr uint32_t CH = UNROLL * BLOCK;
  if (hi <= lo) return;
  if (hi - lo <= CH) {
    switch ((hi - lo + BLOCK - 1) / BLOCK) {
      case 1: lift_contig<V, 1>(g, sh, f, base, lo, hi, hub, hub_n); break;
      case 2: lift_contig<V, 2>(g, sh, f, base, lo, hi, hub, hub_n); break;
      case 3: lift_contig<V, 3>(g, sh, f, base, lo, hi, hub, hub_n); break;
      default: lift_contig<V, UNROLL>(g, sh, f, base, lo, hi, hub, hub_n); break;
    }
    return;
  }
  const uint32_t tid = threadIdx.x;
  int2 ed[UNROLL];
  V fu[UNROLL];
#pragma unroll
  for (int j = 0; j < UNROLL; j++) {
    const uint32_t x = lo + j * BLOCK + tid;
    ed[j] = load_edge_nt(g.edges, base + (x < hi ? x : hi - 1));
  }
#pragma unroll
  for (int j = 0; j < UNROLL; j++) fu[j] = (uint32_t)ed[j].x < hub_n ? hub[ed[j].x] : f[ed[j].x];
  uint32_t buf = 0;
  for (uint32_t x0 = lo; x0 < hi; x0 += CH, buf ^= 1u) {
    V* term = sh.term[buf];
#pragma unroll
    for (int j = 0; j < UNROLL; j++) {
      const V tm = fu[j] - (V)ed[j].y;
      term[term_slot(j * BLOCK + tid)] = tm > V(0) ? tm : V(0);
    }
    const uint32_t nx = x0 + CH;
    const bool more = nx < hi;  // block-uniform
    if (more) {
#pragma unroll
      for (int j = 0; j < UNROLL; j++) {
        const uint32_t x = nx + j * BLOCK + tid;
        ed[j] = load_edge_nt(g.edges, base + (x < hi ? x : hi - 1));
      }
    }
    block_sync();  // chunk k's terms are in place
    if (more) {
#pragma unroll
      for (int j = 0; j < UNROLL; j++) fu[j] = (uint32_t)ed[j].x < hub_n ? hub[ed[j].x] : f[ed[j].x];
    }
    fold_contig<V>(sh, term, x0, hi);
  }
  block_sync();  // the last fold is done
}

// First edge of the rows of vertex tile t when the active set of a dense round
// holds every vertex of the tile (E out-edges in all: every vertex has at
// least one, so E equals the span of the tile's rows exactly then), else
// NO_CONTIG.
__device__ __forceinline__ uint32_t contig_base(const DevGame& g, uint32_t t, uint32_t E) {
  const uint32_t first = t * TILE;
  const uint32_t last1 = min((uint32_t)g.n, first + TILE);
  const uint32_t b = g.rs[first] & ROW_MASK;
  return (g.rs[last1] & ROW_MASK) - b == E ? b : NO_CONTIG;
}

// Predecessor entries [x0, x0 + J * BLOCK) of the tile's changed vertices,
// loaded the same way, then activated for the next round.
// With the player-1 frontier filter (g.rev_w set), a player-1 predecessor p of
// a changed v is left out when f(p) >= f(v) (-) w(p, v) already holds (Alg. 1's
// test, Sec. 3.1): lifting p cannot raise it through this edge.  In the device
// encoding the term is TOP (> B) when f(v) - w > B, else max(0, f(v) - w); a
// TOP f(p) satisfies every test.  Exact under in-place updates: f(p) only
// rises, so a test that holds now holds until f(v) rises again, and that rise
// tests again; a stale, lower f(p) only lets more in.
template <bool DENSE, typename V, int J>
__device__ __forceinline__ void scan_preds(const DevGame& g, RoundShared<V>& sh, uint32_t x0, uint32_t P,
                                           uint8_t* act_next, int32_t* wl_out, uint32_t* cnt_out,
                                           unsigned long long& pushes, unsigned long long& filtered) {
  const uint32_t tid = threadIdx.x;
  int32_t pr[J];
  uint32_t k[J], slot[J];
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t x = x0 + j * BLOCK + tid;
    const uint32_t xc = x < P ? x : P - 1;
    const uint32_t s = find_range(sh.ppre, xc);
    slot[j] = s;
    k[j] = sh.pbeg[s] + (xc - sh.ppre[s]);
    pr[j] = load_stream(g.rev_src + k[j]);
    if (x >= P) pr[j] = -1;
  }
  if (g.rev_w) {
    const V* f = (const V*)g.f;
    const V bound = (V)g.bound, top = (V)g.top;
    int32_t w[J];
    uint32_t raw[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
      w[j] = load_stream(g.rev_w + k[j]);
      raw[j] = g.rs[pr[j] >= 0 ? pr[j] : 0];
    }
#pragma unroll
    for (int j = 0; j < J; j++) {
      if (pr[j] >= 0 && (raw[j] & OWNER_BIT)) {
        const V fp = f[pr[j]];
        const V t = sh.pval[slot[j]] - (V)w[j];
        const bool holds = fp == top || (t <= bound && fp >= (t > V(0) ? t : V(0)));
        if (holds) {
          pr[j] = -1;
          filtered++;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < J; j++) activate<DENSE>(g, sh, pr[j] >= 0, pr[j], act_next, wl_out, cnt_out, pushes);
}


// Build L_1: f = 0 (kept on resume) and the round-1 flag on the initially active
// vertices, whose flags were derived from the weights when the game was
// created (player 0: every out-edge negative; player 1: some out-edge
// negative; Alg. 3 line 3); with resume every vertex is active.  Each block
// records how many it activated.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_init(DevGame g, int resume) {
  __shared__ uint32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  block_sync();
  V* f = (V*)g.f;
  uint32_t mine = 0;
  for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * BLOCK) {
    const bool act = resume || ((g.act_bits[v >> 5] >> (v & 31)) & 1u);
    if (!resume) f[v] = 0;
    g.act0[v] = 0;
    g.act1[v] = act ? 1 : 0;
    mine += act;
  }
  atomicAdd(&s_cnt, mine);
  block_sync();
  if (threadIdx.x == 0) {
    g.blk_chg[blockIdx.x] = s_cnt;
    if (s_cnt) g.ctrl[C_ANY0 + 0] = 1;
  }
}

// L_r as a list from its flags (used when a dense round is followed by sparse ones).
__global__ __launch_bounds__(BLOCK) void k_compact(DevGame g, uint32_t r) {
  __shared__ int32_t buf[PUSH_CAP];
  __shared__ uint32_t nb, base;
  int32_t* wl = (r & 1) ? g.wl1 : g.wl0;
  uint32_t* cnt = &g.ctrl[C_CNT0 + r % 3];
  if (threadIdx.x == 0) nb = 0;
  block_sync();
  const uint32_t ntiles = ((uint32_t)g.n + TILE - 1) / TILE;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t v = t * TILE + threadIdx.x;
    lds_append(v < (uint32_t)g.n && ((r & 1) ? g.act1 : g.act0)[v] != 0, (int32_t)v, buf, &nb);
    block_sync();
    if (nb > PUSH_CAP - TILE || t + gridDim.x >= ntiles) {
      if (threadIdx.x == 0) base = nb ? atomicAdd(cnt, nb) : 0;
      block_sync();
      for (uint32_t i = threadIdx.x; i < nb; i += BLOCK) wl[base + i] = buf[i];
      block_sync();
      if (threadIdx.x == 0) nb = 0;
    }
    block_sync();
  }
}

// Per-thread counters of a round (summed per block at the end).
struct Counters {
  unsigned long long lifts = 0, edges = 0, changes = 0, pushes = 0, scanned = 0, filtered = 0;
};

// One tile of a round of Alg. 3 (block-uniform call).  The tile holds TILE
// entries of the active set: list entries (sparse) or vertex ids (dense).
// Every active vertex is lifted in place (chaotic updates are exact, see
// above) and the predecessors of every vertex whose value rose join L_{r+1}.
// The block flattens the work: the out-edges of the tile's active vertices
// are numbered by a block scan of their degrees, each thread takes UNROLL
// edges at a stride of BLOCK (coalesced {target, weight} reads, UNROLL
// gathers of f in flight) and folds its terms into the vertex's LDS key with
// an atomic min (player-1 keys are negated terms, so one min serves both
// players, Def. 6).  The predecessor lists of the changed vertices are
// flattened the same way.  Any degree distribution is balanced across the
// block.  Returns with the shared arrays still in use: the caller
// synchronises before the next tile.
constexpr uint32_t LANE_DEG = 32;  // tiles whose active vertices have at most this many out-edges
constexpr int LANE_UNROLL = 8;      // use one lane per vertex, this many edges in flight per lane
                                    // (games that fit the caches, DevGame::lanes_ok: a lane's row
                                    // loads are not coalesced across the wave, which costs more than
                                    // the search and LDS folding they save once rows come from HBM)

// One lane per active vertex (tiles of small out-degrees): the lane walks its
// own row, LANE_UNROLL edges at a time, loads first and gathers second, and
// keeps the running key in a register.  No edge-to-vertex search and no LDS
// atomics.  The trip count is the wave's largest degree; lanes past their own
// degree re-read their last edge and contribute nothing.
template <typename V>
__device__ __forceinline__ V lift_lanes(const DevGame& g, const V* f, int32_t v, uint32_t raw, uint32_t deg) {
  const bool neg = (raw & OWNER_BIT) != 0;
  V k = neg ? V(0) : std::numeric_limits<V>::max();
  uint32_t dmax = deg;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint32_t y = __shfl_xor(dmax, o, WAVE);
    dmax = y > dmax ? y : dmax;
  }
  const uint32_t e0 = raw & ROW_MASK;
  for (uint32_t j0 = 0; j0 < dmax; j0 += LANE_UNROLL) {
    int2 ed[LANE_UNROLL];
#pragma unroll
    for (int jj = 0; jj < LANE_UNROLL; jj++) {
      const uint32_t j = j0 + jj;
      ed[jj] = load_edge(g.edges, v >= 0 ? e0 + (j < deg ? j : deg - 1) : 0u);
    }
    V fu[LANE_UNROLL];
#pragma unroll
    for (int jj = 0; jj < LANE_UNROLL; jj++) fu[jj] = f[ed[jj].x];
#pragma unroll
    for (int jj = 0; jj < LANE_UNROLL; jj++) {
      V tm = fu[jj] - (V)ed[jj].y;
      tm = tm > V(0) ? tm : V(0);
      const V key = neg ? -tm : tm;
      if (j0 + jj < deg && key < k) k = key;
    }
  }
  return k;
}

// ALL (dense only): every vertex is lifted and nothing is activated; used
// while the frontier covers (nearly) every vertex, where lifting all costs
// less than sweeping flags and activating predecessors.  A lift whose inputs
// did not change leaves its value unchanged, so the result is the same.
template <typename V, bool DENSE, bool PART = false, bool ALL = false>
__device__ __forceinline__ void round_tile(const DevGame& g, RoundShared<V>& sh, uint32_t r, uint32_t t,
                                           uint32_t items, Counters& c) {
  const uint32_t tid = threadIdx.x;
  V* f = (V*)g.f;
  const V bound = (V)g.bound, top = (V)g.top;
  uint8_t* act_cur = (r & 1) ? g.act1 : g.act0;
  uint8_t* act_next = (r & 1) ? g.act0 : g.act1;
  const int32_t* wl_in = (r & 1) ? g.wl1 : g.wl0;
  int32_t* wl_out = (r & 1) ? g.wl0 : g.wl1;
  uint32_t* cnt_out = &g.ctrl[C_CNT0 + (r + 1) % 3];

  const uint32_t idx = t * TILE + tid;
  int32_t v = -1;
  if (idx < items) {
    if (ALL) v = (int32_t)idx;
    else if (DENSE) v = act_cur[idx] ? (int32_t)idx : -1;
    else v = wl_in[idx];
  }
  uint32_t raw = 0, deg = 0, pb = 0, pe = 0;
  V old = 0;
  if (v >= 0) {
    if (!ALL) act_cur[v] = 0;  // consumed
    raw = load_stream(g.rs + v);
    deg = (load_stream(g.rs + v + 1) & ROW_MASK) - (raw & ROW_MASK);
    old = f[v];
    if (!ALL) {
      pb = load_stream(g.rev_off + v);
      pe = load_stream(g.rev_off + v + 1);
    }
  }
  const bool wave_big = __ballot(deg > LANE_DEG) != 0;  // every lane takes part in the ballot
  if (lane_id() == 0) sh.wbig[tid / WAVE] = wave_big;
  uint32_t E;
  const uint32_t ex = block_excl_scan(deg, sh.wsum, &E);  // its barrier also publishes wbig
  const bool lanes = g.lanes_ok && !(sh.wbig[0] | sh.wbig[1] | sh.wbig[2] | sh.wbig[3]);
  sh.epre[tid] = ex;
  if (tid == BLOCK - 1) sh.epre[BLOCK] = E;
  sh.ebeg[tid] = raw;
  sh.key[tid] = (raw & OWNER_BIT) ? V(0) : std::numeric_limits<V>::max();
  // every vertex of an all-vertex tile is active: its rows start at thread 0's
  if ((DENSE || ALL) && !PART && tid == 0) sh.cbase = ALL ? (raw & ROW_MASK) : contig_base(g, t, E);
  if (PART && v >= 0) {
    // the slices' partial keys of v, computed by k_partial (one per slice), or
    // its key combined over the slices by k_sliced
    V k = sh.key[tid];
    const V* part = (const V*)g.part;
    const uint32_t nk = g.slice_major ? 1u : g.nparts;
    for (uint32_t q = 0; q < nk; q++) {
      const V y = part[(size_t)q * (uint32_t)g.n + (uint32_t)v];
      k = y < k ? y : k;
    }
    sh.key[tid] = k;
  }
  // slice-major: every key is reset for the next round (a larger key is the
  // identity of the min for both players: every vertex has an out-edge)
  if (PART && g.slice_major && idx < items) ((V*)g.part)[idx] = std::numeric_limits<V>::max();
  block_sync();
  if (E == 0) return;  // block-uniform: no active vertex in this tile

  if (!PART && lanes) {
    sh.key[tid] = lift_lanes<V>(g, f, v, raw, deg);
  } else if (!PART && (DENSE || ALL) && sh.cbase != NO_CONTIG) {
    lift_contig_range<V>(g, sh, f, sh.cbase, 0, E);
  } else if (!PART) {
    for (uint32_t x0 = 0; x0 < E; x0 += BLOCK * UNROLL) {
      switch (std::min<uint32_t>((E - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
        case 1: lift_edges<V, 1>(g, sh, f, x0, E); break;
        case 2: lift_edges<V, 2>(g, sh, f, x0, E); break;
        case 3: lift_edges<V, 3>(g, sh, f, x0, E); break;
        case 4: lift_edges<V, 4>(g, sh, f, x0, E); break;
        case 5: lift_edges<V, 5>(g, sh, f, x0, E); break;
        case 6: lift_edges<V, 6>(g, sh, f, x0, E); break;
        case 7: lift_edges<V, 7>(g, sh, f, x0, E); break;
        default: lift_edges<V, UNROLL>(g, sh, f, x0, E); break;
      }
    }
  }
  block_sync();

  uint32_t ideg = 0;
  V nval = 0;
  if (v >= 0) {
    const V k = sh.key[tid];
    V nv = (raw & OWNER_BIT) ? -k : k;
    if (nv > bound) nv = top;
    // Writes never lower a value.  From f = 0 (or any measure below the least
    // fixpoint that lifts do not lower) this changes nothing; from a measure
    // with values raised by other means it keeps every stop point a
    // pre-fixpoint, and the least pre-fixpoint is the least fixpoint.
    if (nv < old) nv = old;
    c.lifts++;
    c.edges += deg;
    if (nv != old) {
      f[v] = nv;
      nval = nv;
      c.changes++;
      ideg = pe - pb;
    }
    // all-vertex rounds leave a flag on each vertex they raise, in their own
    // (otherwise unused) flag array: k_activate_changed turns the last one's
    // flags into the next active set
    if (ALL) act_cur[v] = nv != old ? 1 : 0;
  }
  if (ALL) return;
  uint32_t P;
  const uint32_t pex = block_excl_scan(ideg, sh.wsum, &P);
  sh.ppre[tid] = pex;
  if (tid == BLOCK - 1) sh.ppre[BLOCK] = P;
  sh.pbeg[tid] = pb;
  sh.pval[tid] = nval;
  c.scanned += ideg;
  block_sync();
  for (uint32_t x0 = 0; x0 < P; x0 += BLOCK * UNROLL) {
    switch (std::min<uint32_t>((P - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
      case 1: scan_preds<DENSE, V, 1>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 2: scan_preds<DENSE, V, 2>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 3: scan_preds<DENSE, V, 3>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 4: scan_preds<DENSE, V, 4>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 5: scan_preds<DENSE, V, 5>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 6: scan_preds<DENSE, V, 6>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      case 7: scan_preds<DENSE, V, 7>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
      default: scan_preds<DENSE, V, UNROLL>(g, sh, x0, P, act_next, wl_out, cnt_out, c.pushes, c.filtered); break;
    }
  }
}

// Records [x0, x0 + J * BLOCK) of a chunk of the target-sliced edge copy into
// the tile's LDS keys (loads first, as in lift_edges).
template <typename V, int J>
__device__ __forceinline__ void slice_edges(const DevGame& g, V* key, const uint32_t* own, const V* f, uint32_t x0,
                                            uint32_t end) {
  const uint32_t tid = threadIdx.x;
  int2 ed[J];
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t x = x0 + j * BLOCK + tid;
    ed[j] = g.pedges[x < end ? x : end - 1];
  }
  V fu[J];
#pragma unroll
  for (int j = 0; j < J; j++) fu[j] = f[(uint32_t)ed[j].x & ((1u << PTILE_SHIFT) - 1)];
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t loc = (uint32_t)ed[j].x >> PTILE_SHIFT;
    V tm = fu[j] - (V)ed[j].y;
    tm = tm > V(0) ? tm : V(0);
    if (x0 + j * BLOCK + tid < end)
      __hip_atomic_fetch_min(&key[loc], ((own[loc >> 5] >> (loc & 31)) & 1u) ? -tm : tm, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Segment `seg` of `nseg` of a dense tile (full-frontier sizes are balanced:
// a tile whose out-degree sum exceeds SEG_EDGES is cut so that no block takes
// much more than SEG_EDGES edges).  Every segment block rebuilds the tile's
// flattened edge range from the flags, which only the last block clears, and
// lifts its share of the range into LDS keys.  An uncut tile finishes in its
// block.  Otherwise each block folds the keys it touched into gkey with
// atomic min, and the block that finishes the tile's last segment (a counter
// per tile) completes the round for the whole tile from gkey: the new values,
// the flag clearing and the predecessor activation.
template <typename V, bool ALL = false>
__device__ __forceinline__ void round_seg(const DevGame& g, RoundShared<V>& sh, uint32_t r, uint32_t t,
                                          uint32_t seg, uint32_t nseg, Counters& c, uint32_t& s_last,
                                          const V* hub, uint32_t hub_n) {
  const uint32_t tid = threadIdx.x;
  V* f = (V*)g.f;
  V* gkey = (V*)g.gkey;
  const V bound = (V)g.bound, top = (V)g.top;
  uint8_t* act_cur = (r & 1) ? g.act1 : g.act0;
  uint8_t* act_next = (r & 1) ? g.act0 : g.act1;
  const uint32_t idx = t * TILE + tid;
  const bool in = idx < (uint32_t)g.n;
  const bool was_active = in && (ALL || act_cur[idx]);
  // A tile with at least half of its vertices active lifts all of them: its
  // rows are then one contiguous run of edges (the cheaper contiguous-row
  // lift), and lifting a vertex whose successors did not change returns its
  // value, so the extra lifts are exact.  Only the active ones are counted as
  // work (lifts, relaxed edges).  Every segment block of a cut tile reads the
  // same flags (the tile's last block clears them), so all decide alike.
  bool lifted = was_active;
  if (!ALL) {
    const uint32_t nact = (uint32_t)__syncthreads_count(was_active);
    const uint32_t nin = min((uint32_t)TILE, (uint32_t)g.n - t * TILE);
    if (2 * nact >= nin) lifted = in;
  }
  int32_t v = lifted ? (int32_t)idx : -1;
  uint32_t raw = 0, deg = 0, pb = 0, pe = 0;
  V old = 0;
  if (v >= 0) {
    raw = load_stream(g.rs + v);
    deg = (load_stream(g.rs + v + 1) & ROW_MASK) - (raw & ROW_MASK);
    old = f[v];
    if (!ALL) {
      pb = load_stream(g.rev_off + v);
      pe = load_stream(g.rev_off + v + 1);
    }
  }
  const bool wave_big = __ballot(deg > LANE_DEG) != 0;  // every lane takes part in the ballot
  if (lane_id() == 0) sh.wbig[tid / WAVE] = wave_big;
  uint32_t E;
  const uint32_t ex = block_excl_scan(deg, sh.wsum, &E);  // its barrier also publishes wbig
  const bool lanes = g.lanes_ok && nseg == 1 && !(sh.wbig[0] | sh.wbig[1] | sh.wbig[2] | sh.wbig[3]);
  sh.epre[tid] = ex;
  if (tid == BLOCK - 1) sh.epre[BLOCK] = E;
  sh.ebeg[tid] = raw;
  const V ident = (raw & OWNER_BIT) ? V(0) : std::numeric_limits<V>::max();
  sh.key[tid] = ident;
  if (tid == 0) sh.cbase = ALL ? (raw & ROW_MASK) : contig_base(g, t, E);
  block_sync();
  if (E == 0) return;  // block-uniform, and the same in every segment block of the tile
  const uint32_t lo = (uint32_t)((uint64_t)E * seg / nseg), hi = (uint32_t)((uint64_t)E * (seg + 1) / nseg);
  const bool contig = !lanes && sh.cbase != NO_CONTIG;
  if (lanes) sh.key[tid] = lift_lanes<V>(g, f, v, raw, deg);
  if (contig) lift_contig_range<V>(g, sh, f, sh.cbase, lo, hi, hub, hub_n);
  for (uint32_t x0 = lo; x0 < (lanes || contig ? lo : hi); x0 += BLOCK * UNROLL) {
    switch (std::min<uint32_t>((hi - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
      case 1: lift_edges<V, 1>(g, sh, f, x0, hi, hub, hub_n); break;
      case 2: lift_edges<V, 2>(g, sh, f, x0, hi, hub, hub_n); break;
      case 3: lift_edges<V, 3>(g, sh, f, x0, hi, hub, hub_n); break;
      default: lift_edges<V, UNROLL>(g, sh, f, x0, hi, hub, hub_n); break;
    }
  }
  block_sync();
  V k = sh.key[tid];
  if (nseg > 1) {
    // Keys, tile counter and the last block's reads are device-scope atomics,
    // performed where every XCD sees them.  Each wave waits until its key
    // updates are performed before the counter is bumped, so the block that
    // takes the last segment reads complete keys.  No fence is used: a fence
    // would write back and invalidate the XCD's L2 and with it the cached f.
    if (v >= 0 && ex < hi && ex + deg > lo)
      __hip_atomic_fetch_min(gkey + v, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    block_sync();
    if (tid == 0)
      s_last = __hip_atomic_fetch_add(&g.tile_done[t], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nseg - 1
                   ? 1u
                   : 0u;
    block_sync();
    if (!s_last) return;
    if (v >= 0) {
      k = __hip_atomic_load(gkey + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      gkey[v] = ident;
    }
    if (tid == 0) g.tile_done[t] = 0;
  }
  uint32_t ideg = 0;
  V nval = 0;
  if (v >= 0) {
    V nv = (raw & OWNER_BIT) ? -k : k;
    if (nv > bound) nv = top;
    if (nv < old) nv = old;  // writes never lower a value (see round_tile)
    // consumed; all-vertex rounds flag the vertices they raise (see round_tile)
    act_cur[v] = ALL && nv != old ? 1 : 0;
    if (was_active) {
      c.lifts++;
      c.edges += deg;
    }
    if (nv != old) {
      f[v] = nv;
      nval = nv;
      c.changes++;
      ideg = pe - pb;
    }
  }
  if (ALL) return;
  uint32_t P;
  const uint32_t pex = block_excl_scan(ideg, sh.wsum, &P);
  sh.ppre[tid] = pex;
  if (tid == BLOCK - 1) sh.ppre[BLOCK] = P;
  sh.pbeg[tid] = pb;
  sh.pval[tid] = nval;
  c.scanned += ideg;
  block_sync();
  for (uint32_t x0 = 0; x0 < P; x0 += BLOCK * UNROLL) {
    switch (std::min<uint32_t>((P - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
      case 1: scan_preds<true, V, 1>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 2: scan_preds<true, V, 2>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 3: scan_preds<true, V, 3>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 4: scan_preds<true, V, 4>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 5: scan_preds<true, V, 5>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 6: scan_preds<true, V, 6>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      case 7: scan_preds<true, V, 7>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      default: scan_preds<true, V, UNROLL>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
    }
  }
}

// A dense round over the segments of the tiles (see round_seg).
template <typename V, bool ALL = false>
__global__ __launch_bounds__(BLOCK) void k_round_seg(DevGame g, uint32_t r) {
  __shared__ RoundShared<V> sh;
  __shared__ uint32_t s_last;
  // copy of f(0 .. hub_n) in LDS, the most gathered values of a game renumbered
  // by in-degree (dynamic shared memory of hub_n values; a copy taken at the
  // start of the round is an earlier value, which the in-place iteration
  // allows: a change after it re-activates the readers)
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  V* hub = reinterpret_cast<V*>(dyn_lds);
  const uint32_t tid = threadIdx.x;
  const uint32_t items = g.ctrl[C_ANY0 + (r - 1) % 3] ? g.nitems : 0u;
  if (blockIdx.x == 0 && tid == 0) {
    g.ctrl[C_CNT0 + (r + 2) % 3] = 0;
    g.ctrl[C_ANY0 + (r + 1) % 3] = 0;
    if (items) g.ctrl[C_ROUNDS] += 1;
  }
  if (items == 0) {
    if (tid == 0) g.blk_chg[blockIdx.x] = 0;
    return;
  }
  if (tid < S_WORDS) sh.st[tid] = 0;
  const uint32_t hub_n = g.hub_n;
  {
    const V* f = (const V*)g.f;
    for (uint32_t i = tid; i < hub_n; i += BLOCK) hub[i] = f[i];
  }
  Counters c;
  for (uint32_t x = blockIdx.x; x < items; x += gridDim.x) {
    block_sync();  // the previous item is done with the shared arrays (and the hub copy is in place)
    const uint32_t t = g.item_tile[x];
    round_seg<V, ALL>(g, sh, r, t, g.item_seg[x], g.tile_nseg[t], c, s_last, hub, hub_n);
  }
  block_counters(sh, c);
  if (tid < S_WORDS) g.slots[blockIdx.x * S_WORDS + tid] += sh.st[tid];
  if (tid == 0) {
    g.blk_chg[blockIdx.x] = (uint32_t)sh.st[S_CHANGES];
    if (sh.st[S_CHANGES]) g.ctrl[C_ANY0 + r % 3] = 1;
  }
}

template <typename V>
__global__ void k_gkey_init(DevGame g) {
  V* gkey = (V*)g.gkey;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x)
    gkey[v] = (g.rs[v] & OWNER_BIT) ? V(0) : std::numeric_limits<V>::max();
}

// Partial keys of every vertex of a tile over the targets of one slice, for a
// dense round that reads the partitioned edge copy.  Block b works on the
// slices of XCD b % 8 (workgroups are dealt to the XCDs in turn), so each
// XCD gathers f only from its own slices, which stay in its L2.  Keys are
// computed for all vertices of the tile; the combining round uses those of
// active vertices only.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_partial(DevGame g, uint32_t r) {
  __shared__ V key[PTILE];
  __shared__ uint32_t own[PTILE / 32];
  if (g.ctrl[C_ANY0 + (r - 1) % 3] == 0) return;  // L_r is empty
  const V* f = (const V*)g.f;
  const uint32_t tid = threadIdx.x;
  const uint32_t n = (uint32_t)g.n, nparts = g.nparts;
  const uint32_t ntiles = (n + PTILE - 1) / PTILE;
  const uint32_t xcd = blockIdx.x % 8, lb = blockIdx.x / 8, nlb = gridDim.x / 8;
  const uint32_t per_xcd = nparts / 8;
  const uint32_t items = ntiles * per_xcd;
  const uint32_t nwords = (n + 31) / 32;
  for (uint32_t i = lb; i < items; i += nlb) {
    const uint32_t tile = i / per_xcd, q = xcd + 8 * (i % per_xcd);
    const uint32_t v0 = tile * PTILE;
    block_sync();
    for (uint32_t j = tid; j < PTILE / 32; j += BLOCK) own[j] = v0 / 32 + j < nwords ? g.own_bits[v0 / 32 + j] : 0u;
    block_sync();
    for (uint32_t j = tid; j < PTILE; j += BLOCK)
      key[j] = ((own[j >> 5] >> (j & 31)) & 1u) ? V(0) : std::numeric_limits<V>::max();
    block_sync();
    const uint32_t c = tile * nparts + q;
    const uint32_t beg = g.poff[c], end = g.poff[c + 1];
    for (uint32_t x0 = beg; x0 < end; x0 += BLOCK * UNROLL) {
      switch (std::min<uint32_t>((end - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
        case 1: slice_edges<V, 1>(g, key, own, f, x0, end); break;
        case 2: slice_edges<V, 2>(g, key, own, f, x0, end); break;
        case 3: slice_edges<V, 3>(g, key, own, f, x0, end); break;
        case 4: slice_edges<V, 4>(g, key, own, f, x0, end); break;
        case 5: slice_edges<V, 5>(g, key, own, f, x0, end); break;
        case 6: slice_edges<V, 6>(g, key, own, f, x0, end); break;
        case 7: slice_edges<V, 7>(g, key, own, f, x0, end); break;
        default: slice_edges<V, UNROLL>(g, key, own, f, x0, end); break;
      }
    }
    block_sync();
    V* part = (V*)g.part + (size_t)q * n;
    for (uint32_t j = tid; j < PTILE && v0 + j < n; j += BLOCK) part[v0 + j] = key[j];
  }
}

// Slice-major dense round, first kernel (partition mode 3).  The edge copy is
// grouped by (tile of PTILE sources, target slice), with slices of about
// SL_SLICE_BYTES of f.  Every block owns the work items sl_items[sl_begin[b]
// .. sl_begin[b+1]) (tiles, or equal parts of the edges of a tile whose edges
// exceed a block's share), balanced by edges when the game is created, and
// takes them SL_SLOTS at a time: their keys stay in LDS while the block sweeps
// the slices in order, so that all blocks gather f from about the same slice
// at the same time and the gathers hit in L2.  The keys of a group then go to
// part[]: a plain store for a whole tile, an atomic min for the parts of a cut
// tile (part[] is reset to the largest key by the combining round, which turns
// the keys into values: round_tile with PART).  Only f is read, so the keys
// are those of a synchronous round.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_sliced(DevGame g, uint32_t r) {
  static_assert(SL_SLOTS * 64 <= BLOCK, "one chunk of the group per thread in the scan");
  __shared__ V key[SL_SLOTS * PTILE];
  __shared__ uint32_t own[SL_SLOTS * (PTILE / 32)];
  __shared__ uint2 s_item[SL_SLOTS];
  __shared__ uint32_t cpre[BLOCK + 1];  // exclusive prefix of the chunk lengths, slice-major
  __shared__ uint32_t cbeg[BLOCK];      // first edge of each chunk in the edge copy
  __shared__ uint32_t wsum[BLOCK / WAVE];
  if (g.ctrl[C_ANY0 + (r - 1) % 3] == 0) return;  // L_r is empty
  const V* f = (const V*)g.f;
  V* part = (V*)g.part;
  const uint32_t tid = threadIdx.x;
  const uint32_t n = (uint32_t)g.n, nparts = g.nparts;
  const uint32_t nwords = (n + 31) / 32;
  const uint32_t ib = g.sl_begin[blockIdx.x], ie = g.sl_begin[blockIdx.x + 1];
  for (uint32_t i0 = ib; i0 < ie; i0 += SL_SLOTS) {
    const uint32_t ni = min(SL_SLOTS, ie - i0);
    block_sync();  // the previous group's keys have been written out
    if (tid < ni) s_item[tid] = g.sl_items[i0 + tid];
    block_sync();
    for (uint32_t j = tid; j < ni * (PTILE / 32); j += BLOCK) {
      const uint32_t w = s_item[j / (PTILE / 32)].x * (PTILE / 32) + j % (PTILE / 32);
      own[j] = w < nwords ? g.own_bits[w] : 0u;
    }
    // chunk c = slice * ni + slot of the group: its edge range in the copy
    const uint32_t nch = nparts * ni;
    uint32_t len = 0;
    if (tid < nch) {
      const uint2 it = s_item[tid % ni];
      const uint32_t c = it.x * nparts + tid / ni;
      const uint32_t a = g.poff[c], b = g.poff[c + 1];
      const uint32_t pj = it.y >> 16, pc = it.y & 0xFFFFu;
      const uint32_t lo = a + (uint32_t)((uint64_t)(b - a) * pj / pc);
      const uint32_t hi = a + (uint32_t)((uint64_t)(b - a) * (pj + 1) / pc);
      cbeg[tid] = lo;
      len = hi - lo;
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan(len, wsum, &total);  // its barrier also publishes own and cbeg
    cpre[tid] = ex;
    if (tid == BLOCK - 1) cpre[BLOCK] = total;
    for (uint32_t j = tid; j < ni * PTILE; j += BLOCK)
      key[j] = ((own[j >> 5] >> (j & 31)) & 1u) ? V(0) : std::numeric_limits<V>::max();
    block_sync();
    // The group's chunks as one range of `total` edges, slice by slice: every
    // step keeps UNROLL * BLOCK edges in flight and moves through the slices
    // in order.  Each lane walks its own chunk cursor forward (its positions
    // only grow).
    uint32_t cur = 0;
    for (uint32_t x0 = 0; x0 < total; x0 += BLOCK * UNROLL) {
      int2 ed[UNROLL];
      uint32_t slot[UNROLL];
#pragma unroll
      for (int jj = 0; jj < UNROLL; jj++) {
        const uint32_t x = x0 + jj * BLOCK + tid;
        const uint32_t xc = x < total ? x : total - 1;
        while (cpre[cur + 1] <= xc) cur++;
        slot[jj] = cur % ni;
        ed[jj] = load_edge_nt(g.pedges, cbeg[cur] + (xc - cpre[cur]));
      }
      V fu[UNROLL];
#pragma unroll
      for (int jj = 0; jj < UNROLL; jj++) fu[jj] = f[(uint32_t)ed[jj].x & ((1u << PTILE_SHIFT) - 1)];
#pragma unroll
      for (int jj = 0; jj < UNROLL; jj++) {
        const uint32_t loc = slot[jj] * PTILE + ((uint32_t)ed[jj].x >> PTILE_SHIFT);
        V tm = fu[jj] - (V)ed[jj].y;
        tm = tm > V(0) ? tm : V(0);
        if (x0 + jj * BLOCK + tid < total)
          __hip_atomic_fetch_min(&key[loc], ((own[loc >> 5] >> (loc & 31)) & 1u) ? -tm : tm, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    block_sync();
    for (uint32_t j = tid; j < ni * PTILE; j += BLOCK) {
      const uint2 it = s_item[j / PTILE];
      const uint32_t v = it.x * PTILE + j % PTILE;
      if (v >= n) continue;
      if ((it.y & 0xFFFFu) == 1) part[v] = key[j];
      else __hip_atomic_fetch_min(part + v, key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename V>
__global__ void k_fill_max(V* p, int32_t n) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)n; v += gridDim.x * blockDim.x)
    p[v] = std::numeric_limits<V>::max();
}

// Sum the counters of the block into LDS (sh.st must be zero on entry).
template <typename V>
__device__ __forceinline__ void block_counters(RoundShared<V>& sh, const Counters& c) {
  atomicAdd(&sh.st[S_LIFTS], c.lifts);
  atomicAdd(&sh.st[S_EDGES], c.edges);
  atomicAdd(&sh.st[S_CHANGES], c.changes);
  atomicAdd(&sh.st[S_PUSHES], c.pushes);
  atomicAdd(&sh.st[S_SCANNED], c.scanned);
  atomicAdd(&sh.st[S_FILTERED], c.filtered);
  block_sync();
}

// After all-vertex rounds: the predecessors of the vertices that the last one
// (round r - 1) raised join L_r (flags of round r, cleared by the caller), with
// the same predecessor scan and filter as the end of a dense round; the raise
// flags are cleared for the flags of round r + 1.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_activate_changed(DevGame g, uint32_t r) {
  __shared__ RoundShared<V> sh;
  const uint32_t tid = threadIdx.x;
  uint8_t* raised = (r & 1) ? g.act0 : g.act1;  // flags of round r - 1 (= r + 1)
  uint8_t* act_next = (r & 1) ? g.act1 : g.act0;
  const V* f = (const V*)g.f;
  if (tid < S_WORDS) sh.st[tid] = 0;
  Counters c;
  const uint32_t ntiles = ((uint32_t)g.n + TILE - 1) / TILE;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t v = t * TILE + tid;
    uint32_t ideg = 0, pb = 0;
    V val = 0;
    if (v < (uint32_t)g.n && raised[v]) {
      raised[v] = 0;
      pb = g.rev_off[v];
      ideg = g.rev_off[v + 1] - pb;
      val = f[v];
    }
    uint32_t P;
    const uint32_t pex = block_excl_scan(ideg, sh.wsum, &P);  // also orders the previous tile's reads
    sh.ppre[tid] = pex;
    if (tid == BLOCK - 1) sh.ppre[BLOCK] = P;
    sh.pbeg[tid] = pb;
    sh.pval[tid] = val;
    c.scanned += ideg;
    block_sync();
    for (uint32_t x0 = 0; x0 < P; x0 += BLOCK * UNROLL) {
      switch (std::min<uint32_t>((P - x0 + BLOCK - 1) / BLOCK, UNROLL)) {
        case 1: scan_preds<true, V, 1>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
        case 2: scan_preds<true, V, 2>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
        case 3: scan_preds<true, V, 3>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
        default: scan_preds<true, V, UNROLL>(g, sh, x0, P, act_next, nullptr, nullptr, c.pushes, c.filtered); break;
      }
    }
    block_sync();  // the next tile rewrites ppre, pbeg and pval
  }
  block_counters(sh, c);
  if (tid < S_WORDS) g.slots[blockIdx.x * S_WORDS + tid] += sh.st[tid];
}

// One round of Alg. 3 over L_r of one game: blocks take the tiles of the
// active set in turn (see round_tile).
template <typename V, bool DENSE, bool PART = false, bool ALL = false>
__global__ __launch_bounds__(BLOCK) void k_round(DevGame g, uint32_t r) {
  __shared__ RoundShared<V> sh;
  const uint32_t tid = threadIdx.x;
  uint32_t items;
  if (DENSE) items = g.ctrl[C_ANY0 + (r - 1) % 3] ? (uint32_t)g.n : 0u;
  else items = g.ctrl[C_CNT0 + r % 3];
  if (blockIdx.x == 0 && tid == 0) {
    g.ctrl[C_CNT0 + (r + 2) % 3] = 0;  // recycled for round r+2
    g.ctrl[C_ANY0 + (r + 1) % 3] = 0;  // written by round r+1
    if (items) g.ctrl[C_ROUNDS] += 1;
  }
  if (items == 0) {
    if (tid == 0) g.blk_chg[blockIdx.x] = 0;
    return;
  }
  if (tid == 0) sh.n_push = 0;
  if (tid < S_WORDS) sh.st[tid] = 0;
  Counters c;
  const uint32_t ntiles = (items + TILE - 1) / TILE;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    block_sync();  // the previous tile is done with the shared arrays
    round_tile<V, DENSE, PART, ALL>(g, sh, r, t, items, c);
  }
  block_counters(sh, c);
  if (!DENSE) {
    uint32_t* cnt_out = &g.ctrl[C_CNT0 + (r + 1) % 3];
    int32_t* wl_out = (r & 1) ? g.wl0 : g.wl1;
    const uint32_t nf = sh.n_push < (uint32_t)PUSH_CAP ? sh.n_push : (uint32_t)PUSH_CAP;
    if (tid == 0) sh.base = nf ? atomicAdd(cnt_out, nf) : 0u;
    block_sync();
    for (uint32_t i = tid; i < nf; i += BLOCK) wl_out[sh.base + i] = sh.push[i];
  }
  if (tid < S_WORDS) g.slots[blockIdx.x * S_WORDS + tid] += sh.st[tid];
  if (tid == 0) {
    g.blk_chg[blockIdx.x] = (uint32_t)sh.st[S_CHANGES];
    if (sh.st[S_CHANGES]) g.ctrl[C_ANY0 + r % 3] = 1;
  }
}

// Many rounds of one game in a single block, for small active sets: a round
// of a few tiles costs a few dependent cache hits here instead of a kernel
// launch.  Starts at round r0 (sparse list), stops before a round whose list
// is empty (the fixpoint) or longer than `limit`, or after `max_rounds`, and
// returns the round to run next (k_rounds_small stores it in ctrl[C_NEXT]).
// All waves of the block share one CU and its caches, so the block barrier
// orders rounds.
// deadline (nonzero): also stop before a round that would start after this
// value of the constant-rate realtime counter (s_memrealtime).
template <typename V>
__device__ uint32_t small_rounds(const DevGame& g, RoundShared<V>& sh, uint32_t r0, uint32_t max_rounds,
                                 uint32_t limit, uint32_t& s_items, int& s_changed, Counters& c,
                                 uint64_t deadline = 0) {
  const uint32_t tid = threadIdx.x;
  uint32_t r = r0;
  for (uint32_t k = 0; k < max_rounds; k++, r++) {
    block_sync();
    if (tid == 0) {
      uint32_t items = g.ctrl[C_CNT0 + r % 3];
      // out of time: stop as before an oversized round (nothing is changed)
      if (deadline && k > 0 && __builtin_amdgcn_s_memrealtime() >= deadline) items = 0xFFFFFFFFu;
      s_items = items;
      s_changed = 0;
      sh.n_push = 0;
      if (items != 0 && items <= limit) {
        g.ctrl[C_CNT0 + (r + 2) % 3] = 0;
        g.ctrl[C_ANY0 + (r + 1) % 3] = 0;
        g.ctrl[C_ROUNDS] += 1;
      }
    }
    block_sync();
    const uint32_t items = s_items;
    if (items == 0 || items > limit) break;
    const unsigned long long before = c.changes;
    const uint32_t ntiles = (items + TILE - 1) / TILE;
    for (uint32_t t = 0; t < ntiles; t++) {
      block_sync();
      round_tile<V, false>(g, sh, r, t, items, c);
    }
    block_sync();
    if (c.changes != before) s_changed = 1;
    uint32_t* cnt_out = &g.ctrl[C_CNT0 + (r + 1) % 3];
    int32_t* wl_out = (r & 1) ? g.wl0 : g.wl1;
    const uint32_t nf = sh.n_push < (uint32_t)PUSH_CAP ? sh.n_push : (uint32_t)PUSH_CAP;
    if (tid == 0) sh.base = nf ? atomicAdd(cnt_out, nf) : 0u;
    block_sync();
    for (uint32_t i = tid; i < nf; i += BLOCK) wl_out[sh.base + i] = sh.push[i];
    if (tid == 0 && s_changed) g.ctrl[C_ANY0 + r % 3] = 1;
  }
  block_sync();
  return r;
}

template <typename V>
__global__ __launch_bounds__(BLOCK) void k_rounds_small(DevGame g, uint32_t r0, uint32_t max_rounds,
                                                         uint32_t limit) {
  __shared__ RoundShared<V> sh;
  __shared__ uint32_t s_items;
  __shared__ int s_changed;
  const uint32_t tid = threadIdx.x;
  if (tid < S_WORDS) sh.st[tid] = 0;
  Counters c;
  const uint32_t r = small_rounds<V>(g, sh, r0, max_rounds, limit, s_items, s_changed, c);
  block_counters(sh, c);
  if (tid < S_WORDS) g.slots[tid] += sh.st[tid];
  if (tid == 0) g.ctrl[C_NEXT] = r;
}

hipError_t launch_rounds_small(const DevGame& g, int vbits, uint32_t r0, uint32_t max_rounds, uint32_t limit,
                               hipStream_t s) {
  if (vbits == 32)
    hipLaunchKernelGGL(k_rounds_small<int32_t>, dim3(1), dim3(BLOCK), 0, s, g, r0, max_rounds, limit);
  else
    hipLaunchKernelGGL(k_rounds_small<int64_t>, dim3(1), dim3(BLOCK), 0, s, g, r0, max_rounds, limit);
  return hipGetLastError();
}

// ---------------------------------------------------------------- TOP seeding
//
// A vertex is TOP exactly when player 1 wins from it.  A cheap proof: fix for
// every player-1 vertex one out-edge (sigma1), and take the forced subgraph of
// player-1 vertices and player-0 vertices of out-degree 1.  A cycle of the
// chosen edges whose weights sum below zero can be forced by player 1 forever
// (every player-0 vertex on it has no other edge), so by Lemma 1 all its
// vertices are TOP.  sigma1(v) is the out-edge into the forced subgraph with
// the largest term under the current measure (the lowest index on ties): the
// edge a player-1 lift would follow.  The chosen edges form a functional
// graph; after ceil(log2 n) + 1 doublings succ^(2^k)(v) lies on the cycle that
// v's walk ends in, the image of that map is exactly the set of cycle
// vertices, and the smallest vertex id along 2^k >= n steps names the cycle.
// Setting TOP on those vertices keeps the measure below the least fixpoint,
// and with writes that never lower a value the iteration still ends at it.

__global__ void k_seed_forced(DevGame g, SeedBuf sb) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const uint32_t a = g.rs[v], b = g.rs[v + 1] & ROW_MASK;
    sb.forced[v] = (a & OWNER_BIT) || b - (a & ROW_MASK) == 1 ? 1 : 0;
  }
}

// Edges per lane per step of the seeding scans.
constexpr int SEED_UNROLL = 4;
// Predecessor lists of new TOP vertices up to this length are flagged by their
// own lane, longer ones by the whole wave.
constexpr uint32_t SEED_SHORT = 32;
// Player-1 rows up to SEED_FLAT edges are scanned flattened per tile; longer
// ones go to lists scanned a row per wave (up to SEED_LONG edges) and a row
// per block, so that no tile of hubs (the hubs of power-law games sit next to
// each other, and renumbering puts them together) holds up one block.
// Predecessor lists longer than SEED_LONG are flagged by a block each too.
constexpr uint32_t SEED_FLAT = 64;
constexpr uint32_t SEED_LONG = 2048;
constexpr int SEED_LONG_GRID = 1024;
constexpr int SEED_MID_GRID = 2048;

// Candidate order of sigma1: a negative self-loop first (player 1 can stay on
// it forever, so it is always a certificate), then the largest term, then the
// lowest edge index.  Returns true when (lb, tb, kb) beats (la, ta, ka).
template <typename V>
__device__ __forceinline__ bool seed_better(bool lb, V tb, uint32_t kb, bool la, V ta, uint32_t ka) {
  if (lb != la) return lb;
  if (tb != ta) return tb > ta;
  return kb < ka;
}

// Segmented fold over the lanes of a wave whose slots run in contiguous
// groups: afterwards the first lane of each group holds the group's best
// (has, x) under better(); lanes with has = false hold no candidate.
template <typename T, typename Better>
__device__ __forceinline__ void wave_seg_fold(bool& has, T& x, uint32_t slot, Better better) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const T xo = __shfl_down(x, o, WAVE);
    const bool ho = __shfl_down((int)has, o, WAVE) != 0;
    const uint32_t so = __shfl_down(slot, o, WAVE);
    if (lane + o < (uint32_t)WAVE && so == slot && ho && (!has || better(xo, x))) {
      x = xo;
      has = true;
    }
  }
}

// Bellman-Ford seeding passes (sb.fbf set): the values iterated are those of
// the game restricted to the forced subgraph, where player 1 picks among
// forced successors and player 0 has no choice; from f (a measure below the
// least fixpoint) they stay below it, since that restriction only drops
// player-1 options.  The chosen edge's term under them raises v's value
// (capped at the TOP encoding; a value above B proves TOP).
template <typename V>
__device__ __forceinline__ void seed_raise(const DevGame& g, const SeedBuf& sb, int32_t v, int32_t to, int32_t w) {
  if (!sb.fbf || to < 0) return;
  V* b = (V*)sb.fbf;
  V tm = b[to] - (V)w;
  tm = tm > V(0) ? tm : V(0);
  if (tm > (V)g.top) tm = (V)g.top;
  if (tm > b[v]) b[v] = tm;
}

// The values a choice pass reads: f, or the Bellman-Ford values.
template <typename V>
__device__ __forceinline__ const V* seed_values(const DevGame& g, const SeedBuf& sb) {
  return sb.fbf ? (const V*)sb.fbf : (const V*)g.f;
}

// sigma1 for every player-1 vertex over its out-edges into the forced
// subgraph, and the single edge of every player-0 vertex of out-degree 1.
// The player-1 rows of up to SEED_FLAT edges of a tile of BLOCK vertices are
// flattened as in the lift, so that consecutive lanes read consecutive edges
// whatever the degrees.  A candidate's rank is one 64-bit key, the negative
// self-loop flag above the term (terms stay below 2^63), larger first, and
// then the lower edge index.  Per chunk of the flattened range: the keys are
// folded into the row's LDS maximum; the lanes holding that maximum fold
// their indices into the row's LDS minimum; and the row's own thread keeps
// the chunk's index only when the chunk raised the maximum or the row had no
// candidate yet (an earlier chunk holds the lower indices of an equal key).
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_seed_choose(DevGame g, SeedBuf sb, int32_t* longs_out,
                                                       int32_t* mids_out, bool f_zero) {
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  constexpr int J = SEED_UNROLL;
  __shared__ uint32_t epre[BLOCK + 1];
  __shared__ uint32_t ebeg[BLOCK];
  __shared__ unsigned long long kmax[BLOCK];
  __shared__ uint32_t kidx[BLOCK];
  __shared__ uint32_t wsum[BLOCK / WAVE];
  const V* f = seed_values<V>(g, sb);
  const uint32_t n = (uint32_t)g.n, tid = threadIdx.x, lane = lane_id();
  const uint32_t ntiles = (n + BLOCK - 1) / BLOCK;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t v = t * BLOCK + tid;
    uint32_t e0 = 0, deg = 0;
    bool p1 = false;
    if (v < n) {
      const uint32_t a = g.rs[v];
      e0 = a & ROW_MASK;
      deg = (g.rs[v + 1] & ROW_MASK) - e0;
      p1 = (a & OWNER_BIT) != 0;
    }
    // longer rows: k_seed_choose_rows up to SEED_LONG edges, then
    // k_seed_choose_pieces (their choice stays "none" here and is written
    // there)
    wave_append(v < n && p1 && deg > SEED_LONG, (int32_t)v, longs_out, sb.count + 1);
    wave_append(v < n && p1 && deg > SEED_FLAT && deg <= SEED_LONG, (int32_t)v, mids_out, sb.count + 3);
    uint32_t E;
    const uint32_t ex = block_excl_scan(v < n && p1 && deg <= SEED_FLAT ? deg : 0u, wsum, &E);
    epre[tid] = ex;
    if (tid == BLOCK - 1) epre[BLOCK] = E;
    ebeg[tid] = e0;
    kmax[tid] = 0;
    kidx[tid] = NONE;
    uint32_t best = NONE;         // this thread's row: the chosen edge index
    unsigned long long prev = 0;  // and its maximum key before the chunk
    block_sync();
    for (uint32_t x0 = 0; x0 < E; x0 += J * BLOCK) {
      uint32_t slot[J], idx[J];
      int2 ed[J];
#pragma unroll
      for (int j = 0; j < J; j++) {
        const uint32_t x = x0 + j * BLOCK + tid;
        const uint32_t xc = x < E ? x : E - 1;
        const uint32_t sl = find_range(epre, xc);
        slot[j] = x < E ? sl : (uint32_t)BLOCK;
        idx[j] = xc - epre[sl];
        ed[j] = g.edges[ebeg[sl] + idx[j]];
      }
      uint8_t fz[J];
      V fu[J];
#pragma unroll
      for (int j = 0; j < J; j++) {
        fz[j] = sb.forced[ed[j].x];
        fu[j] = f_zero ? V(0) : f[ed[j].x];
      }
      unsigned long long key[J];
      bool cand[J];
#pragma unroll
      for (int j = 0; j < J; j++) {
        const uint32_t sl = slot[j];
        const bool loop = ed[j].x == (int32_t)(t * BLOCK + sl) && ed[j].y < 0;
        V tm = fu[j] - (V)ed[j].y;
        tm = tm > V(0) ? tm : V(0);
        cand[j] = sl < (uint32_t)BLOCK && fz[j] != 0;
        key[j] = ((unsigned long long)loop << 63) | (unsigned long long)(int64_t)tm;
        bool h = cand[j];
        unsigned long long k = key[j];
        wave_seg_fold(h, k, sl, [](unsigned long long a, unsigned long long b) { return a > b; });
        const uint32_t sprev = __shfl_up(sl, 1, WAVE);
        if (h && (lane == 0 || sprev != sl))
          __hip_atomic_fetch_max(&kmax[sl], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      block_sync();
      const unsigned long long km = kmax[tid];  // stable until the next chunk's first barrier
#pragma unroll
      for (int j = 0; j < J; j++) {
        const uint32_t sl = slot[j];
        bool h = cand[j] && key[j] == kmax[sl < (uint32_t)BLOCK ? sl : 0];
        uint32_t i = idx[j];
        wave_seg_fold(h, i, sl, [](uint32_t a, uint32_t b) { return a < b; });
        const uint32_t sprev = __shfl_up(sl, 1, WAVE);
        if (h && (lane == 0 || sprev != sl))
          __hip_atomic_fetch_min(&kidx[sl], i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      block_sync();
      const uint32_t ci = kidx[tid];
      if (ci != NONE) {
        if (best == NONE || km != prev) best = ci;
        kidx[tid] = NONE;  // read again only after the next chunk's first barrier
      }
      prev = km;
    }
    if (v < n) {
      if (!p1 && deg == 1) best = 0;
      int32_t to = -1, bw = 0;
      if (best != NONE) {
        const int2 ed = g.edges[e0 + best];
        to = ed.x;
        bw = ed.y;
      }
      sb.succ[v] = to;
      sb.wgt[v] = bw;
      sb.pl[0][v] = make_int2(to, (int32_t)v);
      sb.oncyc[v] = 0;
      sb.sum[v] = 0;
      seed_raise<V>(g, sb, (int32_t)v, to, bw);
    }
    // the next tile rewrites epre, ebeg, kmax and kidx only after its scan's
    // barrier, which every thread reaches after its last read of them here
  }
}

// sigma1 for the player-1 rows of SEED_FLAT + 1 to SEED_LONG edges listed by
// k_seed_choose: a wave per row, SEED_UNROLL * WAVE edges per step, the same
// candidate order.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_seed_choose_rows(DevGame g, SeedBuf sb, const int32_t* list,
                                                            const uint32_t* count, bool f_zero) {
  const V* f = seed_values<V>(g, sb);
  const uint32_t lane = lane_id();
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  const uint32_t cnt = *count;
  const uint32_t waves = gridDim.x * (BLOCK / WAVE);
  // the loop bound is uniform over the wave
  for (uint32_t i = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE; i < cnt; i += waves) {
    const int32_t v = list[i];
    const uint32_t e0 = g.rs[v] & ROW_MASK;
    const uint32_t d = (g.rs[v + 1] & ROW_MASK) - e0;
    bool l = false;
    V t = -1;
    uint32_t kk = NONE;
    for (uint32_t k0 = 0; k0 < d; k0 += SEED_UNROLL * WAVE) {
      int2 ed[SEED_UNROLL];
#pragma unroll
      for (int j = 0; j < SEED_UNROLL; j++) ed[j] = g.edges[e0 + min(k0 + j * WAVE + lane, d - 1)];
      uint8_t fz[SEED_UNROLL];
      V fu[SEED_UNROLL];
#pragma unroll
      for (int j = 0; j < SEED_UNROLL; j++) {
        fz[j] = sb.forced[ed[j].x];
        fu[j] = f_zero ? V(0) : f[ed[j].x];
      }
#pragma unroll
      for (int j = 0; j < SEED_UNROLL; j++) {
        const uint32_t k = k0 + j * WAVE + lane;
        if (k >= d || !fz[j]) continue;
        const bool lj = ed[j].x == v && ed[j].y < 0;
        V tm = fu[j] - (V)ed[j].y;
        tm = tm > V(0) ? tm : V(0);
        if (kk == NONE || seed_better<V>(lj, tm, k, l, t, kk)) {
          l = lj;
          t = tm;
          kk = k;
        }
      }
    }
    // the wave's best candidate (NONE loses to every candidate)
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const bool lo_ = __shfl_xor((int)l, o, WAVE) != 0;
      const V to = __shfl_xor(t, o, WAVE);
      const uint32_t ko = __shfl_xor(kk, o, WAVE);
      if (ko != NONE && (kk == NONE || seed_better<V>(lo_, to, ko, l, t, kk))) {
        l = lo_;
        t = to;
        kk = ko;
      }
    }
    if (lane == 0) {
      int32_t best = -1, bw = 0;
      if (kk != NONE) {
        const int2 ed = g.edges[e0 + kk];
        best = ed.x;
        bw = ed.y;
      }
      sb.succ[v] = best;
      sb.wgt[v] = bw;
      sb.pl[0][v].x = best;
      seed_raise<V>(g, sb, v, best, bw);
    }
  }
}

// sigma1 for the player-1 rows longer than SEED_LONG (few, but the largest
// would hold one block for its whole length): each row is cut into
// SEED_PIECES pieces, one block per piece, in two passes over the pieces
// and a closing one over the rows.  PHASE 0 folds each piece's best
// (negative self-loop, term) key into the row's 64-bit maximum (in the
// per-cycle sum array, zero until the doubling ends); PHASE 1 folds the
// lowest edge index among the candidates holding that maximum into the row's
// entry of succ (NONE from k_seed_choose); k_seed_choose_close turns the index
// into the chosen edge and clears the maximum.  The order is the same as in
// the other choice kernels.
constexpr uint32_t SEED_PIECES = 16;

template <typename V, int PHASE>
__global__ __launch_bounds__(BLOCK) void k_seed_choose_pieces(DevGame g, SeedBuf sb, const int32_t* list,
                                                              const uint32_t* count, bool f_zero) {
  __shared__ unsigned long long s_key[BLOCK / WAVE];
  __shared__ uint32_t s_has[BLOCK / WAVE];
  const V* f = seed_values<V>(g, sb);
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid / WAVE;
  const uint32_t total = *count * SEED_PIECES;
  for (uint32_t x = blockIdx.x; x < total; x += gridDim.x) {  // block-uniform
    const int32_t v = list[x / SEED_PIECES];
    const uint32_t j = x % SEED_PIECES;
    const uint32_t e0 = g.rs[v] & ROW_MASK, d = (g.rs[v + 1] & ROW_MASK) - e0;
    const uint32_t lo = (uint32_t)((uint64_t)d * j / SEED_PIECES), hi = (uint32_t)((uint64_t)d * (j + 1) / SEED_PIECES);
    const unsigned long long target = PHASE == 1 ? (unsigned long long)sb.sum[v] : 0ull;
    bool has = false;
    unsigned long long best = 0;  // PHASE 0: the largest key; PHASE 1: the lowest index holding the target
    for (uint32_t k0 = lo; k0 < hi; k0 += SEED_UNROLL * BLOCK) {
      int2 ed[SEED_UNROLL];
#pragma unroll
      for (int q = 0; q < SEED_UNROLL; q++) ed[q] = g.edges[e0 + min(k0 + q * BLOCK + tid, hi - 1)];
      uint8_t fz[SEED_UNROLL];
      V fu[SEED_UNROLL];
#pragma unroll
      for (int q = 0; q < SEED_UNROLL; q++) {
        fz[q] = sb.forced[ed[q].x];
        fu[q] = f_zero ? V(0) : f[ed[q].x];
      }
#pragma unroll
      for (int q = 0; q < SEED_UNROLL; q++) {
        const uint32_t k = k0 + q * BLOCK + tid;
        if (k >= hi || !fz[q]) continue;
        V tm = fu[q] - (V)ed[q].y;
        tm = tm > V(0) ? tm : V(0);
        const unsigned long long key =
            ((unsigned long long)(ed[q].x == v && ed[q].y < 0) << 63) | (unsigned long long)(int64_t)tm;
        if (PHASE == 0) {
          if (!has || key > best) best = key;
          has = true;
        } else if (key == target) {
          if (!has || k < best) best = k;
          has = true;
        }
      }
    }
    // the block's fold: largest key (PHASE 0) or lowest index (PHASE 1)
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const unsigned long long bo = __shfl_xor(best, o, WAVE);
      const bool ho = __shfl_xor((int)has, o, WAVE) != 0;
      if (ho && (!has || (PHASE == 0 ? bo > best : bo < best))) best = bo;
      has = has || ho;
    }
    if (lane == 0) {
      s_key[wid] = best;
      s_has[wid] = has;
    }
    block_sync();
    if (tid == 0) {
      for (int w = 1; w < BLOCK / WAVE; w++)
        if (s_has[w] && (!has || (PHASE == 0 ? s_key[w] > best : s_key[w] < best))) {
          best = s_key[w];
          has = true;
        }
      if (has) {
        if (PHASE == 0) atomicMax((unsigned long long*)&sb.sum[v], best);
        else atomicMin((uint32_t*)&sb.succ[v], (uint32_t)best);
      }
    }
    block_sync();  // the next piece rewrites s_key and s_has
  }
}

template <typename V>
__global__ void k_seed_choose_close(DevGame g, SeedBuf sb, const int32_t* list, const uint32_t* count) {
  const uint32_t cnt = *count;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const int32_t v = list[i];
    const uint32_t k = (uint32_t)sb.succ[v];
    int32_t to = -1, bw = 0;
    if (k != 0xFFFFFFFFu) {
      const int2 ed = g.edges[(g.rs[v] & ROW_MASK) + k];
      to = ed.x;
      bw = ed.y;
    }
    sb.succ[v] = to;
    sb.wgt[v] = bw;
    sb.pl[0][v].x = to;
    sb.sum[v] = 0;
    seed_raise<V>(g, sb, v, to, bw);
  }
}

// One doubling step on {pointer, smallest id} pairs (one gather per vertex).
__global__ void k_seed_jump(int32_t n, const int2* pl, int2* pl2) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int2 a = pl[v];
    if (a.x >= 0) {
      const int2 b = pl[a.x];
      pl2[v] = make_int2(b.x, min(a.y, b.y));
    } else {
      pl2[v] = a;
    }
  }
}

__global__ void k_seed_mark(int32_t n, const int2* pl, uint8_t* oncyc) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int32_t u = pl[v].x;
    if (u >= 0) oncyc[u] = 1;
  }
}

__global__ void k_seed_sum(int32_t n, const SeedBuf sb, const int2* pl) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (sb.oncyc[v]) atomicAdd((unsigned long long*)&sb.sum[pl[v].y], (unsigned long long)(long long)sb.wgt[v]);
}

// TOP on the vertices of negative cycles; their predecessors join L_r (flags).
// A short predecessor list is flagged by its lane, a long one by the whole wave.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_seed_apply(DevGame g, const SeedBuf sb, const int2* pl, uint32_t r,
                                                      int32_t* longs_out) {
  V* f = (V*)g.f;
  const V top = (V)g.top;
  uint8_t* act = (r & 1) ? g.act1 : g.act0;
  const uint32_t n = (uint32_t)g.n;
  const uint32_t lane = lane_id();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t mine = 0;
  for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x - lane; v0 < n; v0 += stride) {
    const uint32_t v = v0 + lane;
    bool set = false;
    uint32_t pb = 0, pe = 0;
    const bool proven = v < n && ((sb.oncyc[v] && sb.sum[pl[v].y] < 0) || (sb.fbf && ((const V*)sb.fbf)[v] > (V)g.bound));
    if (proven && f[v] != top) {
      f[v] = top;
      mine++;
      set = true;
      pb = g.rev_off[v];
      pe = g.rev_off[v + 1];
      if (pe - pb <= SEED_SHORT)
        for (uint32_t k = pb; k < pe; k++) act[g.rev_src[k]] = 1;
    }
    // lists longer than SEED_LONG: k_seed_apply_long
    wave_append(set && pe - pb > SEED_LONG, (int32_t)v, longs_out, sb.count + 2);
    unsigned long long longs = __ballot(set && pe - pb > SEED_SHORT && pe - pb <= SEED_LONG);
    while (longs) {
      const uint32_t src = (uint32_t)__ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const uint32_t b = __shfl(pb, (int)src, WAVE), e = __shfl(pe, (int)src, WAVE);
      for (uint32_t k = b + lane; k < e; k += WAVE) act[g.rev_src[k]] = 1;
    }
  }
  if (mine) atomicAdd(sb.count, mine);
}

// The predecessors of the TOP vertices listed by k_seed_apply join L_r: the
// grid splits into groups of gridDim / cnt blocks (at least one), and a group
// flags one list at a time, so that a few hubs with long lists are spread
// over the whole grid.
__global__ __launch_bounds__(BLOCK) void k_seed_apply_long(DevGame g, const SeedBuf sb, const int32_t* list,
                                                           uint32_t r) {
  uint8_t* act = (r & 1) ? g.act1 : g.act0;
  const uint32_t cnt = sb.count[2];
  if (cnt == 0) return;
  const uint32_t per = max(1u, gridDim.x / cnt);  // blocks per list
  const uint32_t groups = gridDim.x / per;
  const uint32_t grp = blockIdx.x / per, part = blockIdx.x % per;
  if (grp >= groups) return;
  for (uint32_t i = grp; i < cnt; i += groups) {
    const int32_t v = list[i];
    const uint32_t pb = g.rev_off[v], pe = g.rev_off[v + 1];
    for (uint32_t k = pb + part * BLOCK + threadIdx.x; k < pe; k += per * BLOCK) act[g.rev_src[k]] = 1;
  }
}

size_t seed_bytes(int32_t n) {
  const size_t nn = (size_t)n;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return 2 * up(4 * nn) + 3 * up(8 * nn) + 2 * up(nn) + up(16);
}

void bind_seed(SeedBuf& sb, void* base, int32_t n) {
  const size_t nn = (size_t)n;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* b = (char*)base;
  sb.succ = (int32_t*)b;
  b += up(4 * nn);
  sb.wgt = (int32_t*)b;
  b += up(4 * nn);
  for (auto& q : sb.pl) {
    q = (int2*)b;
    b += up(8 * nn);
  }
  sb.forced = (uint8_t*)b;
  b += up(nn);
  sb.oncyc = (uint8_t*)b;
  b += up(nn);
  sb.sum = (long long*)b;
  b += up(8 * nn);
  sb.count = (uint32_t*)b;
  sb.fbf = nullptr;  // one choice pass unless the caller supplies the values of Bellman-Ford passes
}

// One seeding pass before round r; sb.count receives the number of vertices
// set to TOP.  When it is nonzero the caller runs round r as a dense round
// (ctrl[C_ANY0 + (r - 1) % 3] is set here).  With passes > 1 (sb.fbf set) the
// choice runs that many times as Bellman-Ford passes over the forced
// subgraph from f, each on the values the last one raised, and the cycles
// are read off the last choice.
template <typename V>
static void launch_choice(const DevGame& g, const SeedBuf& sb, int32_t* longs, int32_t* mids, bool f_zero, int grid,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_seed_choose<V>, dim3(grid), dim3(BLOCK), 0, s, g, sb, longs, mids, f_zero);
  hipLaunchKernelGGL(k_seed_choose_rows<V>, dim3(SEED_MID_GRID), dim3(BLOCK), 0, s, g, sb, (const int32_t*)mids,
                     (const uint32_t*)sb.count + 3, f_zero);
  hipLaunchKernelGGL((k_seed_choose_pieces<V, 0>), dim3(SEED_LONG_GRID), dim3(BLOCK), 0, s, g, sb,
                     (const int32_t*)longs, (const uint32_t*)sb.count + 1, f_zero);
  hipLaunchKernelGGL((k_seed_choose_pieces<V, 1>), dim3(SEED_LONG_GRID), dim3(BLOCK), 0, s, g, sb,
                     (const int32_t*)longs, (const uint32_t*)sb.count + 1, f_zero);
  hipLaunchKernelGGL(k_seed_choose_close<V>, dim3(SEED_LONG_GRID / 4), dim3(BLOCK), 0, s, g, sb,
                     (const int32_t*)longs, (const uint32_t*)sb.count + 1);
}

hipError_t launch_seed(const DevGame& g, int vbits, const SeedBuf& sb, uint32_t r, bool f_zero, int passes,
                       hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + BLOCK - 1) / BLOCK, 8192));
  if (!sb.fbf) passes = 1;
  hipError_t e = hipSuccess;
  if (sb.fbf) e = hipMemcpyAsync(sb.fbf, g.f, (size_t)g.n * (size_t)(vbits / 8), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seed_forced, dim3(grid), dim3(BLOCK), 0, s, g, sb);
  // the long-row list and the medium-row list live in the two halves of
  // pl[1] until the first doubling pass writes it
  int32_t* longs = (int32_t*)sb.pl[1];
  int32_t* mids = longs + g.n;
  for (int p = 0; p < passes; p++) {
    // count[0]: vertices set to TOP; count[1], count[2]: long rows and long
    // predecessor lists handed to the block-per-piece and group kernels,
    // count[3]: rows handed to the wave-per-row kernel
    e = hipMemsetAsync(sb.count, 0, 16, s);
    if (e != hipSuccess) return e;
    if (vbits == 32) launch_choice<int32_t>(g, sb, longs, mids, f_zero && p == 0, grid, s);
    else launch_choice<int64_t>(g, sb, longs, mids, f_zero && p == 0, grid, s);
  }
  int cur = 0;
  for (int64_t span = 1; span <= 2 * (int64_t)g.n; span *= 2, cur ^= 1)
    hipLaunchKernelGGL(k_seed_jump, dim3(grid), dim3(BLOCK), 0, s, g.n, (const int2*)sb.pl[cur], sb.pl[cur ^ 1]);
  hipLaunchKernelGGL(k_seed_mark, dim3(grid), dim3(BLOCK), 0, s, g.n, (const int2*)sb.pl[cur], sb.oncyc);
  hipLaunchKernelGGL(k_seed_sum, dim3(grid), dim3(BLOCK), 0, s, g.n, sb, (const int2*)sb.pl[cur]);
  // the long-list list lives in pl[cur ^ 1], free after the last doubling pass
  int32_t* lists = (int32_t*)sb.pl[cur ^ 1];
  if (vbits == 32)
    hipLaunchKernelGGL(k_seed_apply<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, sb, (const int2*)sb.pl[cur], r,
                       lists);
  else
    hipLaunchKernelGGL(k_seed_apply<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, sb, (const int2*)sb.pl[cur], r,
                       lists);
  hipLaunchKernelGGL(k_seed_apply_long, dim3(SEED_LONG_GRID), dim3(BLOCK), 0, s, g, sb, (const int32_t*)lists, r);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemsetAsync(g.ctrl + C_ANY0 + (r + 2) % 3, 0xFF, 1, s);
}

// ---------------------------------------------------------------- batched games
//
// Many games share one launch per round.  The slot table holds one DevGame
// per resident game and the round each game runs next, independently of the
// others.  Each epoch is two launches: k_plan (one block) retires the games
// whose previous round raised nothing, sends games whose next active set is
// small to k_batch_small, and lays out the tasks of the epoch, one per tile
// of every other running game (dense representation); k_batch_round (a fixed
// grid) takes tasks in turn.

__global__ __launch_bounds__(1024) void k_plan(BatchTable bt) {
  __shared__ uint32_t wsum[1024 / WAVE];
  __shared__ uint32_t carry;
  const uint32_t tid = threadIdx.x;
  const uint32_t epoch = bt.ctl[B_EPOCH] + 1;
  if (tid == 0) carry = 0;
  block_sync();
  for (uint32_t base = 0; base < bt.nslots; base += 1024) {
    const uint32_t s = base + tid;
    uint32_t tasks = 0;
    // k_batch_small runs beside this kernel on another stream and hands a slot
    // back by a release store of BM_DENSE after writing the slot's round and
    // control words; the acquire load orders the reads of those words below
    // after it (a relaxed load could see the mode and then stale words).
    if (s < bt.nslots && bt.state[s] == SLOT_RUN &&
        __hip_atomic_load(&bt.mode[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == BM_DENSE) {
      const uint32_t r = bt.round[s];
      const DevGame& g = bt.games[s];
      if (g.ctrl[C_ANY0 + (r - 1) % 3] == 0) {  // round r-1 raised nothing: L_r is empty
        bt.rounds[s] = r - 1;
        bt.state[s] = SLOT_DONE;
      } else if (r > 1 && g.ctrl[C_CNT0 + r % 3] <= bt.small_limit) {
        // at most small_limit predecessor entries were activated for L_r:
        // the game continues in k_batch_small
        __hip_atomic_store(&bt.mode[s], BM_SMALL_NEW, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        g.ctrl[C_ANY0 + (r + 1) % 3] = 0;  // written by round r+1
        g.ctrl[C_CNT0 + (r + 1) % 3] = 0;  // summed by round r: entries activated for L_{r+1}
        bt.cur[s] = r;
        bt.round[s] = r + 1;
        tasks = ((uint32_t)g.n + TILE - 1) / TILE;
      }
    }
    // exclusive scan of tasks over the 1024 slots of this chunk
    const uint32_t lane = lane_id(), wid = tid / WAVE;
    uint32_t incl = tasks;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, WAVE);
      if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == WAVE - 1) wsum[wid] = incl;
    block_sync();
    uint32_t off = carry, tot = 0;
    for (int w = 0; w < 1024 / WAVE; w++) {
      off += (uint32_t)w < wid ? wsum[w] : 0u;
      tot += wsum[w];
    }
    if (s < bt.nslots) bt.task_begin[s] = off + incl - tasks;
    block_sync();
    if (tid == 0) carry += tot;
    block_sync();
  }
  if (tid == 0) {
    bt.task_begin[bt.nslots] = carry;
    bt.ctl[B_TASKS] = carry;
    bt.ctl[B_EPOCH] = epoch;
  }
}

// slot whose task range holds task x (task_begin[0] = 0 <= x < task_begin[nslots])
__device__ __forceinline__ uint32_t find_slot(const uint32_t* begin, uint32_t nslots, uint32_t x) {
  uint32_t lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (begin[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename V>
__device__ __forceinline__ void batch_task(const BatchTable& bt, RoundShared<V>& sh, uint32_t s, uint32_t t) {
  const DevGame& g = bt.games[s];
  const uint32_t r = bt.cur[s];
  if (threadIdx.x < S_WORDS) sh.st[threadIdx.x] = 0;
  Counters c;
  round_tile<V, true>(g, sh, r, t, (uint32_t)g.n, c);
  block_sync();
  block_counters(sh, c);
  if (threadIdx.x < S_WORDS && sh.st[threadIdx.x]) atomicAdd(&bt.st[s * S_WORDS + threadIdx.x], sh.st[threadIdx.x]);
  if (threadIdx.x == 0) {
    if (sh.st[S_CHANGES]) g.ctrl[C_ANY0 + r % 3] = 1;
    if (sh.st[S_SCANNED])
      atomicAdd(&g.ctrl[C_CNT0 + (r + 1) % 3], (uint32_t)std::min<unsigned long long>(sh.st[S_SCANNED], 1u << 30));
  }
}

// LDS of a block that runs games of either value width.
union RoundSharedAny {
  RoundShared<int32_t> v32;
  RoundShared<int64_t> v64;
};

__global__ __launch_bounds__(BLOCK) void k_batch_round(BatchTable bt) {
  __shared__ RoundSharedAny sh;
  const uint32_t ntasks = bt.ctl[B_TASKS];
  for (uint32_t x = blockIdx.x; x < ntasks; x += gridDim.x) {
    block_sync();
    const uint32_t s = find_slot(bt.task_begin, bt.nslots, x);
    const uint32_t t = x - bt.task_begin[s];
    // the width the game was laid out with (the rule every launcher follows)
    if (bt.games[s].vbits == 32)
      batch_task<int32_t>(bt, sh.v32, s, t);
    else
      batch_task<int64_t>(bt, sh.v64, s, t);
  }
}

// Games of the batch whose active set is small run here, one block per game
// and many rounds per launch, on a stream of their own beside the epochs of
// the others (a slot is either in the epochs or here, by its mode word).
// A slot that enters from the epochs first turns its round's flags into a
// list.  Afterwards the slot is finished (empty list), handed back to the
// epochs (list longer than small_limit) or kept here.
template <typename V>
__device__ void batch_small_slot(const BatchTable& bt, RoundShared<V>& sh, uint32_t s, uint32_t mode,
                                 uint32_t max_rounds, uint64_t deadline, uint32_t& s_items, int& s_changed) {
  const DevGame& g = bt.games[s];
  const uint32_t tid = threadIdx.x;
  const uint32_t n = (uint32_t)g.n;
  uint32_t r = bt.round[s];
  if (mode == BM_SMALL_NEW) {
    if (tid == 0) s_items = 0;
    block_sync();
    const uint8_t* act = (r & 1) ? g.act1 : g.act0;
    int32_t* wl = (r & 1) ? g.wl1 : g.wl0;
    for (uint32_t v0 = 0; v0 < n; v0 += BLOCK) {
      const uint32_t v = v0 + tid;
      wave_append(v < n && act[v] != 0, (int32_t)v, wl, &s_items);
    }
    block_sync();
    if (tid == 0) {
      g.ctrl[C_CNT0 + r % 3] = s_items;
      g.ctrl[C_CNT0 + (r + 1) % 3] = 0;
      g.ctrl[C_CNT0 + (r + 2) % 3] = 0;
    }
  }
  if (tid < S_WORDS) sh.st[tid] = 0;
  Counters c;
  r = small_rounds<V>(g, sh, r, max_rounds, bt.small_limit, s_items, s_changed, c, deadline);
  block_counters(sh, c);
  if (tid < S_WORDS && sh.st[tid]) atomicAdd(&bt.st[s * S_WORDS + tid], sh.st[tid]);
  if (tid == 0) {
    const uint32_t items = g.ctrl[C_CNT0 + r % 3];
    bt.round[s] = r;
    if (items == 0) bt.rounds[s] = r - 1;
    if (items == 0)
      __hip_atomic_store(&bt.state[s], SLOT_DONE, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_store(&bt.mode[s], items > bt.small_limit ? BM_DENSE : BM_SMALL, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

// budget_ticks (nonzero): each slot's rounds stop once this many ticks of the
// realtime counter have passed since the block started.
__global__ __launch_bounds__(BLOCK) void k_batch_small(BatchTable bt, uint32_t max_rounds, uint64_t budget_ticks) {
  __shared__ RoundSharedAny sh;
  __shared__ uint32_t s_items, s_mode;
  __shared__ int s_changed;
  const uint64_t deadline = budget_ticks ? __builtin_amdgcn_s_memrealtime() + budget_ticks : 0;
  for (uint32_t s = blockIdx.x; s < bt.nslots; s += gridDim.x) {
    block_sync();
    if (threadIdx.x == 0) {
      s_mode = bt.state[s] == SLOT_RUN ? __hip_atomic_load(&bt.mode[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                       : (uint32_t)BM_DENSE;
      // the slot's game data was released by k_plan or by a previous launch
      // of this kernel; acquire it only for the slots this block runs
      if (s_mode != BM_DENSE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    block_sync();
    if (s_mode == BM_DENSE) continue;
    if (bt.games[s].vbits == 32)
      batch_small_slot<int32_t>(bt, sh.v32, s, s_mode, max_rounds, deadline, s_items, s_changed);
    else
      batch_small_slot<int64_t>(bt, sh.v64, s, s_mode, max_rounds, deadline, s_items, s_changed);
  }
}

hipError_t launch_epoch(const BatchTable& bt, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, bt);
  hipLaunchKernelGGL(k_batch_round, dim3(grid), dim3(BLOCK), 0, s, bt);
  return hipGetLastError();
}

hipError_t launch_batch_small(const BatchTable& bt, uint32_t max_rounds, uint64_t budget_ticks, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_small, dim3(bt.nslots), dim3(BLOCK), 0, s, bt, max_rounds, budget_ticks);
  return hipGetLastError();
}

// stats[k] = sum over blocks of slots[b][k]
__global__ void k_reduce_slots(DevGame g, uint32_t nblocks) {
  __shared__ unsigned long long acc[S_WORDS];
  if (threadIdx.x < S_WORDS) acc[threadIdx.x] = 0;
  block_sync();
  for (uint32_t b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int k = 0; k < S_WORDS; k++) atomicAdd(&acc[k], g.slots[b * S_WORDS + k]);
  block_sync();
  if (threadIdx.x < S_WORDS) g.stats[threadIdx.x] = acc[threadIdx.x];
}

template <typename V>
__global__ void k_output(DevGame g, int64_t* out) {
  const V* f = (const V*)g.f;
  const V top = (V)g.top;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const V x = f[g.perm ? (uint32_t)g.perm[v] : v];
    out[v] = x == top ? INT64_MAX : (int64_t)x;
  }
}

template <typename V>
__global__ void k_input(DevGame g, const int64_t* in) {
  V* f = (V*)g.f;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)g.n; v += gridDim.x * blockDim.x) {
    const int64_t x = in[v];
    f[g.perm ? (uint32_t)g.perm[v] : v] = x == INT64_MAX ? (V)g.top : (V)x;
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

static int vertex_grid(const DevGame& g, int max_grid) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + TILE - 1) / TILE, max_grid));
}

hipError_t launch_init(const DevGame& g, int vbits, int resume, int grid, hipStream_t s) {
  if (vbits == 32) hipLaunchKernelGGL(k_init<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, resume);
  else hipLaunchKernelGGL(k_init<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, resume);
  return hipGetLastError();
}

hipError_t launch_activate_changed(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s) {
  if (vbits == 32) hipLaunchKernelGGL(k_activate_changed<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  else hipLaunchKernelGGL(k_activate_changed<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  return hipGetLastError();
}

hipError_t launch_compact(const DevGame& g, uint32_t r, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(grid), dim3(BLOCK), 0, s, g, r);
  return hipGetLastError();
}

hipError_t launch_round(const DevGame& g, int vbits, int h, bool dense, uint32_t r, int grid, hipStream_t s) {
  (void)h;
  if (vbits == 32) {
    if (dense) hipLaunchKernelGGL((k_round<int32_t, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
    else hipLaunchKernelGGL((k_round<int32_t, false>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  } else {
    if (dense) hipLaunchKernelGGL((k_round<int64_t, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
    else hipLaunchKernelGGL((k_round<int64_t, false>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  }
  return hipGetLastError();
}

hipError_t launch_round_seg(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s, bool all) {
  const size_t hub_bytes = (size_t)g.hub_n * (size_t)(vbits / 8);
  if (vbits == 32) {
    if (all) hipLaunchKernelGGL((k_round_seg<int32_t, true>), dim3(grid), dim3(BLOCK), hub_bytes, s, g, r);
    else hipLaunchKernelGGL((k_round_seg<int32_t, false>), dim3(grid), dim3(BLOCK), hub_bytes, s, g, r);
  } else {
    if (all) hipLaunchKernelGGL((k_round_seg<int64_t, true>), dim3(grid), dim3(BLOCK), hub_bytes, s, g, r);
    else hipLaunchKernelGGL((k_round_seg<int64_t, false>), dim3(grid), dim3(BLOCK), hub_bytes, s, g, r);
  }
  return hipGetLastError();
}

hipError_t launch_round_all(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s) {
  if (vbits == 32) hipLaunchKernelGGL((k_round<int32_t, true, false, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  else hipLaunchKernelGGL((k_round<int64_t, true, false, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  return hipGetLastError();
}

hipError_t launch_gkey_init(const DevGame& g, int vbits, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + BLOCK - 1) / BLOCK, 8192));
  if (vbits == 32) hipLaunchKernelGGL(k_gkey_init<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g);
  else hipLaunchKernelGGL(k_gkey_init<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_partial(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s) {
  if (vbits == 32) hipLaunchKernelGGL(k_partial<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  else hipLaunchKernelGGL(k_partial<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  return hipGetLastError();
}

hipError_t launch_round_parts(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s, bool all) {
  if (vbits == 32) {
    if (all) hipLaunchKernelGGL((k_round<int32_t, true, true, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
    else hipLaunchKernelGGL((k_round<int32_t, true, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  } else {
    if (all) hipLaunchKernelGGL((k_round<int64_t, true, true, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
    else hipLaunchKernelGGL((k_round<int64_t, true, true>), dim3(grid), dim3(BLOCK), 0, s, g, r);
  }
  return hipGetLastError();
}

hipError_t launch_sliced(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s) {
  if (vbits == 32) hipLaunchKernelGGL(k_sliced<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  else hipLaunchKernelGGL(k_sliced<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, r);
  return hipGetLastError();
}

hipError_t launch_fill_max(void* p, int32_t n, int vbits, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n + BLOCK - 1) / BLOCK, 8192));
  if (vbits == 32) hipLaunchKernelGGL(k_fill_max<int32_t>, dim3(grid), dim3(BLOCK), 0, s, (int32_t*)p, n);
  else hipLaunchKernelGGL(k_fill_max<int64_t>, dim3(grid), dim3(BLOCK), 0, s, (int64_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_reduce_stats(const DevGame& g, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_slots, dim3(1), dim3(1024), 0, s, g, (uint32_t)nblocks);
  return hipGetLastError();
}

hipError_t launch_output(const DevGame& g, int vbits, int64_t* out, hipStream_t s) {
  const int grid = vertex_grid(g, 8192);
  if (vbits == 32) hipLaunchKernelGGL(k_output<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, out);
  else hipLaunchKernelGGL(k_output<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, out);
  return hipGetLastError();
}

hipError_t launch_input(const DevGame& g, int vbits, const int64_t* in, hipStream_t s) {
  const int grid = vertex_grid(g, 8192);
  if (vbits == 32) hipLaunchKernelGGL(k_input<int32_t>, dim3(grid), dim3(BLOCK), 0, s, g, in);
  else hipLaunchKernelGGL(k_input<int64_t>, dim3(grid), dim3(BLOCK), 0, s, g, in);
  return hipGetLastError();
}

}  // namespace eg
