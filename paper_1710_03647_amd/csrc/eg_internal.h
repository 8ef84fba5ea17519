// Internal declarations of libeg: device layout of a game and the kernel
// launchers used by the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "eg.h"

namespace eg {

// Row starts are uint32 (m < 2^31); bit 31 of rs[v] carries the owner of v
// (1 = player 1, the max player), so one load yields both.
constexpr uint32_t OWNER_BIT = 0x80000000u;
constexpr uint32_t ROW_MASK = 0x7FFFFFFFu;

// ctrl[] words (uint32) in device memory
enum Ctrl : int {
  C_CNT0 = 0,    // C_CNT0 + (r % 3): length of the active list of round r (sparse rounds)
  C_ANY0 = 3,    // C_ANY0 + (r % 3): nonzero if some value rose in round r (round 0 = init)
  C_ROUNDS = 6,  // rounds with a non-empty active set
  C_NEXT = 7,    // single-block driver: the round to run next
  C_WORDS = 8
};
// counters per block (slots) and totals (stats), uint64
// S_FILTERED: predecessor entries the player-1 frontier filter left out
enum Stat : int { S_LIFTS = 0, S_EDGES = 1, S_PUSHES = 2, S_CHANGES = 3, S_SCANNED = 4, S_FILTERED = 5, S_WORDS = 6 };

// Everything a kernel needs to see of one game (passed by value).
struct DevGame {
  int32_t n;
  uint32_t m;
  const uint32_t* rs;       // n+1 row starts | owner bit
  const int2* edges;        // m {target, weight}
  const uint32_t* rev_off;  // n+1 predecessor-list starts (the paper's CSC)
  const int32_t* rev_src;   // m predecessor ids, one per edge
  void* f;                  // n values, int32 or int64 (vbits)
  uint8_t* act0;            // n (padded to 4): flags of the active set of even rounds
  uint8_t* act1;            // n (padded to 4): flags of the active set of odd rounds
  int32_t* wl0;             // n: active list of even rounds
  int32_t* wl1;             // n: active list of odd rounds
  const uint32_t* act_bits; // ceil(n/32): initially active vertices (Alg. 3 line 3)
  uint32_t* ctrl;           // C_WORDS
  uint32_t* blk_chg;        // per block: values raised in its last round (init: vertices activated)
  unsigned long long* slots;  // per block: S_WORDS counters accumulated over the solve
  unsigned long long* stats;  // S_WORDS totals
  int64_t bound;            // B
  int64_t top;              // device encoding of TOP: B + P + 1, P = largest stored weight
  int32_t vbits;            // 32 or 64: width of f
  // target-partitioned copy of the edges for dense rounds (nparts > 1)
  uint32_t nparts;          // slices of the vertex range (1 = no partitioned copy)
  uint32_t part_size;       // vertices per slice
  const int2* pedges;       // m: {target | tile-local source << 22, weight}, grouped by (tile, slice)
  const uint32_t* poff;     // nchunks + 1: chunk (tile * nparts + slice) starts
  const uint32_t* own_bits; // ceil(n/32): owner bits (1 = player 1)
  void* part;               // nparts * n keys of width vbits (per-slice partial keys); slice-major
                            // rounds: n keys (combined over the slices, reset by the round)
  // slice-major dense rounds (partition mode 3): each block of k_sliced owns
  // the work items sl_items[sl_begin[b] .. sl_begin[b+1]) and sweeps the slices
  // in order for them, holding their keys in LDS (nullptr: not used)
  uint32_t slice_major;
  const uint2* sl_items;    // {tile of PTILE sources, part << 16 | parts}: a tile or one part of a cut tile
  const uint32_t* sl_begin; // grid + 1: each block's first item
  // edge-balanced dense rounds: a tile whose out-degree sum exceeds SEG_EDGES
  // is cut into segments taken by different blocks (nitems = 0: not used)
  uint32_t nitems;          // work items of a dense round: one per segment
  const uint32_t* item_tile; // nitems: tile of the item
  const uint32_t* item_seg;  // nitems: segment of the tile
  const uint32_t* tile_nseg; // ntiles: segments of the tile
  uint32_t* tile_done;      // ntiles: segments of the tile finished in this round
  void* gkey;               // n keys (width vbits) combined over the segments of cut tiles
  const int32_t* perm;      // n: internal id of each caller vertex (nullptr: ids are the caller's)
  uint32_t lanes_ok;        // small-degree tiles may use one lane per vertex (game fits the caches)
  // player-1 frontier filter (Alg. 1's predecessor test, player-1 predecessors):
  // a player-1 predecessor p of a changed v joins the next active set only if
  // f(p) < f(v) (-) w(p, v); nullptr: every predecessor joins (Alg. 3)
  const int32_t* rev_w;     // m: weight of the edge of each predecessor entry (stored, clamped)
  // component schedule: only predecessors on level cur_level join the next
  // active set (nullptr: no level filter)
  const int32_t* level;     // n: level of each vertex's component in the condensation
  int32_t cur_level;
  // cut-tile rounds (k_round_seg) read f(0 .. hub_n) from a copy in LDS taken
  // at the start of the round (0: off); set for games renumbered by in-degree
  uint32_t hub_n;
};

// A game whose edges and values fit in this many bytes may lift small-degree
// tiles with one lane per vertex.
constexpr size_t LANES_BYTES = (size_t)64 << 20;
inline uint32_t lanes_ok_for(int32_t n, int64_t m, int vbits) {
  return (size_t)m * 8 + (size_t)n * (size_t)(vbits / 8) <= LANES_BYTES ? 1u : 0u;
}

constexpr uint32_t SEG_EDGES = 8192;    // out-edges per segment of a cut tile (full frontier)

constexpr uint32_t PTILE = 1024;        // vertices per tile of the partitioned copy
constexpr uint32_t PTILE_SHIFT = 22;    // tile-local source index sits above the 22 target bits
constexpr uint32_t SL_SLOTS = 4;        // slice-major rounds: tiles whose keys a block holds in LDS at once
constexpr int SL_BLOCKS_PER_CU = 4;     // resident blocks of k_sliced per compute unit
constexpr uint32_t SL_SLICE_BYTES = 1u << 20;  // f bytes per target slice (a few slices fit one XCD's L2)
constexpr uint32_t HUB_BYTES = 16u << 10;       // default LDS copy of the most gathered values (cut-tile rounds)

// Scratch of one TOP-seeding pass (device arrays of n entries unless noted).
struct SeedBuf {
  int32_t* succ;      // chosen successor in the forced subgraph, -1 if none
  int32_t* wgt;       // weight of that edge
  int2* pl[2];        // pointer doubling (double buffered): {successor 2^k steps on, smallest vertex id
                      // on the walk so far}
  uint8_t* forced;    // 1 for player-1 vertices and for player-0 vertices of out-degree 1
  uint8_t* oncyc;     // 1 for vertices on a cycle of the chosen edges
  long long* sum;     // per cycle (indexed by its smallest vertex): total weight
  void* fbf;          // Bellman-Ford seeding passes: n values of the game's width (nullptr: one choice pass)
  uint32_t* count;    // 4 words: [0] vertices newly set to TOP, [1] long rows, [2] long predecessor
                      // lists, [3] medium rows
};
// Strongly connected components and condensation levels (component schedule).
struct SccBuf {
  int32_t* comp;       // n: component label (a vertex id of the component); -1 while unassigned
  int32_t* lev;        // n: level of the vertex's component (0 = sink components)
  int32_t* color;      // n: colouring of a phase
  uint8_t* mark;       // n: reached from the root in a phase
  uint32_t* flag;      // change counter of a sweep
  int32_t* max_level;  // next word: the largest level
  int32_t* long_in;    // n: vertices with more than SCC_LONG predecessor entries (taken a block each)
  int32_t* long_out;   // n: vertices with more than SCC_LONG out-edges
  uint32_t* nlong;     // 2 words: the lengths of long_in and long_out
};
struct SccInfo {
  uint32_t components, levels;
  uint64_t sweeps, phases;
};
size_t scc_bytes(int32_t n);
void bind_scc(SccBuf& sc, void* base, int32_t n);
// h_word: pinned host memory of two words.  Synchronises s.
hipError_t compute_scc(const DevGame& g, const SccBuf& sc, uint32_t* h_word, hipStream_t s, SccInfo* info);
// comp_out[v], lev_out[v] for caller vertex v (labels are internal vertex ids)
hipError_t launch_scc_output(const DevGame& g, const SccBuf& sc, int32_t* comp_out, int32_t* lev_out, hipStream_t s);
// L_r := the vertices of `level` (flags of round parity r), per-block counts in blk_chg
hipError_t launch_level_activate(const DevGame& g, const int32_t* lev, int32_t level, uint32_t r, int grid,
                                 hipStream_t s);
size_t seed_bytes(int32_t n);
void bind_seed(SeedBuf& sb, void* base, int32_t n);
// f_zero: f is 0 everywhere (the pass before the first round of a solve that
// does not resume), so the choice reads no values.
// passes > 1 (with sb.fbf set): that many Bellman-Ford passes over the forced
// subgraph before the cycles are read off the last choice.
hipError_t launch_seed(const DevGame& g, int vbits, const SeedBuf& sb, uint32_t r, bool f_zero, int passes,
                       hipStream_t s);

// Slot states of the batched iteration, and where a running slot's rounds run:
// in the epochs (flag sweeps, one round per epoch) or in k_batch_small (lists,
// many rounds per launch; SMALL_NEW until its flags have become a list).
constexpr uint32_t SLOT_FREE = 0, SLOT_RUN = 1, SLOT_DONE = 2;
constexpr uint32_t BM_DENSE = 0, BM_SMALL_NEW = 1, BM_SMALL = 2;

// Slot table of the batched iteration (device pointers, passed by value).
enum BatchCtl : int { B_EPOCH = 0, B_TASKS = 1, B_WORDS = 4 };
struct BatchTable {
  const DevGame* games;       // nslots descriptors
  uint32_t* state;            // SLOT_FREE / SLOT_RUN / SLOT_DONE
  uint32_t* mode;             // BM_DENSE / BM_SMALL_NEW / BM_SMALL
  uint32_t* round;            // next round of each running game
  uint32_t* cur;              // round a slot in the epochs runs in the current epoch
  uint32_t* rounds;           // rounds run, written when the game finishes
  uint32_t* task_begin;       // nslots + 1: first task of each slot in the current epoch
  unsigned long long* st;     // nslots * S_WORDS counters
  uint32_t* ctl;              // B_WORDS
  uint32_t nslots;
  uint32_t small_limit;       // lists up to this length run in k_batch_small
};

// Device layout of one game: every array in one allocation.
enum LayoutPart : int {
  L_RS, L_EDGES, L_ROFF, L_RSRC, L_F, L_ACT, L_WL0, L_WL1, L_OUT, L_CTRL, L_STATS, L_ACTBITS, L_BLK, L_SLOTS,
  L_PEDGES, L_POFF, L_OWNB, L_PART, L_RW, L_N
};
struct GameLayout {
  size_t off[L_N];
  size_t total;
};
// filter: room for the reverse weights of the player-1 frontier filter
// slice_major: part holds one key array instead of one per slice
GameLayout plan_layout(int32_t n, int64_t m, int vbits, size_t nblocks, uint32_t nparts = 1, bool filter = false,
                       bool slice_major = false);
void bind_layout(DevGame& dg, char* base, const GameLayout& L, int32_t n, int64_t m, int vbits,
                 uint32_t nparts = 1, bool filter = false);
// slices of the target-partitioned edge copy for eg_config.partition (1 = none)
uint32_t choose_parts(int32_t n, int64_t m, int vbits, int mode);
hipError_t launch_partition(const DevGame& dg, const uint8_t* owner_bits, uint32_t* cursor, uint32_t* scan_tmp,
                            size_t scan_words, hipStream_t s);
size_t partition_scratch_words(int32_t n, uint32_t nparts);
hipError_t launch_partial(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s);
hipError_t launch_round_parts(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s, bool all = false);
// slice-major rounds: k_sliced on its own grid (the one sl_begin was built for)
hipError_t launch_sliced(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s);
hipError_t launch_fill_max(void* p, int32_t n, int vbits, hipStream_t s);

// Host-side preparation of a validated game.
struct HostPrep {
  eg_game_info info;
  int64_t clamp;                   // largest stored weight P
  std::vector<uint32_t> act_bits;  // initially active vertices
  std::vector<uint32_t> tile_nseg; // segments per tile of TILE_VERTICES vertices (empty: no tile is cut)
  // vertices renumbered by decreasing in-degree (perm empty: not renumbered)
  std::vector<int32_t> perm;       // caller id -> internal id
  std::vector<int64_t> r_off;      // the game in internal ids
  std::vector<int32_t> r_tgt, r_w;
  std::vector<uint8_t> r_own;
};
int check_host(const eg_game_desc* d, int bound_mode, eg_game_info* info, std::string* why,
               int64_t* clamp_out, std::vector<uint32_t>* act_bits);
// Host copy of a game given by device pointers.
struct HostCopy {
  std::vector<int64_t> off;
  std::vector<int32_t> tgt, w;
  std::vector<uint8_t> own;
};
// hd = desc for host descriptors; for device descriptors the arrays are copied
// into hc on stream s (synchronised) and hd points at them.  EG_OK, EG_EINVAL
// or EG_EDEVICE (message in the thread's error).
int host_view(const eg_game_desc* desc, hipStream_t s, HostCopy& hc, eg_game_desc& hd);
// H2D copy (host descriptor) or device-to-device use (device descriptor), layout,
// initial-activity flags and predecessor lists into a bound DevGame, on stream s.
// staging: scratch of staging_bytes(n, m, host, weights) bytes, free once s has
// completed (weights: room for the reverse weights' build).
size_t staging_bytes(int32_t n, int64_t m, bool host_inputs, bool weights);
hipError_t upload_game(const eg_game_desc* d, const HostPrep& prep, DevGame& dg, void* staging, hipStream_t s,
                       hipEvent_t after_layout, hipEvent_t after_rcsr = nullptr);
hipError_t launch_epoch(const BatchTable& bt, int grid, hipStream_t s);
// budget_ticks: 0, or a time budget per slot in ticks of the 100 MHz realtime counter
hipError_t launch_batch_small(const BatchTable& bt, uint32_t max_rounds, uint64_t budget_ticks, hipStream_t s);
hipError_t launch_round_seg(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s, bool all);
hipError_t launch_round_all(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s);
hipError_t launch_gkey_init(const DevGame& g, int vbits, hipStream_t s);

// Layout and predecessor lists (eg_kernels.hip)
hipError_t launch_layout(const int64_t* off, const uint8_t* owner_bits, const int32_t* tgt,
                         const int32_t* w, int32_t n, uint32_t m, int32_t wclamp, uint32_t* rs,
                         int2* edges, hipStream_t s);
// Scratch of the reverse-CSR build, free once its stream has completed: the
// entries grouped by bucket of targets and the bucket counters.
constexpr uint32_t RB_BUCKETS = 4096;  // buckets of targets (at most)
struct RcsrScratch {
  int2* ent;       // m: {source, target} per edge, grouped by bucket
  int32_t* entw;   // m: their weights (needed only when rev_w is built)
  uint32_t* bcnt;  // RB_BUCKETS + 1: bucket totals, then their exclusive scan
  uint32_t* bcur;  // RB_BUCKETS: write cursors of the buckets
};
// rev_w (nullable): also the weight of each predecessor entry's edge
hipError_t launch_reverse_csr(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                              uint32_t* rev_off, int32_t* rev_src, int32_t* rev_w, uint32_t* cursor,
                              uint32_t* scan_tmp, size_t scan_tmp_words, const RcsrScratch& rx, hipStream_t s);
size_t scan_tmp_words(size_t count);

// Solve steps
constexpr int TILE_VERTICES = 256;  // vertices (or list entries) per block tile
hipError_t launch_init(const DevGame& g, int vbits, int resume, int grid, hipStream_t s);
// After all-vertex rounds up to r - 1: the predecessors of the vertices raised
// in round r - 1 are flagged for round r (whose flags must be zero), and the
// raise flags cleared.
hipError_t launch_activate_changed(const DevGame& g, int vbits, uint32_t r, int grid, hipStream_t s);
hipError_t launch_compact(const DevGame& g, uint32_t r, int grid, hipStream_t s);
hipError_t launch_round(const DevGame& g, int vbits, int h, bool dense, uint32_t r, int grid, hipStream_t s);
hipError_t launch_reduce_stats(const DevGame& g, int nblocks, hipStream_t s);
hipError_t launch_rounds_small(const DevGame& g, int vbits, uint32_t r0, uint32_t max_rounds, uint32_t limit,
                               hipStream_t s);
constexpr uint32_t SMALL_LIMIT = 1024;  // active-set size up to which one block runs the rounds
hipError_t launch_output(const DevGame& g, int vbits, int64_t* out, hipStream_t s);
hipError_t launch_input(const DevGame& g, int vbits, const int64_t* in, hipStream_t s);
// Player 0's strategy from the current measure: choice[c] per caller vertex
// (n entries), missing = player-0 vertices with finite value and no witness.
hipError_t launch_strategy(const DevGame& g, int vbits, int32_t* choice, uint32_t* missing, hipStream_t s);

int pick_h(double avg_deg);
int round_grid(int device);

}  // namespace eg
