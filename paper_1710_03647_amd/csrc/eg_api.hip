// libeg host runtime and C-ABI: validation, device layout, the round driver
// of the frontier iteration (Alg. 3), result conversion and statistics.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "eg.h"
#include "eg_internal.h"
#include "eg_serve.h"

namespace {

thread_local std::string t_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(EG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace eg {

void set_error(const char* msg) { t_err = msg; }
const char* get_error() { return t_err.c_str(); }

// Host-side validation of a game (host pointers).  Fills info; 0 or EG_EINVAL.
int check_host(const eg_game_desc* d, int bound_mode, eg_game_info* info, std::string* why,
               int64_t* clamp_out, std::vector<uint32_t>* act_bits) {
  auto bad = [&](const char* fmt, auto... a) {
    char buf[256];
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wformat-security"
    snprintf(buf, sizeof buf, fmt, a...);
#pragma clang diagnostic pop
    *why = buf;
    return EG_EINVAL;
  };
  if (!d) return bad("null game descriptor");
  if (d->n < 1) return bad("n = %d: a game needs at least one vertex", d->n);
  if (d->m < 0 || d->m >= ((int64_t)1 << 31)) return bad("m = %lld outside [0, 2^31)", (long long)d->m);
  if (!d->offsets || !d->owner_bits) return bad("null offsets or owner_bits");
  if (d->m > 0 && (!d->targets || !d->weights)) return bad("null targets or weights");
  if (d->W < 0) return bad("W = %d is negative", d->W);
  if (bound_mode != EG_BOUND_NW && bound_mode != EG_BOUND_MG) return bad("unknown bound mode %d", bound_mode);
  const int32_t n = d->n;
  const int64_t* off = d->offsets;
  if (off[0] != 0) return bad("offsets[0] = %lld, must be 0", (long long)off[0]);
  if (off[n] != d->m) return bad("offsets[n] = %lld, must equal m = %lld", (long long)off[n], (long long)d->m);
  int32_t max_out = 0;
  int64_t mg = 0;
  int32_t most_negative = 0, most_positive = 0;
  if (act_bits) act_bits->assign(((size_t)n + 31) / 32, 0u);
  for (int32_t v = 0; v < n; v++) {
    const int64_t a = off[v], b = off[v + 1];
    if (b < a) return bad("offsets decrease at vertex %d", v);
    if (b == a) return bad("vertex %d has no out-edge: the arena is not total", v);
    max_out = std::max<int32_t>(max_out, (int32_t)std::min<int64_t>(b - a, INT32_MAX));
    int32_t worst = 0;
    int64_t negatives = 0;
    for (int64_t e = a; e < b; e++) {
      const int32_t t = d->targets[e];
      if (t < 0 || t >= n) return bad("edge %lld of vertex %d targets %d, outside [0, %d)", (long long)e, v, t, n);
      const int32_t w = d->weights[e];
      if (w < 0 && -(int64_t)w > worst) worst = (int32_t)std::min<int64_t>(-(int64_t)w, INT32_MAX);
      if (w > most_positive) most_positive = w;
      negatives += w < 0;
    }
    // initial active set of Alg. 3 (line 3) and Alg. 1 (lines 1-2): player 0 with
    // every out-edge negative, player 1 with some negative out-edge
    const bool p1 = (d->owner_bits[v >> 3] >> (v & 7)) & 1;
    if (act_bits && (p1 ? negatives > 0 : negatives == b - a)) (*act_bits)[v >> 5] |= 1u << (v & 31);
    mg += worst;
    most_negative = std::max(most_negative, worst);
  }
  if ((int64_t)d->W < most_negative)
    return bad("W = %d is below the largest negative weight magnitude %d", d->W, most_negative);
  const int64_t bound = bound_mode == EG_BOUND_MG ? mg : (int64_t)(n - 1) * (int64_t)d->W;
  // On the device positive weights are clamped to P = min(max w, B + 1), which
  // leaves every finite term max(0, f(u) - w) with f(u) <= B unchanged, and TOP
  // is encoded as B + P + 1 so that TOP - w > B for every stored w.  The largest
  // intermediate value is then TOP + W.
  const int64_t clamp = std::min<int64_t>(most_positive, bound + 1);
  const __int128 hi = (__int128)bound + clamp + 1 + (__int128)d->W;
  if (hi > (__int128)INT64_MAX) return bad("bound %lld too large for int64 arithmetic", (long long)bound);
  if (clamp_out) *clamp_out = clamp;
  std::vector<int32_t> indeg(n, 0);
  int32_t max_in = 0;
  for (int64_t e = 0; e < d->m; e++) max_in = std::max(max_in, ++indeg[d->targets[e]]);
  if (info) {
    info->n = n;
    info->m = d->m;
    info->bound = bound;
    info->value_bits = hi < ((__int128)1 << 31) ? 32 : 64;
    info->max_outdeg = max_out;
    info->max_indeg = max_in;
    info->device_bytes = plan_layout(n, d->m, info->value_bits, 1, choose_parts(n, d->m, info->value_bits, 0)).total;
  }
  return EG_OK;
}

}  // namespace eg

struct eg_ctx {
  eg_config cfg;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int grid = 2048;
  std::mutex solve_mu;
  std::mutex server_mu;        // guards server and closing
  eg::Server* server = nullptr;
  bool closing = false;        // eg_ctx_destroy has started: no new serving thread
  std::mutex games_mu;
  std::set<eg_game*> games;    // live games, freed by eg_ctx_destroy
};

struct eg_game {
  eg_ctx* ctx = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  int32_t W = 0;
  int64_t bound = 0;
  int vbits = 64;
  int h = 1;
  eg_game_info info{};
  void* arena = nullptr;
  eg::DevGame dg{};
  int64_t* out64 = nullptr;
  size_t arena_bytes = 0;
  int grid = 1;
  int part_grid = 8;
  double avg_indeg = 1;
  uint32_t* h_blk = nullptr;
  uint32_t* h_ctrl = nullptr;
  unsigned long long* h_stats = nullptr;
  hipEvent_t ev[6] = {};
  void* seed_mem = nullptr;  // TOP-seeding scratch, allocated by the first seeding solve
  void* fbf_mem = nullptr;   // values of the Bellman-Ford seeding passes (top_seeding > 1)
  void* seg_mem = nullptr;   // segment tables and combined keys of edge-balanced dense rounds
  void* perm_mem = nullptr;  // internal id of each caller vertex (renumbered games)
  eg::SeedBuf sb{};
  uint32_t* h_seed = nullptr;
  void* sl_mem = nullptr;    // slice-major rounds: the blocks' work items
  int sl_grid = 0;           // k_sliced's grid (the one its work items are balanced over)
  void* scc_mem = nullptr;   // components and levels (component schedule), computed by the first such solve
  uint32_t* h_scc = nullptr;
  eg::SccBuf scc{};
  eg::SccInfo scc_info{};
  bool at_fixpoint = false;  // the device measure is the least fixpoint (last solve returned EG_OK)
};

// The exported functions keep the C linkage of their declarations in eg.h.

const char* eg_last_error(eg_ctx*) { return t_err.c_str(); }

int eg_check(const eg_game_desc* desc, int bound_mode, eg_game_info* info, char* msg, size_t msg_len) {
  std::string why;
  if (desc && desc->mem != EG_MEM_HOST) {
    why = "eg_check takes host pointers only";
    if (msg && msg_len) snprintf(msg, msg_len, "%s", why.c_str());
    return fail(EG_EINVAL, "%s", why.c_str());
  }
  int rc = eg::check_host(desc, bound_mode, info, &why, nullptr, nullptr);
  if (msg && msg_len) snprintf(msg, msg_len, "%s", why.c_str());
  if (rc != EG_OK) return fail(rc, "%s", why.c_str());
  return EG_OK;
}

int eg_ctx_create(const eg_config* cfg, eg_ctx** out) {
  if (!out) return fail(EG_EINVAL, "null output pointer");
  *out = nullptr;
  eg_config c{};
  if (cfg) c = *cfg;
  if (c.bound_mode != EG_BOUND_NW && c.bound_mode != EG_BOUND_MG)
    return fail(EG_EINVAL, "unknown bound mode %d", c.bound_mode);
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (c.device < 0 || c.device >= ndev) return fail(EG_EDEVICE, "device %d not present (%d devices)", c.device, ndev);
  HIPCHK(hipSetDevice(c.device));
  eg_ctx* ctx = new eg_ctx();
  ctx->cfg = c;
  if (c.hip_stream) {
    ctx->stream = (hipStream_t)c.hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete ctx;
      return fail(EG_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    ctx->own_stream = true;
  }
  if (c.blocks_per_cu < 0 || c.blocks_per_cu > 32 || c.dense_div < 0 || c.small_limit < 0 || c.small_limit > 65536 ||
      c.partition < 0 || c.partition > 3 || c.top_seeding < 0 || c.top_seeding > 64 || c.seg_edges < -1 ||
      c.p1_filter < 0 || c.p1_filter > 1 || c.scc_schedule < 0 || c.scc_schedule > 1 || c.hub_cache < -1 || c.hub_cache > 64 ||
      c.relabel < 0 || c.relabel > 2 ||
      (c.seg_edges > 0 && c.seg_edges < 256)) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return fail(EG_EINVAL, "launch-shape field out of range");
  }
  ctx->grid = eg::round_grid(c.device) / 8 * (c.blocks_per_cu ? c.blocks_per_cu : 8);
  *out = ctx;
  return EG_OK;
}

static void game_free(eg_game* g);

int eg_ctx_destroy(eg_ctx* ctx) {
  if (!ctx) return fail(EG_EINVAL, "null context");
  (void)hipSetDevice(ctx->cfg.device);
  eg::Server* srv = nullptr;
  {
    std::lock_guard<std::mutex> lock(ctx->server_mu);
    ctx->closing = true;
    srv = ctx->server;
    ctx->server = nullptr;
  }
  // cancels every pending and running ticket, wakes the threads blocked in
  // eg_wait and waits until every serving call in progress has returned
  if (srv) eg::server_destroy(srv);
  {
    std::lock_guard<std::mutex> solve_lock(ctx->solve_mu);  // a solve in progress finishes first
    std::lock_guard<std::mutex> lock(ctx->games_mu);
    for (eg_game* g : ctx->games) game_free(g);
    ctx->games.clear();
  }
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return EG_OK;
}

static void game_free(eg_game* g) {
  if (!g) return;
  if (g->arena) (void)hipFree(g->arena);
  if (g->h_ctrl) (void)hipHostFree(g->h_ctrl);
  if (g->h_blk) (void)hipHostFree(g->h_blk);
  if (g->h_stats) (void)hipHostFree(g->h_stats);
  if (g->seed_mem) (void)hipFree(g->seed_mem);
  if (g->fbf_mem) (void)hipFree(g->fbf_mem);
  if (g->seg_mem) (void)hipFree(g->seg_mem);
  if (g->perm_mem) (void)hipFree(g->perm_mem);
  if (g->h_seed) (void)hipHostFree(g->h_seed);
  if (g->scc_mem) (void)hipFree(g->scc_mem);
  if (g->sl_mem) (void)hipFree(g->sl_mem);
  if (g->h_scc) (void)hipHostFree(g->h_scc);
  for (auto& e : g->ev)
    if (e) (void)hipEventDestroy(e);
  delete g;
}

int eg::host_view(const eg_game_desc* desc, hipStream_t s, HostCopy& hc, eg_game_desc& hd) {
  hd = *desc;
  if (desc->mem == EG_MEM_HOST) return EG_OK;
  if (desc->mem != EG_MEM_DEVICE) return fail(EG_EINVAL, "unknown memory kind %d", desc->mem);
  if (desc->n < 1 || desc->m < 0 || desc->m >= ((int64_t)1 << 31))
    return fail(EG_EINVAL, "n = %d, m = %lld", desc->n, (long long)desc->m);
  if (!desc->offsets || !desc->owner_bits || (desc->m > 0 && (!desc->targets || !desc->weights)))
    return fail(EG_EINVAL, "null device pointer");
  hc.off.resize((size_t)desc->n + 1);
  hc.tgt.resize((size_t)desc->m);
  hc.w.resize((size_t)desc->m);
  hc.own.resize(((size_t)desc->n + 7) / 8);
  HIPCHK(hipMemcpyAsync(hc.off.data(), desc->offsets, 8 * hc.off.size(), hipMemcpyDeviceToHost, s));
  if (desc->m > 0) {
    HIPCHK(hipMemcpyAsync(hc.tgt.data(), desc->targets, 4 * hc.tgt.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hc.w.data(), desc->weights, 4 * hc.w.size(), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipMemcpyAsync(hc.own.data(), desc->owner_bits, hc.own.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  hd.offsets = hc.off.data();
  hd.targets = hc.tgt.data();
  hd.weights = hc.w.data();
  hd.owner_bits = hc.own.data();
  hd.mem = EG_MEM_HOST;
  return EG_OK;
}

namespace eg {

// Target-sliced dense rounds (8 slices, one per XCD) only when asked for
// (mode 2; the tile-local source index needs targets below 2^22).  A sliced
// round reads nothing written in the same round, so it is a synchronous
// (Jacobi) round: cheaper per round on large games, but the solve needs more
// rounds than with in-place updates, which carry values along paths within a
// round.  Measured to the fixpoint, unsliced rounds won on every large game
// tried (uniform 2^20: 66 s against 158 s; R-MAT 2^18: 6.4 s against 21 s).
uint32_t choose_parts(int32_t n, int64_t, int vbits, int mode) {
  // the chunk counters of the build reuse the n + 1 words of a cursor
  if (n > (1 << PTILE_SHIFT) || (uint64_t)((n + PTILE - 1) / PTILE) * 64 > (uint64_t)n) return 1;
  if (mode == 2) return 8;  // one slice per XCD
  if (mode == 3) {
    // slice-major: slices of about SL_SLICE_BYTES of f, 8 to 64 of them
    const uint64_t bytes = (uint64_t)n * (uint64_t)(vbits / 8);
    uint32_t s = 8;
    while (s < 64 && bytes > (uint64_t)s * SL_SLICE_BYTES) s *= 2;
    return s;
  }
  return 1;
}

GameLayout plan_layout(int32_t n, int64_t m, int vbits, size_t nblk, uint32_t nparts, bool filter, bool slice_major) {
  const size_t nn = (size_t)n, mm = (size_t)m, vb = (size_t)vbits / 8;
  const bool pe = nparts > 1;
  const size_t sizes[L_N] = {4 * (nn + 1), 8 * mm, 4 * (nn + 1), 4 * mm, vb * nn, 2 * align_up(nn + 4), 4 * nn,
                             4 * nn, 8 * nn, 4 * C_WORDS, 8 * S_WORDS, 4 * ((nn + 31) / 32), 4 * nblk,
                             8 * S_WORDS * nblk, pe ? 8 * mm : 0, pe ? 4 * partition_scratch_words(n, nparts) : 0,
                             pe ? 4 * ((nn + 31) / 32) : 0, pe ? vb * nn * (slice_major ? 1 : nparts) : 0,
                             filter ? 4 * mm : 0};
  GameLayout L{};
  for (int i = 0; i < L_N; i++) {
    L.off[i] = L.total;
    L.total += align_up(std::max<size_t>(sizes[i], 4));
  }
  return L;
}

void bind_layout(DevGame& dg, char* base, const GameLayout& L, int32_t n, int64_t m, int vbits, uint32_t nparts,
                 bool filter) {
  dg.n = n;
  dg.m = (uint32_t)m;
  dg.rs = (uint32_t*)(base + L.off[L_RS]);
  dg.edges = (int2*)(base + L.off[L_EDGES]);
  dg.rev_off = (uint32_t*)(base + L.off[L_ROFF]);
  dg.rev_src = (int32_t*)(base + L.off[L_RSRC]);
  dg.f = base + L.off[L_F];
  dg.act0 = (uint8_t*)(base + L.off[L_ACT]);
  dg.act1 = dg.act0 + align_up((size_t)n + 4);
  dg.wl0 = (int32_t*)(base + L.off[L_WL0]);
  dg.wl1 = (int32_t*)(base + L.off[L_WL1]);
  dg.ctrl = (uint32_t*)(base + L.off[L_CTRL]);
  dg.stats = (unsigned long long*)(base + L.off[L_STATS]);
  dg.act_bits = (const uint32_t*)(base + L.off[L_ACTBITS]);
  dg.blk_chg = (uint32_t*)(base + L.off[L_BLK]);
  dg.slots = (unsigned long long*)(base + L.off[L_SLOTS]);
  dg.vbits = vbits;
  dg.nparts = nparts;
  dg.part_size = (uint32_t)(((size_t)n + nparts - 1) / nparts);
  dg.pedges = (const int2*)(base + L.off[L_PEDGES]);
  dg.poff = (const uint32_t*)(base + L.off[L_POFF]);
  dg.own_bits = (const uint32_t*)(base + L.off[L_OWNB]);
  dg.part = base + L.off[L_PART];
  dg.rev_w = filter ? (const int32_t*)(base + L.off[L_RW]) : nullptr;
}

size_t staging_bytes(int32_t n, int64_t m, bool host_inputs, bool weights) {
  const size_t nn = (size_t)n, mm = (size_t)m;
  size_t t = align_up(4 * (nn + 1)) + align_up(4 * scan_tmp_words(nn + 1)) + align_up(4 * ((size_t)RB_BUCKETS + 1)) +
             align_up(4 * (size_t)RB_BUCKETS);
  // the bucketed entries of the reverse-CSR build take the place of the
  // target and weight copies of host inputs, which the layout has consumed
  if (host_inputs) t += align_up(8 * (nn + 1)) + 2 * align_up(std::max<size_t>(4 * mm, 4)) + align_up((nn + 7) / 8);
  else t += align_up(std::max<size_t>(8 * mm, 8));
  if (weights) t += align_up(std::max<size_t>(4 * mm, 4));
  return t;
}

hipError_t upload_game(const eg_game_desc* d, const HostPrep& prep, DevGame& dg, void* staging, hipStream_t s,
                       hipEvent_t after_layout, hipEvent_t after_rcsr) {
  const size_t nn = (size_t)d->n, mm = (size_t)d->m;
  const bool host_in = d->mem == EG_MEM_HOST;
  char* sb = (char*)staging;
  uint32_t* cursor = (uint32_t*)sb;
  sb += align_up(4 * (nn + 1));
  uint32_t* scan_tmp = (uint32_t*)sb;
  const size_t scan_words = scan_tmp_words(nn + 1);
  sb += align_up(4 * scan_words);
  RcsrScratch rx{};
  rx.bcnt = (uint32_t*)sb;
  sb += align_up(4 * ((size_t)RB_BUCKETS + 1));
  rx.bcur = (uint32_t*)sb;
  sb += align_up(4 * (size_t)RB_BUCKETS);
  const int64_t* d_off = d->offsets;
  const int32_t* d_tgt = d->targets;
  const int32_t* d_w = d->weights;
  const uint8_t* d_own = d->owner_bits;
  hipError_t r;
  if (host_in) {
    int64_t* o = (int64_t*)sb;
    sb += align_up(8 * (nn + 1));
    int32_t* t = (int32_t*)sb;
    rx.ent = (int2*)sb;  // written by the reverse-CSR build, after the layout has read t and w
    sb += align_up(std::max<size_t>(4 * mm, 4));
    int32_t* w = (int32_t*)sb;
    sb += align_up(std::max<size_t>(4 * mm, 4));
    uint8_t* ob = (uint8_t*)sb;
    sb += align_up((nn + 7) / 8);
    if ((r = hipMemcpyAsync(o, d->offsets, 8 * (nn + 1), hipMemcpyHostToDevice, s))) return r;
    if (mm && (r = hipMemcpyAsync(t, d->targets, 4 * mm, hipMemcpyHostToDevice, s))) return r;
    if (mm && (r = hipMemcpyAsync(w, d->weights, 4 * mm, hipMemcpyHostToDevice, s))) return r;
    if ((r = hipMemcpyAsync(ob, d->owner_bits, (nn + 7) / 8, hipMemcpyHostToDevice, s))) return r;
    d_off = o;
    d_tgt = t;
    d_w = w;
    d_own = ob;
  } else {
    rx.ent = (int2*)sb;
    sb += align_up(std::max<size_t>(8 * mm, 8));
  }
  if (dg.rev_w) rx.entw = (int32_t*)sb;
  if ((r = hipMemcpyAsync((void*)dg.act_bits, prep.act_bits.data(), 4 * prep.act_bits.size(),
                          hipMemcpyHostToDevice, s)))
    return r;
  if ((r = launch_layout(d_off, d_own, d_tgt, d_w, d->n, (uint32_t)mm, (int32_t)prep.clamp, (uint32_t*)dg.rs,
                         (int2*)dg.edges, s)) != hipSuccess)
    return r;
  if (after_layout && (r = hipEventRecord(after_layout, s))) return r;
  if ((r = launch_reverse_csr(dg.rs, dg.edges, d->n, (uint32_t)mm, (uint32_t*)dg.rev_off, (int32_t*)dg.rev_src,
                              (int32_t*)dg.rev_w, cursor, scan_tmp, scan_words, rx, s)) != hipSuccess)
    return r;
  if (after_rcsr && (r = hipEventRecord(after_rcsr, s))) return r;
  if (dg.nparts > 1) return launch_partition(dg, d_own, cursor, scan_tmp, scan_words, s);
  return hipSuccess;
}

// Renumber the vertices by decreasing in-degree (ties by id) when in-degrees
// are very skewed: the values gathered most often then share cache lines.
static void relabel_by_indegree(const eg_game_desc& d, HostPrep& prep) {
  const int32_t n = d.n;
  const int64_t m = d.m;
  std::vector<int64_t> indeg((size_t)n, 0);
  for (int64_t e = 0; e < m; e++) indeg[(size_t)d.targets[e]]++;
  std::vector<int32_t> order((size_t)n);
  for (int32_t v = 0; v < n; v++) order[(size_t)v] = v;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return indeg[(size_t)a] > indeg[(size_t)b]; });
  prep.perm.assign((size_t)n, 0);
  for (int32_t i = 0; i < n; i++) prep.perm[(size_t)order[(size_t)i]] = i;
  prep.r_off.assign((size_t)n + 1, 0);
  prep.r_tgt.resize((size_t)m);
  prep.r_w.resize((size_t)m);
  prep.r_own.assign(((size_t)n + 7) / 8, 0);
  std::vector<uint32_t> act(prep.act_bits.size(), 0u);
  int64_t k = 0;
  for (int32_t i = 0; i < n; i++) {
    const int32_t v = order[(size_t)i];
    for (int64_t e = d.offsets[v]; e < d.offsets[v + 1]; e++, k++) {
      prep.r_tgt[(size_t)k] = prep.perm[(size_t)d.targets[e]];
      prep.r_w[(size_t)k] = d.weights[e];
    }
    prep.r_off[(size_t)i + 1] = k;
    if ((d.owner_bits[v >> 3] >> (v & 7)) & 1) prep.r_own[(size_t)i >> 3] |= (uint8_t)(1u << (i & 7));
    if ((prep.act_bits[(size_t)v >> 5] >> (v & 31)) & 1u) act[(size_t)i >> 5] |= 1u << (i & 31);
  }
  prep.act_bits.swap(act);
}

int prepare(const eg_game_desc* desc, int bound_mode, hipStream_t s, HostPrep& prep, std::string* why,
            uint32_t seg_edges, int relabel) {
  eg::HostCopy hc;
  eg_game_desc hd;
  int rc = host_view(desc, s, hc, hd);
  if (rc != EG_OK) {
    *why = t_err;
    return rc;
  }
  rc = check_host(&hd, bound_mode, &prep.info, why, &prep.clamp, &prep.act_bits);
  if (rc != EG_OK) return rc;
  if (relabel == 2 || (relabel == 0 && hd.n >= 4096 && hd.m > 0)) {
    int64_t max_in = 0;
    if (relabel == 0) {
      std::vector<int32_t> cnt((size_t)hd.n, 0);
      for (int64_t e = 0; e < hd.m; e++) max_in = std::max<int64_t>(max_in, ++cnt[(size_t)hd.targets[e]]);
    }
    // skewed: the largest in-degree is at least 64 times the average
    if (relabel == 2 || max_in * hd.n >= 64 * hd.m) {
      relabel_by_indegree(hd, prep);
      hd.offsets = prep.r_off.data();
    }
  }
  // segments per tile for edge-balanced dense rounds (full-frontier out-degree sums)
  if (seg_edges == 0) return EG_OK;
  const int64_t ntiles = ((int64_t)hd.n + TILE_VERTICES - 1) / TILE_VERTICES;
  std::vector<uint32_t> nseg((size_t)ntiles);
  bool cut = false;
  for (int64_t t = 0; t < ntiles; t++) {
    const int64_t e = hd.offsets[std::min<int64_t>(hd.n, (t + 1) * TILE_VERTICES)] - hd.offsets[t * TILE_VERTICES];
    nseg[(size_t)t] = (uint32_t)std::max<int64_t>(1, (e + seg_edges - 1) / seg_edges);
    cut |= nseg[(size_t)t] > 1;
  }
  if (cut) prep.tile_nseg.swap(nseg);
  return EG_OK;
}

}  // namespace eg

// Work items of the slice-major rounds (k_sliced): one per tile of PTILE
// sources, or, for a tile with more than a block's share of the edges, equal
// parts of its edges; dealt to the blocks largest first, each to the block
// with the fewest edges so far (every block then sweeps about the same number
// of edges per slice), and sorted by tile within a block.  The key array is
// set to the largest key (the rounds keep it so).
static hipError_t build_slice_major(eg_game* g, hipStream_t s) {
  eg::DevGame& dg = g->dg;
  const uint32_t n = (uint32_t)g->n, ntiles = (n + eg::PTILE - 1) / eg::PTILE;
  std::vector<uint32_t> rs((size_t)n + 1);
  hipError_t e = hipMemcpyAsync(rs.data(), dg.rs, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->ctx->cfg.device) != hipSuccess || cus <= 0)
    cus = 256;
  const uint32_t grid = (uint32_t)cus * eg::SL_BLOCKS_PER_CU;
  const uint64_t share = std::max<uint64_t>(4096, ((uint64_t)g->m + grid - 1) / grid);
  struct Item {
    uint64_t load;
    uint32_t tile, word;
  };
  std::vector<Item> items;
  for (uint32_t t = 0; t < ntiles; t++) {
    const uint32_t a = rs[(size_t)t * eg::PTILE] & eg::ROW_MASK;
    const uint32_t b = rs[std::min<size_t>(n, (size_t)(t + 1) * eg::PTILE)] & eg::ROW_MASK;
    const uint64_t edges = b - a;
    const uint32_t parts = (uint32_t)std::min<uint64_t>(0xFFFF, std::max<uint64_t>(1, (edges + share - 1) / share));
    for (uint32_t j = 0; j < parts; j++) items.push_back({edges / parts + 1, t, (j << 16) | parts});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.load > y.load; });
  std::vector<std::vector<Item>> per((size_t)grid);
  std::vector<std::pair<uint64_t, uint32_t>> heap;  // (load, block), a min-heap
  for (uint32_t b = 0; b < grid; b++) heap.push_back({0, b});
  auto cmp = [](const std::pair<uint64_t, uint32_t>& x, const std::pair<uint64_t, uint32_t>& y) { return x > y; };
  std::make_heap(heap.begin(), heap.end(), cmp);
  for (const Item& it : items) {
    std::pop_heap(heap.begin(), heap.end(), cmp);
    heap.back().first += it.load;
    per[heap.back().second].push_back(it);
    std::push_heap(heap.begin(), heap.end(), cmp);
  }
  std::vector<uint32_t> begin((size_t)grid + 1, 0);
  std::vector<uint32_t> flat;  // {tile, part word} pairs
  for (uint32_t b = 0; b < grid; b++) {
    auto& v = per[b];
    std::sort(v.begin(), v.end(), [](const Item& x, const Item& y) { return x.tile < y.tile; });
    begin[b] = (uint32_t)(flat.size() / 2);
    for (const Item& it : v) {
      flat.push_back(it.tile);
      flat.push_back(it.word);
    }
  }
  begin[grid] = (uint32_t)(flat.size() / 2);
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t bytes = up(4 * flat.size()) + up(4 * begin.size());
  if ((e = hipMalloc(&g->sl_mem, bytes)) != hipSuccess) return e;
  dg.sl_items = (const uint2*)g->sl_mem;
  dg.sl_begin = (const uint32_t*)((char*)g->sl_mem + up(4 * flat.size()));
  dg.slice_major = 1;
  g->sl_grid = (int)grid;
  if ((e = hipMemcpyAsync((void*)dg.sl_items, flat.data(), 4 * flat.size(), hipMemcpyHostToDevice, s))) return e;
  if ((e = hipMemcpyAsync((void*)dg.sl_begin, begin.data(), 4 * begin.size(), hipMemcpyHostToDevice, s))) return e;
  if ((e = eg::launch_fill_max(dg.part, g->n, g->vbits, s))) return e;
  return hipStreamSynchronize(s);
}

int eg_create(eg_ctx* ctx, const eg_game_desc* desc, eg_game** out, eg_stats* st) {
  if (!ctx || !desc || !out) return fail(EG_EINVAL, "null argument");
  *out = nullptr;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  hipStream_t s = ctx->stream;
  eg::HostPrep prep;
  std::string why;
  const uint32_t seg_edges = ctx->cfg.seg_edges < 0 ? 0u : ctx->cfg.seg_edges ? (uint32_t)ctx->cfg.seg_edges : eg::SEG_EDGES;
  // renumbering gathers the hubs into the first tiles, which only cut tiles
  // spread over blocks: automatic renumbering needs unsliced, cut dense rounds
  const int relabel = ctx->cfg.relabel == 0 && (seg_edges == 0 || ctx->cfg.partition == 2) ? 1 : ctx->cfg.relabel;
  int rc = eg::prepare(desc, ctx->cfg.bound_mode, s, prep, &why, seg_edges, relabel);
  if (rc != EG_OK) return fail(rc, "%s", why.c_str());

  eg_game* g = new eg_game();
  g->ctx = ctx;
  g->n = desc->n;
  g->m = desc->m;
  g->W = desc->W;
  g->bound = prep.info.bound;
  g->vbits = prep.info.value_bits;
  g->info = prep.info;
  g->h = eg::pick_h((double)desc->m / desc->n);
  const size_t nn = (size_t)g->n;
  const size_t nblk = (size_t)std::max(1, std::min<int>(ctx->grid, (int)((nn + eg::TILE_VERTICES - 1) / eg::TILE_VERTICES)));
  g->grid = (int)nblk;
  g->part_grid = std::max(8, ctx->grid / 8 * 8);
  const uint32_t nparts = eg::choose_parts(g->n, g->m, g->vbits, ctx->cfg.partition);
  const bool filter = ctx->cfg.p1_filter != 0;
  const bool slice_major = nparts > 1 && ctx->cfg.partition == 3;
  const eg::GameLayout L = eg::plan_layout(g->n, g->m, g->vbits, nblk, nparts, filter, slice_major);
  hipError_t e = hipMalloc(&g->arena, L.total);
  if (e != hipSuccess) {
    game_free(g);
    return fail(EG_ENOMEM, "device allocation of %zu bytes failed: %s", L.total, hipGetErrorString(e));
  }
  g->arena_bytes = L.total;
  eg::DevGame& dg = g->dg;
  eg::bind_layout(dg, (char*)g->arena, L, g->n, g->m, g->vbits, nparts, filter);
  g->out64 = (int64_t*)((char*)g->arena + L.off[eg::L_OUT]);
  dg.bound = g->bound;
  dg.top = g->bound + prep.clamp + 1;
  dg.lanes_ok = eg::lanes_ok_for(g->n, g->m, g->vbits);
  g->avg_indeg = (double)g->m / (double)nn;
  // renumbered games: the first ids are the most gathered values
  if (!prep.perm.empty() && ctx->cfg.hub_cache >= 0) {
    const size_t bytes = ctx->cfg.hub_cache ? (size_t)ctx->cfg.hub_cache << 10 : eg::HUB_BYTES;
    dg.hub_n = (uint32_t)std::min<size_t>(nn, bytes / (size_t)(g->vbits / 8));
  }

  auto cleanup_fail = [&](int code, const char* what, hipError_t err) {
    game_free(g);
    return fail(code, "%s: %s", what, hipGetErrorString(err));
  };
  if ((e = hipHostMalloc((void**)&g->h_ctrl, 4 * eg::C_WORDS, hipHostMallocDefault)) != hipSuccess)
    return cleanup_fail(EG_EDEVICE, "hipHostMalloc", e);
  if ((e = hipHostMalloc((void**)&g->h_stats, 8 * eg::S_WORDS, hipHostMallocDefault)) != hipSuccess)
    return cleanup_fail(EG_EDEVICE, "hipHostMalloc", e);
  if ((e = hipHostMalloc((void**)&g->h_blk, 4 * nblk, hipHostMallocDefault)) != hipSuccess)
    return cleanup_fail(EG_EDEVICE, "hipHostMalloc", e);
  if ((e = hipHostMalloc((void**)&g->h_seed, 4, hipHostMallocDefault)) != hipSuccess)
    return cleanup_fail(EG_EDEVICE, "hipHostMalloc", e);
  for (auto& ev : g->ev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) return cleanup_fail(EG_EDEVICE, "hipEventCreate", e);

  // the game as uploaded: the caller's arrays, or their renumbered copy
  eg_game_desc ud = *desc;
  if (!prep.perm.empty()) {
    ud = eg_game_desc{desc->n, desc->m, prep.r_off.data(), prep.r_tgt.data(), prep.r_w.data(), prep.r_own.data(),
                      desc->W, EG_MEM_HOST};
    if ((e = hipMalloc(&g->perm_mem, 4 * nn)) != hipSuccess) return cleanup_fail(EG_ENOMEM, "renumbering", e);
    if ((e = hipMemcpyAsync(g->perm_mem, prep.perm.data(), 4 * nn, hipMemcpyHostToDevice, s)) != hipSuccess)
      return cleanup_fail(EG_EDEVICE, "renumbering", e);
    dg.perm = (const int32_t*)g->perm_mem;
  }
  void* staging = nullptr;
  if ((e = hipMalloc(&staging, eg::staging_bytes(g->n, g->m, ud.mem == EG_MEM_HOST, filter))) != hipSuccess)
    return cleanup_fail(EG_ENOMEM, "staging allocation", e);
  auto run = [&]() -> hipError_t {
    hipError_t r;
    if ((r = hipEventRecord(g->ev[0], s)) != hipSuccess) return r;
    if ((r = eg::upload_game(&ud, prep, dg, staging, s, g->ev[1], g->ev[5])) != hipSuccess) return r;
    if ((r = hipEventRecord(g->ev[2], s)) != hipSuccess) return r;
    return hipStreamSynchronize(s);
  };
  e = run();
  (void)hipFree(staging);
  if (e != hipSuccess) return cleanup_fail(EG_EDEVICE, "upload/layout/reverse CSR", e);
  if (slice_major) {
    if ((e = build_slice_major(g, s)) != hipSuccess) return cleanup_fail(EG_EDEVICE, "slice-major work items", e);
  }
  if (!prep.tile_nseg.empty() && (dg.nparts == 1 || slice_major)) {
    // edge-balanced dense rounds: one work item per segment of every tile
    const size_t ntiles = prep.tile_nseg.size();
    std::vector<uint32_t> item_tile, item_seg;
    for (size_t t = 0; t < ntiles; t++)
      for (uint32_t j = 0; j < prep.tile_nseg[t]; j++) {
        item_tile.push_back((uint32_t)t);
        item_seg.push_back(j);
      }
    const size_t ni = item_tile.size();
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t bytes = 2 * up(4 * ni) + 2 * up(4 * ntiles) + up((size_t)(g->vbits / 8) * nn);
    if ((e = hipMalloc(&g->seg_mem, bytes)) != hipSuccess) return cleanup_fail(EG_ENOMEM, "segment tables", e);
    char* b = (char*)g->seg_mem;
    dg.item_tile = (const uint32_t*)b;
    b += up(4 * ni);
    dg.item_seg = (const uint32_t*)b;
    b += up(4 * ni);
    dg.tile_nseg = (const uint32_t*)b;
    b += up(4 * ntiles);
    dg.tile_done = (uint32_t*)b;
    b += up(4 * ntiles);
    dg.gkey = b;
    dg.nitems = (uint32_t)ni;
    auto seg_setup = [&]() -> hipError_t {
      hipError_t r;
      if ((r = hipMemcpyAsync((void*)dg.item_tile, item_tile.data(), 4 * ni, hipMemcpyHostToDevice, s))) return r;
      if ((r = hipMemcpyAsync((void*)dg.item_seg, item_seg.data(), 4 * ni, hipMemcpyHostToDevice, s))) return r;
      if ((r = hipMemcpyAsync((void*)dg.tile_nseg, prep.tile_nseg.data(), 4 * ntiles, hipMemcpyHostToDevice, s)))
        return r;
      if ((r = hipMemsetAsync(dg.tile_done, 0, 4 * ntiles, s))) return r;
      if ((r = eg::launch_gkey_init(dg, g->vbits, s))) return r;
      return hipStreamSynchronize(s);
    };
    if ((e = seg_setup()) != hipSuccess) return cleanup_fail(EG_EDEVICE, "segment tables", e);
  }
  if (st) {
    memset(st, 0, sizeof *st);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[1]);
    st->t_upload = ms * 1e-3;
    (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[5]);
    st->t_rcsr = ms * 1e-3;
    (void)hipEventElapsedTime(&ms, g->ev[5], g->ev[2]);
    st->t_slices = ms * 1e-3;
  }
  {
    std::lock_guard<std::mutex> lock(ctx->games_mu);
    ctx->games.insert(g);
  }
  *out = g;
  return EG_OK;
}

int eg_destroy(eg_game* g) {
  if (!g) return fail(EG_EINVAL, "null game");
  eg_ctx* ctx = g->ctx;
  (void)hipSetDevice(ctx->cfg.device);
  {
    std::lock_guard<std::mutex> lock(ctx->games_mu);
    if (!ctx->games.erase(g)) return fail(EG_EINVAL, "unknown game");
  }
  game_free(g);
  return EG_OK;
}

int eg_set_measure(eg_game* g, const int64_t* f) {
  if (!g || !f) return fail(EG_EINVAL, "null argument");
  for (int32_t v = 0; v < g->n; v++)
    if (f[v] != EG_TOP && (f[v] < 0 || f[v] > g->bound))
      return fail(EG_EINVAL, "f[%d] = %lld outside [0, %lld] and not EG_TOP", v, (long long)f[v], (long long)g->bound);
  std::lock_guard<std::mutex> lock(g->ctx->solve_mu);
  g->at_fixpoint = false;
  HIPCHK(hipSetDevice(g->ctx->cfg.device));
  hipStream_t s = g->ctx->stream;
  HIPCHK(hipMemcpyAsync(g->out64, f, 8 * (size_t)g->n, hipMemcpyHostToDevice, s));
  HIPCHK(eg::launch_input(g->dg, g->vbits, g->out64, s));
  HIPCHK(hipStreamSynchronize(s));
  return EG_OK;
}

// Rounds run in batches enqueued without waiting; after each batch the host
// reads the control words and the per-block change counts to detect the
// fixpoint (an empty active set) and to choose the representation of the next
// batch: dense while the active set is a large fraction of V, sparse (a list)
// otherwise.  Extra rounds enqueued after the fixpoint find no work and return.
// fixed_sb: seeding scratch supplied by the caller (seeding is then on
// whatever the context says); nullptr: the game's own, allocated by its first
// seeded solve.
static int solve_impl(eg_game* g, const eg_solve_opts* opts, int64_t* credits, eg_stats* st,
                      const eg::SeedBuf* fixed_sb) {
  if (!g) return fail(EG_EINVAL, "null game");
  eg_solve_opts o{};
  if (opts) o = *opts;
  if (o.driver != 0) return fail(EG_EINVAL, "eg_solve_opts.driver is reserved and must be 0");
  eg_ctx* ctx = g->ctx;
  const uint64_t max_rounds = o.max_rounds ? o.max_rounds : ctx->cfg.max_rounds;
  const double budget = o.time_budget_s > 0 ? o.time_budget_s : ctx->cfg.time_budget_s;
  std::lock_guard<std::mutex> lock(ctx->solve_mu);
  g->at_fixpoint = false;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  hipStream_t s = ctx->stream;
  const eg::DevGame& dg = g->dg;
  const int grid = g->grid;
  const double t0 = now_s();
  const bool scc = ctx->cfg.scc_schedule != 0;
  double t_scc = 0;
  if (scc && !g->scc_mem) {
    // components and levels of the game graph, once per game
    HIPCHK(hipMalloc(&g->scc_mem, eg::scc_bytes(g->n)));
    HIPCHK(hipHostMalloc((void**)&g->h_scc, 8, hipHostMallocDefault));
    eg::bind_scc(g->scc, g->scc_mem, g->n);
    const double ts = now_s();
    HIPCHK(eg::compute_scc(dg, g->scc, g->h_scc, s, &g->scc_info));
    t_scc = now_s() - ts;
  }
  // the level filter of the schedule (cleared again below when it is off)
  g->dg.level = scc ? g->scc.lev : nullptr;
  g->dg.cur_level = 0;
  const uint64_t dense_at = std::max<uint64_t>(1, (uint64_t)g->n / (ctx->cfg.dense_div ? ctx->cfg.dense_div : 32));
  const uint64_t small_limit = ctx->cfg.small_limit ? (uint64_t)ctx->cfg.small_limit : eg::SMALL_LIMIT;
  const bool seeding = fixed_sb || ctx->cfg.top_seeding != 0;
  if (fixed_sb) {
    g->sb = *fixed_sb;
  } else if (seeding) {
    if (!g->seed_mem) HIPCHK(hipMalloc(&g->seed_mem, eg::seed_bytes(g->n)));
    eg::bind_seed(g->sb, g->seed_mem, g->n);
    if (ctx->cfg.top_seeding > 1) {
      if (!g->fbf_mem) HIPCHK(hipMalloc(&g->fbf_mem, (size_t)g->n * (size_t)(g->vbits / 8)));
      g->sb.fbf = g->fbf_mem;
    }
  }
  uint64_t next_seed = 0, seeded = 0, seed_passes = 0;  // passes before the first round, then at doubling round counts
  double t_seed = 0;                                    // device time of the seeding passes
  HIPCHK(hipMemsetAsync(dg.ctrl, 0, 4 * eg::C_WORDS, s));
  HIPCHK(hipMemsetAsync(dg.slots, 0, 8 * eg::S_WORDS * (size_t)grid, s));
  HIPCHK(hipEventRecord(g->ev[0], s));
  HIPCHK(eg::launch_init(dg, g->vbits, o.resume ? 1 : 0, grid, s));
  // component schedule: level 0 replaces the initial active set
  if (scc) HIPCHK(eg::launch_level_activate(dg, g->scc.lev, 0, 1, grid, s));
  // the first seeding pass needs no decision of the host: it goes with init,
  // and one synchronization reads both
  if (seeding) {
    HIPCHK(hipEventRecord(g->ev[3], s));
    HIPCHK(eg::launch_seed(dg, g->vbits, g->sb, 1, !o.resume, ctx->cfg.top_seeding, s));
    HIPCHK(hipEventRecord(g->ev[4], s));
    HIPCHK(hipMemcpyAsync(g->h_seed, g->sb.count, 4, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipMemcpyAsync(g->h_blk, dg.blk_chg, 4 * (size_t)grid, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (seeding) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g->ev[3], g->ev[4]);
    t_seed += ms * 1e-3;
    seed_passes = 1;
    next_seed = 64;
    seeded += *g->h_seed;
  }
  uint64_t active = 0;
  for (int b = 0; b < grid; b++) active += g->h_blk[b];
  const int32_t nlevels = scc ? (int32_t)g->scc_info.levels : 1;
  bool wide = false;  // slice-major games: the next dense round lifts about half of V or more
  int32_t level = 0;
  uint32_t r = 1;
  uint64_t launched = 0;
  int status = EG_OK;
  // representation of the active set: a flag sweep for large sets, a list
  // for medium ones, and for small ones a single block running many rounds
  // ALL: every vertex lifted, nothing activated (while the frontier covers
  // about every vertex; not with per-XCD slices)
  enum { SPARSE, DENSE, SMALL, ALL };
  auto pick = [&](uint64_t size) { return size <= small_limit ? SMALL : size >= dense_at ? DENSE : SPARSE; };
  int mode = pick(active);
  // Each initially active vertex rises in round 1 (its flag means that its
  // lift from 0 is positive; on resume every vertex is active).  When their
  // predecessors would cover V, the first rounds lift every vertex instead of
  // flagging predecessors one store at a time.
  if (mode == DENSE && !scc && (dg.nparts == 1 || dg.slice_major) &&
      (double)active * g->avg_indeg >= (double)g->n)
    mode = ALL;
  // the predecessors of the first pass's TOP vertices are flagged for round 1
  if (seeding && *g->h_seed && mode != ALL) mode = DENSE;
  if (active && mode != DENSE && mode != ALL) HIPCHK(eg::launch_compact(dg, 1, grid, s));
  wide = 2 * active >= (uint64_t)g->n;
  uint32_t batch = 2;
  double t_kernels = 0;  // device time of the round kernels (back to back within a batch)
  uint64_t dense_rounds = 0, all_rounds = 0, all_streak = 0;
  for (;;) {
    if (!active) {
      // the active set is empty: the fixpoint, or with the component
      // schedule the end of a level (the next one starts from its vertices)
      if (++level >= nlevels) break;
      g->dg.cur_level = level;
      HIPCHK(eg::launch_level_activate(dg, g->scc.lev, level, r, grid, s));
      HIPCHK(hipMemcpyAsync(g->h_blk, dg.blk_chg, 4 * (size_t)grid, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int b = 0; b < grid; b++) active += g->h_blk[b];
      if (!active) continue;
      mode = pick(active);
      if (mode != DENSE) HIPCHK(eg::launch_compact(dg, r, grid, s));
      batch = 2;
    }
    if (seeding && launched >= next_seed) {
      HIPCHK(hipEventRecord(g->ev[3], s));
      HIPCHK(eg::launch_seed(dg, g->vbits, g->sb, r, seed_passes == 0 && !o.resume, ctx->cfg.top_seeding, s));
      HIPCHK(hipEventRecord(g->ev[4], s));
      HIPCHK(hipMemcpyAsync(g->h_seed, g->sb.count, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, g->ev[3], g->ev[4]);
        t_seed += ms * 1e-3;
      }
      seed_passes++;
      next_seed = std::max<uint64_t>(64, 2 * launched);
      if (*g->h_seed) {
        // the predecessors of the new TOP vertices are flagged for round r
        seeded += *g->h_seed;
        if (mode != ALL) mode = DENSE;  // ALL rounds lift every vertex anyway
        batch = 2;
      }
    }
    uint64_t allowed = 64;
    if (mode == SMALL) allowed = 8192;
    // All-vertex rounds each cost a full lift, and a batch may overshoot the
    // end of the phase: one at a time at first, then batches of half the
    // phase so far (long phases, as on the uniform game, pay few syncs).
    // (the first two rounds of a solve that starts with them are both of
    // this kind: round 1 raises every initially active vertex)
    else if (mode == ALL) allowed = launched == 0 ? 2 : std::min<uint64_t>(64, std::max<uint64_t>(1, all_streak / 2));
    else allowed = batch;
    if (max_rounds) allowed = std::min<uint64_t>(allowed, max_rounds - launched);
    HIPCHK(hipEventRecord(g->ev[3], s));
    if (mode == SMALL) {
      HIPCHK(eg::launch_rounds_small(dg, g->vbits, r, (uint32_t)allowed, (uint32_t)small_limit, s));
    } else {
      for (uint32_t j = 0; j < allowed; j++, r++) {
        if (dg.slice_major && (mode == ALL || (mode == DENSE && wide))) {
          HIPCHK(eg::launch_sliced(dg, g->vbits, r, g->sl_grid, s));
          HIPCHK(eg::launch_round_parts(dg, g->vbits, r, grid, s, mode == ALL));
        } else if (mode == DENSE && dg.nparts > 1 && !dg.slice_major) {
          HIPCHK(eg::launch_partial(dg, g->vbits, r, g->part_grid, s));
          HIPCHK(eg::launch_round_parts(dg, g->vbits, r, grid, s));
        } else if ((mode == DENSE || mode == ALL) && dg.nitems) {
          HIPCHK(eg::launch_round_seg(dg, g->vbits, r, grid, s, mode == ALL));
        } else if (mode == ALL) {
          HIPCHK(eg::launch_round_all(dg, g->vbits, r, grid, s));
        } else {
          HIPCHK(eg::launch_round(dg, g->vbits, g->h, mode == DENSE, r, grid, s));
        }
      }
    }
    HIPCHK(hipEventRecord(g->ev[4], s));
    HIPCHK(hipMemcpyAsync(g->h_ctrl, dg.ctrl, 4 * eg::C_WORDS, hipMemcpyDeviceToHost, s));
    if (mode == DENSE || mode == ALL)
      HIPCHK(hipMemcpyAsync(g->h_blk, dg.blk_chg, 4 * (size_t)grid, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, g->ev[3], g->ev[4]);
      t_kernels += ms * 1e-3;
    }
    if (mode == SMALL) {
      const uint32_t next_r = g->h_ctrl[eg::C_NEXT];
      launched += next_r - r;
      r = next_r;
      all_streak = 0;
    } else {
      launched += allowed;
      dense_rounds += mode == DENSE || mode == ALL ? allowed : 0;
      all_rounds += mode == ALL ? allowed : 0;
      all_streak = mode == ALL ? all_streak + allowed : 0;
    }
    int next_mode = mode;
    if (mode == DENSE || mode == ALL) {
      if (g->h_ctrl[eg::C_ANY0 + (r - 1) % 3] == 0) {  // nothing rose in the last round
        active = 0;
        continue;
      }
      uint64_t changed = 0;
      for (int b = 0; b < grid; b++) changed += g->h_blk[b];
      // predecessors of the changed vertices, at most
      const double est = (double)changed * g->avg_indeg;
      wide = est >= (double)g->n / 2;
      if (mode == ALL) {
        // (a list round would give a hub's row to one block; flag rounds cut it)
        if (est < (double)g->n / 2) next_mode = est <= (double)small_limit ? SMALL : DENSE;
      } else if (est >= (double)g->n && (dg.nparts == 1 || dg.slice_major) && !scc) {
        next_mode = ALL;
      } else if (est <= (double)small_limit) {
        next_mode = SMALL;
      } else if (est < (double)dense_at / 4) {
        next_mode = SPARSE;
      }
    } else {
      const uint64_t next = g->h_ctrl[eg::C_CNT0 + r % 3];
      if (next == 0) {
        active = 0;
        continue;
      }
      next_mode = pick(next);
    }
    if ((max_rounds && launched >= max_rounds) || (budget > 0 && now_s() - t0 > budget) || r > 0xFFFFFF00u) {
      status = EG_ETIMEDOUT;
      break;
    }
    if (next_mode != mode) {
      if (mode == DENSE && next_mode != ALL) HIPCHK(eg::launch_compact(dg, r, grid, s));
      if (mode == ALL) {
        // ALL rounds activate nothing but flag the vertices they raise: the
        // predecessors of the last one's raises form L_r, as a dense round
        // would have flagged them
        uint8_t* act_r = (r & 1) ? dg.act1 : dg.act0;
        HIPCHK(hipMemsetAsync(act_r, 0, (size_t)g->n, s));
        HIPCHK(eg::launch_activate_changed(dg, g->vbits, r, grid, s));
        if (next_mode != DENSE) HIPCHK(eg::launch_compact(dg, r, grid, s));
      }
      mode = next_mode;
      batch = 2;
    } else if (batch < 64) {
      batch *= 2;
    }
  }
  HIPCHK(hipEventRecord(g->ev[1], s));
  HIPCHK(eg::launch_reduce_stats(dg, grid, s));
  HIPCHK(hipMemcpyAsync(g->h_stats, dg.stats, 8 * eg::S_WORDS, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(g->h_ctrl, dg.ctrl, 4 * eg::C_WORDS, hipMemcpyDeviceToHost, s));
  if (credits) {
    HIPCHK(eg::launch_output(dg, g->vbits, g->out64, s));
    HIPCHK(hipMemcpyAsync(credits, g->out64, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipEventRecord(g->ev[2], s));
  HIPCHK(hipStreamSynchronize(s));
  if (st) {
    memset(st, 0, sizeof *st);
    st->rounds = g->h_ctrl[eg::C_ROUNDS];
    st->lifts = g->h_stats[eg::S_LIFTS];
    st->relaxed_edges = g->h_stats[eg::S_EDGES];
    st->pushes = g->h_stats[eg::S_PUSHES];
    st->changes = g->h_stats[eg::S_CHANGES];
    st->scanned_preds = g->h_stats[eg::S_SCANNED];
    st->filtered_preds = g->h_stats[eg::S_FILTERED];
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[1]);
    st->t_solve = ms * 1e-3;
    (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[2]);
    st->t_d2h = ms * 1e-3;
    const double vb = g->vbits / 8;
    // algorithmic bytes: per relaxed edge the {target, weight} pair and f(target);
    // per lift the active-set entry, the two row starts and f(v); per change the
    // store of f(v) and the two predecessor-list starts; per scanned predecessor
    // its id and its flag; per push the new entry
    st->model_bytes = st->relaxed_edges * (8 + vb) + st->lifts * (4 + 8 + vb) + st->changes * (vb + 8) +
                      st->scanned_preds * 8.0 + st->pushes * 4.0;
    st->achieved_gbps = st->t_solve > 0 ? st->model_bytes / st->t_solve / 1e9 : 0;
    st->t_round_kernels = t_kernels;
    st->launched_rounds = launched;
    st->seeded = seeded;
    st->seed_passes = seed_passes;
    st->dense_rounds = dense_rounds;
    st->all_rounds = all_rounds;
    st->t_seed = t_seed;
    if (scc) {
      st->scc_components = g->scc_info.components;
      st->scc_levels = g->scc_info.levels;
      st->t_scc = t_scc;
    }
  }
  if (status != EG_OK) return fail(status, "budget exhausted after %llu rounds", (unsigned long long)launched);
  g->at_fixpoint = true;
  return EG_OK;
}

int eg_solve_ex(eg_game* g, const eg_solve_opts* opts, int64_t* credits, eg_stats* st) {
  return solve_impl(g, opts, credits, st, nullptr);
}

int eg_solve(eg_game* g, int64_t* credits, eg_stats* st) { return eg_solve_ex(g, nullptr, credits, st); }

// ---------------------------------------------------------------- seeded solve without allocation
//
// The seeding scratch of eg_solve_seeded_noalloc: one array per device, which
// each device holds from the first such call until the process ends.  In host
// code `scratch` names a host-side stand-in; the device address of a device's
// copy comes from hipGetSymbolAddress, taken once per device on its first
// call (not at context creation, so that processes that never make this call
// do not load and hold the array).
namespace {
constexpr size_t pad256(size_t x) { return (x + 255) & ~(size_t)255; }
// the layout of eg::seed_bytes for EG_NOALLOC_MAX_N vertices
constexpr size_t NOALLOC_SCRATCH_BYTES = 2 * pad256(4 * (size_t)EG_NOALLOC_MAX_N) +
                                         3 * pad256(8 * (size_t)EG_NOALLOC_MAX_N) +
                                         2 * pad256((size_t)EG_NOALLOC_MAX_N) + pad256(16);
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_DEVICES = 64;
std::mutex scratch_table_mu;
void* scratch_ptr[NOALLOC_DEVICES];           // device address of each device's copy (nullptr: not taken yet)
std::mutex scratch_use_mu[NOALLOC_DEVICES];   // one call at a time per device uses its copy

int noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= NOALLOC_DEVICES) return fail(EG_EDEVICE, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> lock(scratch_table_mu);
  if (!scratch_ptr[device]) {
    HIPCHK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(EG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return EG_OK;
}
}  // namespace

int eg_solve_seeded_noalloc(eg_game* g, const eg_solve_opts* opts, int64_t* credits, eg_stats* st) {
  if (!g) return fail(EG_EINVAL, "null game");
  if (g->n > EG_NOALLOC_MAX_N)
    return fail(EG_EINVAL, "n = %d exceeds EG_NOALLOC_MAX_N = %d, the vertices the static seeding scratch holds",
                g->n, EG_NOALLOC_MAX_N);
  static_assert(NOALLOC_SCRATCH_BYTES >= 34 * (size_t)EG_NOALLOC_MAX_N, "scratch smaller than seed_bytes");
  const int device = g->ctx->cfg.device;
  void* base = nullptr;
  const int rc = noalloc_scratch(device, &base);
  if (rc != EG_OK) return rc;
  if (eg::seed_bytes(g->n) > NOALLOC_SCRATCH_BYTES) return fail(EG_EINVAL, "seeding scratch layout too large");
  // calls on one device share its copy: they run one after another
  std::lock_guard<std::mutex> lock(scratch_use_mu[device]);
  eg::SeedBuf sb{};
  eg::bind_seed(sb, base, g->n);
  return solve_impl(g, opts, credits, st, &sb);
}

int eg_strategy(eg_game* g, int32_t* choice, double* t_kernel) {
  if (!g || !choice) return fail(EG_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(g->ctx->solve_mu);
  if (!g->at_fixpoint) return fail(EG_EINVAL, "no least fixpoint on the device: eg_solve must return EG_OK first");
  HIPCHK(hipSetDevice(g->ctx->cfg.device));
  hipStream_t s = g->ctx->stream;
  // the output staging buffer (8n bytes) holds the n choices and the counter
  int32_t* d_choice = (int32_t*)g->out64;
  uint32_t* d_missing = (uint32_t*)(d_choice + g->n);
  uint32_t missing = 0;
  HIPCHK(hipMemsetAsync(d_missing, 0, 4, s));
  HIPCHK(hipEventRecord(g->ev[0], s));
  HIPCHK(eg::launch_strategy(g->dg, g->vbits, d_choice, d_missing, s));
  HIPCHK(hipEventRecord(g->ev[1], s));
  HIPCHK(hipMemcpyAsync(choice, d_choice, 4 * (size_t)g->n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&missing, d_missing, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (t_kernel) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[1]);
    *t_kernel = ms * 1e-3;
  }
  if (missing) return fail(EG_EDEVICE, "%u player-0 vertices have no witnessing edge", missing);
  return EG_OK;
}

int eg_components(eg_game* g, int32_t* comp, int32_t* level, uint32_t* components, uint32_t* levels) {
  if (!g || !comp || !level) return fail(EG_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(g->ctx->solve_mu);
  HIPCHK(hipSetDevice(g->ctx->cfg.device));
  hipStream_t s = g->ctx->stream;
  if (!g->scc_mem) {
    HIPCHK(hipMalloc(&g->scc_mem, eg::scc_bytes(g->n)));
    HIPCHK(hipHostMalloc((void**)&g->h_scc, 8, hipHostMallocDefault));
    eg::bind_scc(g->scc, g->scc_mem, g->n);
    HIPCHK(eg::compute_scc(g->dg, g->scc, g->h_scc, s, &g->scc_info));
  }
  // in the caller's numbering, through the output staging buffer (8n bytes)
  int32_t* d_comp = (int32_t*)g->out64;
  int32_t* d_lev = d_comp + g->n;
  HIPCHK(eg::launch_scc_output(g->dg, g->scc, d_comp, d_lev, s));
  HIPCHK(hipMemcpyAsync(comp, d_comp, 4 * (size_t)g->n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(level, d_lev, 4 * (size_t)g->n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (components) *components = g->scc_info.components;
  if (levels) *levels = g->scc_info.levels;
  return EG_OK;
}

// The context's server with one use taken (released by server_leave), so that
// eg_ctx_destroy waits for this call before freeing it; nullptr when there is
// none (and create = false) or the context is being destroyed.
static eg::Server* server_use(eg_ctx* ctx, bool create) {
  std::lock_guard<std::mutex> lock(ctx->server_mu);
  if (ctx->closing) return nullptr;
  if (!ctx->server && create) ctx->server = eg::server_create(ctx->cfg, ctx->stream);
  if (ctx->server) eg::server_enter(ctx->server);
  return ctx->server;
}

int eg_submit(eg_ctx* ctx, const eg_game_desc* desc, eg_ticket* out) {
  if (!ctx || !desc || !out) return fail(EG_EINVAL, "null argument");
  eg::Server* s = server_use(ctx, true);
  if (!s) return fail(EG_ECANCELED, "the context is being destroyed");
  const int rc = eg::server_submit(s, desc, ctx->stream, out);
  eg::server_leave(s);
  return rc;
}

int eg_poll(eg_ctx* ctx, eg_ticket t, int64_t* credits, eg_stats* st) {
  if (!ctx) return fail(EG_EINVAL, "null context");
  eg::Server* s = server_use(ctx, false);
  if (!s) return fail(EG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  const int rc = eg::server_poll(s, t, credits, st);
  eg::server_leave(s);
  return rc;
}

int eg_wait(eg_ctx* ctx, eg_ticket t, int64_t* credits, eg_stats* st, double timeout_s) {
  if (!ctx) return fail(EG_EINVAL, "null context");
  eg::Server* s = server_use(ctx, false);
  if (!s) return fail(EG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  const int rc = eg::server_wait(s, t, credits, st, timeout_s);
  eg::server_leave(s);
  return rc;
}

int eg_solve_batch(eg_ctx* ctx, const eg_game_desc* games, int count, int64_t* const* credits, eg_stats* stats) {
  if (!ctx || (count > 0 && (!games || !credits))) return fail(EG_EINVAL, "null argument");
  if (count < 0) return fail(EG_EINVAL, "count = %d", count);
  std::vector<eg_ticket> t((size_t)count);
  int rc = EG_OK;
  int submitted = 0;
  for (; submitted < count; submitted++) {
    rc = eg_submit(ctx, &games[submitted], &t[(size_t)submitted]);
    if (rc != EG_OK) break;
  }
  const std::string submit_err = rc != EG_OK ? t_err : std::string();
  int first_err = rc;
  for (int i = 0; i < submitted; i++) {
    if (first_err != EG_OK) {
      eg_cancel(ctx, t[(size_t)i]);
      eg_wait(ctx, t[(size_t)i], nullptr, nullptr, 0);
      continue;
    }
    const int r = eg_wait(ctx, t[(size_t)i], credits[i], stats ? &stats[i] : nullptr, 0);
    if (r != EG_OK) first_err = r;
  }
  if (!submit_err.empty()) t_err = submit_err;
  return first_err;
}

int eg_cancel(eg_ctx* ctx, eg_ticket t) {
  if (!ctx) return fail(EG_EINVAL, "null context");
  eg::Server* s = server_use(ctx, false);
  if (!s) return fail(EG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  const int rc = eg::server_cancel(s, t);
  eg::server_leave(s);
  return rc;
}
