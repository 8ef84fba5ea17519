// Serving runtime of libeg: continuous batching of many games.
//
// eg_submit copies a game into a FIFO of pending tickets.  One serving thread
// per context owns the device side:
//   * an HBM arena (one allocation of the budget, first-fit sub-allocation)
//     that holds every resident game's arrays;
//   * a slot table read by the batched kernels (k_plan + k_batch_round): all
//     resident games advance together, one round per epoch, each from its
//     own join epoch, and each is retired when its own round raised nothing;
//   * hipGraphs of K epochs, replayed while games are resident.
// Between graph launches the thread admits pending games in FIFO order while
// a slot is free and the game's footprint fits the arena (upload, layout and
// predecessor lists on a side stream; init and publication of the slot on the
// main stream, so a newcomer starts at the next epoch while the others keep
// running), retires finished games (result conversion, copy to the ticket,
// slot and arena freed), and drops cancelled ones.  With top_seeding a game
// gets one seeding pass (negative cycles that player 1 can force set to TOP,
// exact) between its init and its first epoch.  The per-game arithmetic is
// the single-game kernel's tile code, so a game's credits do not depend on
// what it shares the device with.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "eg_internal.h"
#include "eg_serve.h"

namespace eg {

int prepare(const eg_game_desc* desc, int bound_mode, hipStream_t s, HostPrep& prep, std::string* why,
            uint32_t seg_edges, int relabel);
hipError_t launch_output(const DevGame& g, int vbits, int64_t* out, hipStream_t s);

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit sub-allocator over one device allocation; adjacent free ranges merge.
class Arena {
 public:
  bool init(size_t bytes) {
    capacity_ = align_up(bytes);
    if (hipMalloc(&base_, capacity_) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = capacity_;
    return true;
  }
  void release() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  // offset of a range of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, ALIGN));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      live_[off] = bytes;
      used_ += bytes;
      return off;
    }
    return SIZE_MAX;
  }
  void free(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t size = it->second;
    live_.erase(it);
    used_ -= size;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + size == next->first) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += size;
        return;
      }
    }
    free_[off] = size;
  }
  char* base() const { return (char*)base_; }
  size_t capacity() const { return capacity_; }
  size_t used() const { return used_; }

 private:
  void* base_ = nullptr;
  size_t capacity_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
  std::unordered_map<size_t, size_t> live_;
};

enum TicketState { T_PENDING, T_RUNNING, T_DONE, T_FAILED, T_CANCELLED };

struct Ticket {
  eg_ticket id = 0;
  TicketState state = T_PENDING;
  int error = 0;
  bool cancel = false;
  // host copy of the game
  int32_t n = 0;
  int64_t m = 0;
  int32_t W = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> tgt, w;
  std::vector<uint8_t> own;
  HostPrep prep;
  size_t footprint = 0;
  // while resident
  int slot = -1;
  size_t arena_off = 0;
  DevGame dg{};
  int64_t* out64 = nullptr;
  // result
  std::vector<int64_t> credits;
  eg_stats stats{};
  double t_arrive = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct Server {
  eg_config cfg{};
  int grid = 2048;
  int nslots = 1024;
  size_t max_pending = 65536;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Ticket*> pending;
  std::unordered_map<eg_ticket, std::unique_ptr<Ticket>> tickets;
  eg_ticket next_id = 1;
  bool stop = false;
  int users = 0;  // API calls in progress (server_enter .. server_leave)
  bool device_ok = false;
  std::string device_error;
  std::thread worker;

  // device side (owned by the worker thread after start)
  hipStream_t main = nullptr, side = nullptr;
  Arena arena;
  void* table_mem = nullptr;
  BatchTable bt{};
  DevGame* h_games = nullptr;  // pinned: descriptors to publish
  uint32_t* h_words = nullptr; // pinned: per slot {state, mode, round} staging
  uint32_t* h_state = nullptr; // pinned: readback of state[]
  uint32_t* h_mode = nullptr;  // pinned: readback of mode[]
  uint32_t* h_rounds = nullptr;
  unsigned long long* h_st = nullptr;
  std::vector<Ticket*> slot_ticket;
  std::vector<int> free_slots;
  uint64_t epochs = 0;
  std::map<int, hipGraphExec_t> graphs;
  hipEvent_t ev_upload = nullptr;
  hipEvent_t ev_main = nullptr, ev_side = nullptr;
  hipEvent_t ev_g0 = nullptr, ev_g1 = nullptr;  // around the epochs' graph (timed)
  double epoch_us = 0;                           // recent duration of one epoch (0: not measured yet)

  bool init_device(std::string* why);
  void release_device();
  void run();
  int admit_one(Ticket* t);
  int nrunning = 0;  // worker-owned
  void retire(int slot, bool finished);
  hipGraphExec_t graph_for(int k);
};

static int set_err(int code, const std::string& msg) {
  set_error(msg.c_str());
  return code;
}

bool Server::init_device(std::string* why) {
  auto bad = [&](const char* what, hipError_t e) {
    *why = std::string(what) + ": " + hipGetErrorString(e);
    return false;
  };
  hipError_t e;
  if ((e = hipSetDevice(cfg.device))) return bad("hipSetDevice", e);
  if ((e = hipStreamCreateWithFlags(&main, hipStreamNonBlocking))) return bad("stream", e);
  if ((e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking))) return bad("stream", e);
  if ((e = hipEventCreateWithFlags(&ev_upload, hipEventDisableTiming))) return bad("event", e);
  if ((e = hipEventCreateWithFlags(&ev_main, hipEventDisableTiming))) return bad("event", e);
  if ((e = hipEventCreateWithFlags(&ev_side, hipEventDisableTiming))) return bad("event", e);
  if ((e = hipEventCreate(&ev_g0))) return bad("event", e);
  if ((e = hipEventCreate(&ev_g1))) return bad("event", e);
  size_t free_b = 0, total_b = 0;
  if ((e = hipMemGetInfo(&free_b, &total_b))) return bad("hipMemGetInfo", e);
  size_t budget = cfg.hbm_budget_bytes ? cfg.hbm_budget_bytes : free_b / 4;
  budget = std::min(budget, free_b - std::min(free_b, (size_t)1 << 30));
  if (!arena.init(budget)) {
    *why = "cannot reserve the HBM budget of " + std::to_string(budget) + " bytes";
    return false;
  }
  const size_t ns = (size_t)nslots;
  const size_t sizes[] = {sizeof(DevGame) * ns, 4 * ns, 4 * ns, 4 * ns, 4 * ns, 4 * ns, 4 * (ns + 1),
                          8 * S_WORDS * ns, 4 * B_WORDS};
  constexpr int NARR = sizeof(sizes) / sizeof(sizes[0]);
  size_t offs[NARR], total = 0;
  for (int i = 0; i < NARR; i++) {
    offs[i] = total;
    total += align_up(sizes[i]);
  }
  if ((e = hipMalloc(&table_mem, total))) return bad("slot table", e);
  if ((e = hipMemset(table_mem, 0, total))) return bad("slot table", e);
  char* b = (char*)table_mem;
  bt.games = (const DevGame*)(b + offs[0]);
  bt.state = (uint32_t*)(b + offs[1]);
  bt.mode = (uint32_t*)(b + offs[2]);
  bt.round = (uint32_t*)(b + offs[3]);
  bt.cur = (uint32_t*)(b + offs[4]);
  bt.rounds = (uint32_t*)(b + offs[5]);
  bt.task_begin = (uint32_t*)(b + offs[6]);
  bt.st = (unsigned long long*)(b + offs[7]);
  bt.ctl = (uint32_t*)(b + offs[8]);
  bt.nslots = (uint32_t)ns;
  bt.small_limit = cfg.small_limit > 0 ? (uint32_t)cfg.small_limit : SMALL_LIMIT;
  if ((e = hipHostMalloc((void**)&h_games, sizeof(DevGame) * ns, hipHostMallocDefault))) return bad("pinned", e);
  if ((e = hipHostMalloc((void**)&h_words, 16 * ns, hipHostMallocDefault))) return bad("pinned", e);
  if ((e = hipHostMalloc((void**)&h_state, 4 * ns, hipHostMallocDefault))) return bad("pinned", e);
  if ((e = hipHostMalloc((void**)&h_mode, 4 * ns, hipHostMallocDefault))) return bad("pinned", e);
  for (size_t i = 0; i < ns; i++) h_mode[i] = BM_DENSE;
  if ((e = hipHostMalloc((void**)&h_rounds, 4 * ns, hipHostMallocDefault))) return bad("pinned", e);
  if ((e = hipHostMalloc((void**)&h_st, 8 * S_WORDS * ns, hipHostMallocDefault))) return bad("pinned", e);
  slot_ticket.assign(ns, nullptr);
  for (int i = nslots - 1; i >= 0; i--) free_slots.push_back(i);
  // Every epoch graph the worker uses (1, 2, 4, ..., 64 epochs) is captured
  // here, on the creating thread and before the worker starts: HIP refuses a
  // device-wide synchronization on any thread while some stream captures, so
  // a capture on the worker could fail the caller's own calls.
  for (int k = 1; k <= 64; k *= 2)
    if (!graph_for(k)) return bad("epoch graph capture", hipErrorUnknown);
  return true;
}

void Server::release_device() {
  if (main) (void)hipStreamSynchronize(main);
  if (side) (void)hipStreamSynchronize(side);
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
  arena.release();
  if (table_mem) (void)hipFree(table_mem);
  if (h_games) (void)hipHostFree(h_games);
  if (h_words) (void)hipHostFree(h_words);
  if (h_state) (void)hipHostFree(h_state);
  if (h_mode) (void)hipHostFree(h_mode);
  if (h_rounds) (void)hipHostFree(h_rounds);
  if (h_st) (void)hipHostFree(h_st);
  if (ev_upload) (void)hipEventDestroy(ev_upload);
  if (ev_main) (void)hipEventDestroy(ev_main);
  if (ev_side) (void)hipEventDestroy(ev_side);
  if (ev_g0) (void)hipEventDestroy(ev_g0);
  if (ev_g1) (void)hipEventDestroy(ev_g1);
  if (main) (void)hipStreamDestroy(main);
  if (side) (void)hipStreamDestroy(side);
  table_mem = nullptr;
  main = side = nullptr;
}

// K epochs captured once and replayed (kernels only: the graph holds no memset).
hipGraphExec_t Server::graph_for(int k) {
  auto it = graphs.find(k);
  if (it != graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  for (int i = 0; i < k; i++) (void)launch_epoch(bt, grid, main);
  if (hipStreamEndCapture(main, &g) != hipSuccess) return nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
  (void)hipGraphDestroy(g);
  if (ex) graphs[k] = ex;
  return ex;
}

// Upload one pending game into a free slot and publish it for the next epoch.
// Returns 1 when admitted, 0 when no slot or arena range is free, -1 when the
// device failed (the ticket is then consumed with an error).
int Server::admit_one(Ticket* t) {
  if (free_slots.empty()) return 0;
  const size_t off = arena.alloc(t->footprint);
  if (off == SIZE_MAX) return 0;
  const int slot = free_slots.back();
  free_slots.pop_back();
  t->slot = slot;
  t->arena_off = off;
  char* base = arena.base() + off;
  const int vbits = t->prep.info.value_bits;
  const size_t nblk = (size_t)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)t->n + TILE_VERTICES - 1) / TILE_VERTICES));
  const bool filter = cfg.p1_filter != 0;
  const GameLayout L = plan_layout(t->n, t->m, vbits, nblk, 1, filter);
  DevGame& dg = t->dg;
  bind_layout(dg, base, L, t->n, t->m, vbits, 1, filter);
  dg.bound = t->prep.info.bound;
  dg.top = dg.bound + t->prep.clamp + 1;
  dg.lanes_ok = lanes_ok_for(t->n, t->m, vbits);
  t->out64 = (int64_t*)(base + L.off[L_OUT]);
  eg_game_desc d{t->n, t->m, t->off.data(), t->tgt.data(), t->w.data(), t->own.data(), t->W, EG_MEM_HOST};
  void* staging = base + align_up(L.total);
  hipError_t e = upload_game(&d, t->prep, dg, staging, side, nullptr);
  if (!e) e = hipEventRecord(ev_upload, side);
  if (!e) e = hipStreamWaitEvent(main, ev_upload, 0);
  if (!e) e = hipMemsetAsync(dg.ctrl, 0, 4 * C_WORDS, main);
  if (!e) e = launch_init(dg, vbits, 0, (int)nblk, main);
  if (!e && cfg.top_seeding) {
    // one seeding pass before the first round; its scratch is the staging
    // part of the range, free once the upload (side stream) has completed
    SeedBuf sb{};
    bind_seed(sb, staging, t->n);
    e = launch_seed(dg, vbits, sb, 1, true, 1, main);  // f was just set to 0; one choice pass
  }
  // publish: descriptor, zero counters, mode and first round, then the state
  h_games[slot] = dg;
  h_words[4 * slot] = SLOT_RUN;
  h_words[4 * slot + 1] = BM_DENSE;
  h_words[4 * slot + 2] = 1;
  if (!e) e = hipMemcpyAsync((void*)(bt.games + slot), &h_games[slot], sizeof(DevGame), hipMemcpyHostToDevice, main);
  if (!e) e = hipMemsetAsync(bt.st + (size_t)slot * S_WORDS, 0, 8 * S_WORDS, main);
  if (!e) e = hipMemcpyAsync(bt.mode + slot, &h_words[4 * slot + 1], 4, hipMemcpyHostToDevice, main);
  if (!e) e = hipMemcpyAsync(bt.round + slot, &h_words[4 * slot + 2], 4, hipMemcpyHostToDevice, main);
  if (!e) e = hipMemcpyAsync(bt.state + slot, &h_words[4 * slot], 4, hipMemcpyHostToDevice, main);
  // the staging part of the game's range is free once the side stream is done
  if (!e) e = hipStreamSynchronize(side);
  if (e) {
    t->error = EG_EDEVICE;
    free_slots.push_back(slot);
    arena.free(off);
    t->slot = -1;
    return -1;
  }
  slot_ticket[slot] = t;
  h_mode[slot] = BM_DENSE;
  nrunning++;
  t->t_admit = now_s();
  return 1;
}

// Copy a finished game's result into its ticket (or drop a cancelled one) and free its slot.
void Server::retire(int slot, bool finished) {
  Ticket* t = slot_ticket[slot];
  hipError_t e = hipSuccess;
  h_words[4 * slot] = SLOT_FREE;
  e = hipMemcpyAsync(bt.state + slot, &h_words[4 * slot], 4, hipMemcpyHostToDevice, main);
  if (finished) {
    t->credits.resize((size_t)t->n);
    if (!e) e = launch_output(t->dg, t->dg.vbits, t->out64, main);
    if (!e) e = hipMemcpyAsync(t->credits.data(), t->out64, 8 * (size_t)t->n, hipMemcpyDeviceToHost, main);
    if (!e) e = hipMemcpyAsync(h_st + (size_t)slot * S_WORDS, bt.st + (size_t)slot * S_WORDS, 8 * S_WORDS,
                               hipMemcpyDeviceToHost, main);
  }
  if (!e) e = hipStreamSynchronize(main);
  arena.free(t->arena_off);
  slot_ticket[slot] = nullptr;
  free_slots.push_back(slot);
  nrunning--;
  std::lock_guard<std::mutex> lock(mu);
  t->slot = -1;
  if (!finished || stop) {
    t->state = T_CANCELLED;  // dropped, or its context is being destroyed
  } else if (e) {
    t->state = T_FAILED;
    t->error = EG_EDEVICE;
  } else {
    t->t_done = now_s();
    eg_stats& s = t->stats;
    memset(&s, 0, sizeof s);
    s.rounds = h_rounds[slot];
    s.lifts = h_st[slot * S_WORDS + S_LIFTS];
    s.relaxed_edges = h_st[slot * S_WORDS + S_EDGES];
    s.pushes = h_st[slot * S_WORDS + S_PUSHES];
    s.changes = h_st[slot * S_WORDS + S_CHANGES];
    s.scanned_preds = h_st[slot * S_WORDS + S_SCANNED];
    s.filtered_preds = h_st[slot * S_WORDS + S_FILTERED];
    s.t_solve = t->t_done - t->t_admit;
    s.t_queue = t->t_admit - t->t_arrive;
    s.t_latency = t->t_done - t->t_arrive;
    t->state = T_DONE;
    // the host copy of the game is no longer needed
    std::vector<int64_t>().swap(t->off);
    std::vector<int32_t>().swap(t->tgt);
    std::vector<int32_t>().swap(t->w);
    std::vector<uint8_t>().swap(t->own);
  }
  cv.notify_all();
}

void Server::run() {
  (void)hipSetDevice(cfg.device);
  int k = 1;
  for (;;) {
    std::vector<Ticket*> cands;
    std::vector<int> cancels;
    {
      std::unique_lock<std::mutex> lock(mu);
      cv.wait(lock, [&] { return stop || !pending.empty() || nrunning > 0; });
      if (stop) break;
      for (auto it = pending.begin(); it != pending.end();) {
        if ((*it)->cancel) {
          (*it)->state = T_CANCELLED;
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      for (size_t i = 0; i < pending.size() && i < free_slots.size(); i++) cands.push_back(pending[i]);
      for (int sl = 0; sl < nslots; sl++)
        if (slot_ticket[sl] && slot_ticket[sl]->cancel) cancels.push_back(sl);
    }
    for (int sl : cancels) retire(sl, false);
    // admissions in FIFO order: a game that does not fit holds back the ones behind it
    std::vector<int> outcome;
    for (Ticket* t : cands) {
      const int r = admit_one(t);
      if (r == 0) break;
      outcome.push_back(r);
    }
    if (!outcome.empty()) {
      std::lock_guard<std::mutex> lock(mu);
      for (int r : outcome) {
        Ticket* t = pending.front();
        pending.pop_front();
        if (t->state != T_CANCELLED) t->state = r > 0 ? T_RUNNING : T_FAILED;
      }
      cv.notify_all();
    }
    if (nrunning == 0) {
      k = 1;
      continue;
    }
    // k epochs for the games in the epochs and, beside them on the side
    // stream, many rounds of each game in small mode; then look for finished
    // games.  Slots change hands only through their mode word, and nothing
    // is admitted or retired while either stream runs.
    int in_epochs = 0;
    for (int sl = 0; sl < nslots; sl++) in_epochs += slot_ticket[sl] && h_mode[sl] == BM_DENSE;
    hipError_t e = hipEventRecord(ev_main, main);
    if (!e) e = hipStreamWaitEvent(side, ev_main, 0);
    if (!e && in_epochs) {
      hipGraphExec_t ex = graph_for(k);
      if (!e) e = hipEventRecord(ev_g0, main);
      if (!e) e = ex ? hipGraphLaunch(ex, main) : hipErrorUnknown;
      if (!e) e = hipEventRecord(ev_g1, main);
      epochs += (uint64_t)k;
    }
    // Games in small mode run beside the epochs for about as long as the
    // epochs take (a time budget on the device's 100 MHz realtime counter),
    // so that a game with a long tail of small rounds keeps its pace while
    // others fill the epochs; alone, 8192 rounds per launch.
    if (!e) {
      if (!in_epochs) e = launch_batch_small(bt, 8192u, 0, side);
      else if (epoch_us > 0) e = launch_batch_small(bt, 1u << 20, (uint64_t)(k * epoch_us * 100.0) + 1, side);
      else e = launch_batch_small(bt, 8u * (uint32_t)k, 0, side);
    }
    if (!e) e = hipEventRecord(ev_side, side);
    if (!e) e = hipStreamWaitEvent(main, ev_side, 0);
    if (!e) e = hipMemcpyAsync(h_state, bt.state, 4 * (size_t)nslots, hipMemcpyDeviceToHost, main);
    if (!e) e = hipMemcpyAsync(h_mode, bt.mode, 4 * (size_t)nslots, hipMemcpyDeviceToHost, main);
    if (!e) e = hipMemcpyAsync(h_rounds, bt.rounds, 4 * (size_t)nslots, hipMemcpyDeviceToHost, main);
    if (!e) e = hipStreamSynchronize(main);
    if (!e && in_epochs) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev_g0, ev_g1) == hipSuccess && ms > 0) {
        const double us = 1e3 * ms / k;
        epoch_us = epoch_us > 0 ? 0.75 * epoch_us + 0.25 * us : us;
      }
    }
    if (e) {
      std::lock_guard<std::mutex> lock(mu);
      device_error = std::string("batched iteration: ") + hipGetErrorString(e);
      for (int sl = 0; sl < nslots; sl++)
        if (slot_ticket[sl]) {
          slot_ticket[sl]->state = T_FAILED;
          slot_ticket[sl]->error = EG_EDEVICE;
          slot_ticket[sl] = nullptr;
        }
      for (Ticket* t : pending) {
        t->state = T_FAILED;
        t->error = EG_EDEVICE;
      }
      pending.clear();
      nrunning = 0;
      device_ok = false;
      cv.notify_all();
      break;
    }
    int finished = 0;
    for (int sl = 0; sl < nslots; sl++)
      if (slot_ticket[sl] && h_state[sl] == SLOT_DONE) {
        retire(sl, true);
        finished++;
      }
    bool waiting;
    {
      std::lock_guard<std::mutex> lock(mu);
      waiting = !pending.empty();
    }
    // shorter batches while games finish or wait, longer while nothing changes
    if (finished || waiting) k = std::max(1, k / 2);
    else k = std::min(64, k * 2);
  }
}

Server* server_create(const eg_config& cfg, hipStream_t) {
  Server* s = new Server();
  s->cfg = cfg;
  s->nslots = cfg.max_slots > 0 ? cfg.max_slots : 1024;
  s->max_pending = cfg.max_pending > 0 ? (size_t)cfg.max_pending : 65536;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg.device) != hipSuccess || cus <= 0)
    cus = 256;
  // the epoch kernel's grid: blocks_per_cu resident blocks on every compute unit
  s->grid = cus * (cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : 8);
  std::string why;
  s->device_ok = s->init_device(&why);
  if (!s->device_ok) {
    s->device_error = why;
    s->release_device();
    return s;
  }
  s->worker = std::thread([s] { s->run(); });
  return s;
}

void server_enter(Server* s) {
  std::lock_guard<std::mutex> lock(s->mu);
  s->users++;
}

void server_leave(Server* s) {
  std::lock_guard<std::mutex> lock(s->mu);
  if (--s->users == 0) s->cv.notify_all();
}

void server_destroy(Server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lock(s->mu);
    s->stop = true;
    // every ticket not yet finished fails with EG_ECANCELED; a thread blocked
    // in server_wait sees that and returns
    for (auto& kv : s->tickets) {
      Ticket* t = kv.second.get();
      if (t->state == T_PENDING || t->state == T_RUNNING) {
        t->cancel = true;
        t->state = T_CANCELLED;
      }
    }
    s->cv.notify_all();
    s->cv.wait(lock, [&] { return s->users == 0; });
  }
  if (s->worker.joinable()) s->worker.join();
  s->release_device();
  delete s;
}

int server_submit(Server* s, const eg_game_desc* desc, hipStream_t stream, eg_ticket* out) {
  {
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->device_ok) return set_err(EG_EDEVICE, s->device_error);
  }
  // device-pointer inputs are copied to the host here (the ticket keeps a
  // host copy of every game until it is admitted)
  HostCopy hc;
  eg_game_desc hd;
  int rc = host_view(desc, stream, hc, hd);
  if (rc != EG_OK) return rc;
  desc = &hd;
  auto t = std::make_unique<Ticket>();
  std::string why;
  rc = prepare(desc, s->cfg.bound_mode, nullptr, t->prep, &why, 0, 1);
  if (rc != EG_OK) return set_err(rc, why);
  t->n = desc->n;
  t->m = desc->m;
  t->W = desc->W;
  const size_t nblk = (size_t)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)desc->n + TILE_VERTICES - 1) / TILE_VERTICES));
  size_t scratch = staging_bytes(desc->n, desc->m, true, s->cfg.p1_filter != 0);
  if (s->cfg.top_seeding) scratch = std::max(scratch, seed_bytes(desc->n));
  t->footprint = align_up(plan_layout(desc->n, desc->m, t->prep.info.value_bits, nblk, 1, s->cfg.p1_filter != 0).total) +
                 scratch;
  if (t->footprint > s->arena.capacity())
    return set_err(EG_ENOMEM, "the game needs " + std::to_string(t->footprint) + " bytes, the HBM budget is " +
                                  std::to_string(s->arena.capacity()));
  t->off.assign(desc->offsets, desc->offsets + desc->n + 1);
  t->tgt.assign(desc->targets, desc->targets + desc->m);
  t->w.assign(desc->weights, desc->weights + desc->m);
  t->own.assign(desc->owner_bits, desc->owner_bits + ((size_t)desc->n + 7) / 8);
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->stop) return set_err(EG_ECANCELED, "the context is being destroyed");
  if (s->pending.size() >= s->max_pending) return set_err(EG_EBUSY, "the pending queue is full");
  t->id = s->next_id++;
  t->t_arrive = now_s();
  *out = t->id;
  s->pending.push_back(t.get());
  s->tickets[t->id] = std::move(t);
  s->cv.notify_all();
  return EG_OK;
}

static int poll_locked(Server* s, eg_ticket id, int64_t* credits, eg_stats* st);

int server_poll(Server* s, eg_ticket id, int64_t* credits, eg_stats* st) {
  std::lock_guard<std::mutex> lock(s->mu);
  return poll_locked(s, id, credits, st);
}

int server_wait(Server* s, eg_ticket id, int64_t* credits, eg_stats* st, double timeout_s) {
  std::unique_lock<std::mutex> lock(s->mu);
  auto ready = [&] {
    auto it = s->tickets.find(id);
    return it == s->tickets.end() || (it->second->state != T_PENDING && it->second->state != T_RUNNING);
  };
  if (timeout_s > 0) s->cv.wait_for(lock, std::chrono::duration<double>(timeout_s), ready);
  else s->cv.wait(lock, ready);
  return poll_locked(s, id, credits, st);
}

static int poll_locked(Server* s, eg_ticket id, int64_t* credits, eg_stats* st) {
  auto it = s->tickets.find(id);
  if (it == s->tickets.end()) return set_err(EG_ENOTFOUND, "unknown ticket " + std::to_string(id));
  Ticket* t = it->second.get();
  switch (t->state) {
    case T_PENDING:
    case T_RUNNING:
      return EG_PENDING;
    case T_DONE:
      if (credits) memcpy(credits, t->credits.data(), 8 * t->credits.size());
      if (st) *st = t->stats;
      s->tickets.erase(it);
      return EG_OK;
    case T_CANCELLED:
      s->tickets.erase(it);
      return set_err(EG_ECANCELED, "ticket " + std::to_string(id) + " was cancelled");
    default: {
      const int err = t->error ? t->error : EG_EDEVICE;
      s->tickets.erase(it);
      return set_err(err, "ticket " + std::to_string(id) + " failed: " + s->device_error);
    }
  }
}

int server_cancel(Server* s, eg_ticket id) {
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->tickets.find(id);
    if (it == s->tickets.end()) return set_err(EG_ENOTFOUND, "unknown ticket " + std::to_string(id));
    Ticket* t = it->second.get();
    if (t->state != T_PENDING && t->state != T_RUNNING)
      return set_err(EG_EINVAL, "ticket " + std::to_string(id) + " has already finished");
    t->cancel = true;
  }
  s->cv.notify_all();
  return EG_OK;
}

}  // namespace eg
