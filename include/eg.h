/*
 * libeg: minimum initial credits of energy games on AMD MI355X (gfx950).
 *
 * Problem (Formisano, Gentilini, Vella, arXiv 1710.03647, Sec. 3, Def. 4):
 * given a total weighted arena (every vertex has an out-edge, Sec. 2) whose
 * vertices are split between player 0 and player 1, compute for each vertex v
 * whether player 0 wins from v and, if so, the least initial credit c(v) that
 * keeps every prefix energy level non-negative (Eq. (1), Def. 3).
 *
 * Method: the least energy progress measure (Sec. 3.1, Def. 5) computed by
 * repeated application of the lifting operator of Def. 6,
 *     f(v) <- min (player 0) / max (player 1) over edges (v,u) of f(u) (-) w(v,u),
 * where a (-) b = max(0, a - b) and TOP (-) b = TOP, starting from f = 0.  Values
 * above the bound B become TOP; B = (n-1)*W by default, or M_G (Sec. 3.1).  The
 * device iteration follows the frontier scheme of Alg. 3: each round lifts the
 * active vertices in parallel, in place, and the predecessors of every vertex
 * whose value changed form the next active set (while that set covers about
 * every vertex, rounds lift every vertex instead).  Optionally, cycles that
 * player 1 can force with negative weight are set to TOP between rounds
 * (Lemma 1), which changes the work but not the result.  All arithmetic is
 * integer, so the result equals the sequential worklist of Alg. 1 bit for bit.
 *
 * Output: credits[v] = c(v) for v won by player 0, EG_TOP for v won by player 1.
 *
 * Conventions for every function:
 *  - return EG_OK (0) on success, a negative EG_E* code on failure; nothing
 *    throws across this boundary;
 *  - on failure eg_last_error() returns a message for the calling thread;
 *  - every input array is copied before the call returns (the caller keeps
 *    ownership); output arrays are caller-owned and written in full on EG_OK
 *    (and on EG_ETIMEDOUT, see eg_solve).
 */
#ifndef EG_H
#define EG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EG_TOP INT64_MAX /* credit of a vertex won by player 1 (TOP); keeps the order of Sec. 3.1 */

enum {
  EG_OK = 0,
  EG_PENDING = 1,     /* eg_poll: the game is not finished yet */
  EG_EINVAL = -1,     /* malformed arguments or arena (see eg_check) */
  EG_ENOMEM = -2,     /* device memory or the context's HBM budget cannot hold the game */
  EG_EDEVICE = -3,    /* a HIP call failed */
  EG_ETIMEDOUT = -4,  /* the round or time budget ran out; credits hold a lower bound */
  EG_EBUSY = -5,      /* eg_submit: the pending queue is full */
  EG_ENOTFOUND = -6,  /* unknown or already retired ticket */
  EG_ECANCELED = -7   /* the ticket was cancelled, or its context destroyed */
};

enum { EG_BOUND_NW = 0, /* B = (n-1)*W */ EG_BOUND_MG = 1 /* B = M_G of Sec. 3.1 */ };
enum { EG_MEM_HOST = 0, EG_MEM_DEVICE = 1 };

typedef struct eg_ctx eg_ctx;
typedef struct eg_game eg_game;
typedef uint64_t eg_ticket;

/* Context configuration.  Zero-initialise and set what is needed. */
typedef struct {
  int device;                /* HIP device ordinal */
  void* hip_stream;          /* hipStream_t used by eg_create/eg_solve; NULL = the context's own */
  uint64_t hbm_budget_bytes; /* serving: device bytes the admitted games may hold; 0 = a quarter of the
                                free device memory (at most the free memory less 1 GiB) */
  int max_slots;             /* serving: games resident at once; 0 = 1024 */
  int bound_mode;            /* EG_BOUND_NW or EG_BOUND_MG */
  uint64_t max_rounds;       /* eg_solve round budget; 0 = none */
  double time_budget_s;      /* eg_solve wall-clock budget; 0 = none */
  int max_pending;           /* serving: queue cap of eg_submit; 0 = 65536 */
  int partition;             /* dense rounds over a copy of the edges grouped by target slice
                                (n <= 2^22; 8 bytes per edge more device memory): 0 or 1 = never;
                                2 = every dense round, one slice per XCD, per-slice partial keys;
                                3 = slice-major: all-vertex rounds and dense rounds that lift about
                                half of V or more sweep slices of about 1 MB of f in order, all
                                blocks at about the same slice, keys held in LDS (the other rounds
                                stay in place).  Sliced rounds are synchronous: cheaper per round,
                                possibly more rounds */
  /* launch shape (0 = defaults; set by the autotuner) */
  int blocks_per_cu;         /* resident blocks of 256 threads per compute unit in round kernels: 8 */
  int dense_div;             /* flag sweeps while the active set holds >= n / dense_div vertices: 32 */
  int small_limit;           /* one block runs the rounds while the active set holds <= this: 1024 */
  int top_seeding;           /* 1 = set TOP on the vertices of negative cycles that player 1 can force
                                (Lemma 1): eg_solve runs such a pass before the first round and again
                                at doubling round counts; serving (eg_submit, eg_solve_batch) runs one
                                before each game's first round (its device footprint then includes
                                34 bytes per vertex of scratch).  The pass follows one chosen edge per
                                player-1 vertex (the largest term).  k in 2..64 = eg_solve's passes
                                first run k Bellman-Ford passes over the forced subgraph (player-1
                                vertices and out-degree-1 player-0 vertices, values from f, one more
                                value per vertex of device memory), so that the choice follows the
                                best paths found and finds negative cycles off the first choice;
                                values above B also prove TOP.  Serving and
                                eg_solve_seeded_noalloc run the one-choice pass.  Exact: the credits
                                do not change, only the work (0..64) */
  int seg_edges;             /* launch shape: dense rounds cut a tile of 256 vertices whose out-degrees
                                sum above this into segments taken by different blocks: 8192
                                (0 = default, -1 = never cut; else >= 256) */
  int relabel;               /* eg_create: renumber vertices internally by decreasing in-degree so the
                                most gathered values share cache lines: 0 = when the largest
                                in-degree is >= 64x the average (n >= 4096) and dense rounds are
                                unsliced with tiles cut, 1 = never, 2 = always; credits are always
                                returned in the caller's numbering */
  int p1_filter;             /* 1 = the player-1 frontier filter (Alg. 1's predecessor test, Sec. 3.1):
                                when v's value rises, a player-1 predecessor p joins the next active set
                                only if f(p) < f(v) (-) w(p, v) (every player-0 predecessor still joins,
                                as in Alg. 3).  Exact under the in-place parallel updates (values only
                                rise, so a satisfied test stays satisfied until f(v) rises again, which
                                tests again); the credits do not change, only the work.  Costs 4 bytes
                                per edge of device memory (the weights of the predecessor lists) */
  int scc_schedule;          /* 1 = the component schedule (the refinement proposed in Sec. 6): eg_solve
                                first finds the strongly connected components of the game graph and the
                                levels of their condensation (once per game, 21 bytes per vertex of device
                                memory), then solves level by level from the sink components up, each
                                level from all of its vertices, with predecessors on higher levels kept
                                out of the active set until their level starts.  Exact (a level's
                                successors outside it are already at their least-fixpoint values); the
                                credits do not change, only the work.  eg_solve only (not serving) */
  int hub_cache;             /* launch shape: the cut-tile rounds of a game renumbered by in-degree read
                                the values of its first vertices (the most gathered ones) from a copy
                                in LDS taken at the start of each round: its size in KB (1 to 64;
                                0 = 16), or -1 = off */
} eg_config;

/* A game in CSR form.  Out-edges of v are e in [offsets[v], offsets[v+1]),
 * going to targets[e] with weight weights[e] (a multiset: duplicate edges and
 * self-loops are allowed).  owner_bits is LSB-first, bit v = 1 when v belongs
 * to player 1 (max).  W must satisfy W >= max(0, max_e -weights[e]).
 * mem = EG_MEM_HOST: host pointers.  mem = EG_MEM_DEVICE: device pointers valid
 * on the context's stream until the call returns. */
typedef struct {
  int32_t n;
  int64_t m;
  const int64_t* offsets;    /* n+1 entries, offsets[0] = 0, offsets[n] = m, non-decreasing */
  const int32_t* targets;    /* m entries in [0, n) */
  const int32_t* weights;    /* m entries */
  const uint8_t* owner_bits; /* ceil(n/8) bytes */
  int32_t W;
  int mem;
} eg_game_desc;

/* Counters and times of one solve. */
typedef struct {
  uint64_t rounds;        /* rounds of the frontier iteration that had a non-empty active set */
  uint64_t lifts;         /* applications of the lifting operator */
  uint64_t relaxed_edges; /* out-edges read by those lifts (GTEPS = relaxed_edges / t_solve) */
  uint64_t pushes;        /* insertions into the next active set */
  uint64_t changes;       /* lifts that raised a value */
  uint64_t scanned_preds; /* predecessor-list entries read after those changes */
  double t_upload;        /* eg_create: host-to-device copy and layout, seconds */
  double t_rcsr;          /* eg_create: reverse CSR (predecessor lists) build, seconds */
  double t_solve;         /* eg_solve: from the init launch to the fixpoint, seconds */
  double t_d2h;           /* eg_solve: result conversion and device-to-host copy, seconds */
  double model_bytes;     /* algorithmic bytes moved by the solve (see eg_solve_ex) */
  double achieved_gbps;   /* model_bytes / t_solve / 1e9 */
  double t_round_kernels; /* device time of the round kernels alone, seconds */
  double t_queue;         /* eg_poll: submission to admission, seconds */
  double t_latency;       /* eg_poll: submission to result, seconds */
  uint64_t launched_rounds; /* round kernels launched (empty ones after the fixpoint included) */
  uint64_t dense_rounds;  /* of which in the dense representation */
  uint64_t seeded;        /* vertices set to TOP by seeding passes (top_seeding) */
  uint64_t seed_passes;   /* seeding passes run */
  uint64_t all_rounds;    /* dense rounds that lifted every vertex without activating (frontier ~ V) */
  double t_seed;          /* eg_solve: device time of the seeding passes (top_seeding), seconds */
  uint64_t filtered_preds; /* predecessor entries the player-1 frontier filter kept out (p1_filter) */
  uint64_t scc_components; /* scc_schedule: strongly connected components of the game graph */
  uint64_t scc_levels;     /* scc_schedule: levels of the condensation (sink components are level 0) */
  double t_scc;            /* scc_schedule: wall time of finding them (first solve of the game only), seconds */
  double t_slices;         /* eg_create: the edge copy grouped by target slice (partition 2 or 3), seconds */
} eg_stats;

/* What eg_check derives from a valid game. */
typedef struct {
  int32_t n;
  int64_t m;
  int64_t bound;           /* B */
  int value_bits;          /* 32 or 64: device storage of f */
  uint64_t device_bytes;   /* device footprint of the game */
  int32_t max_outdeg;
  int32_t max_indeg;
} eg_game_info;

/* Per-call options of eg_solve_ex. */
typedef struct {
  uint64_t max_rounds;    /* 0 = the context's budget */
  double time_budget_s;   /* 0 = the context's budget */
  int resume;             /* 0: start from f = 0 with the initial active set of Alg. 3.
                             1: start from the game's current f with every vertex active
                                (any f below the least fixpoint reaches it). */
  int driver;             /* reserved: must be 0 (EG_EINVAL otherwise) */
} eg_solve_opts;

/* Create a context on cfg->device (NULL cfg = all defaults).  Returns EG_EDEVICE
 * when HIP cannot use the device. */
int eg_ctx_create(const eg_config* cfg, eg_ctx** out);

/* Destroy a context.  Every pending or running ticket fails with EG_ECANCELED:
 * a thread blocked in eg_wait on one returns EG_ECANCELED, and serving calls in
 * progress on other threads return before the context is freed.  A solve in
 * progress finishes first.  Then the serving thread stops and every game
 * created in the context that is still alive is freed (its handle must not be
 * used afterwards, eg_destroy included).  Calls that start after this one has
 * returned are undefined: the context no longer exists. */
int eg_ctx_destroy(eg_ctx* ctx);

/* Validate a game without touching a device (host pointers only).  EG_EINVAL
 * when: n < 1; m < 0 or m >= 2^31; offsets not starting at 0, not ending at m,
 * or decreasing; a target outside [0, n); a vertex without out-edges (the arena
 * is not total, Sec. 2); W < max(0, max -w); a null pointer.  info may be NULL. */
int eg_check(const eg_game_desc* desc, int bound_mode, eg_game_info* info, char* msg, size_t msg_len);

/* Validate (as eg_check), copy the game to the device, lay it out and build
 * its predecessor lists (the paper's CSC, Sec. 5).  Synchronises the context's
 * stream.  stats (nullable) receives t_upload and t_rcsr. */
int eg_create(eg_ctx* ctx, const eg_game_desc* desc, eg_game** out, eg_stats* stats);

/* Free a game's device memory.  EG_EINVAL for a game that is not alive in its
 * context. */
int eg_destroy(eg_game* g);

/* Solve one game to the least fixpoint and copy credits (n entries,
 * caller-owned host memory; NULL = keep the result on the device only).
 * Blocks until done.  EG_ETIMEDOUT when a budget ran out: credits then hold the
 * current measure, a lower bound of the least one (TOP only where proven).
 * stats is nullable.  Calls on one context are serialised. */
int eg_solve(eg_game* g, int64_t* credits, eg_stats* stats);

/* eg_solve with per-call options (NULL opts = eg_solve). */
int eg_solve_ex(eg_game* g, const eg_solve_opts* opts, int64_t* credits, eg_stats* stats);

/* For callers that cannot allocate device memory during a solve (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * eg_solve_ex with TOP seeding on (whatever the context's top_seeding says),
 * whose seeding scratch is a static device array of the library instead of
 * memory allocated by the first seeded solve.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the game, its
 * buffers and the pinned host words it uses were allocated by eg_create.  The
 * array holds the scratch of games up to EG_NOALLOC_MAX_N vertices (34 bytes
 * per vertex, 136 MiB in all); each device holds its own copy from its first
 * such call until the process ends.  Every call on one device uses that
 * device's copy, so calls on one device are serialised (a call waits while
 * another, from any context, runs); every scratch word a pass reads is written
 * by that pass first, so no state carries over between calls.  EG_EINVAL
 * when g has more than EG_NOALLOC_MAX_N vertices; otherwise as eg_solve_ex,
 * with the same credits. */
#define EG_NOALLOC_MAX_N (1 << 22)
int eg_solve_seeded_noalloc(eg_game* g, const eg_solve_opts* opts, int64_t* credits, eg_stats* stats);

/* Replace the game's current measure (n entries, host memory, EG_TOP allowed)
 * before an eg_solve_ex with resume = 1.  EG_EINVAL if a finite value is
 * negative or above the bound. */
int eg_set_measure(eg_game* g, const int64_t* f);

/* Player 0's positional winning strategy (Def. 4 item 2, Def. 5, Lemma 1),
 * read off the least progress measure that the last eg_solve of g reached
 * (a resumed solve that started above it stops at a larger fixpoint, which
 * is still a progress measure: the strategy then wins with that credit).
 * choice (n entries, caller-owned host memory): for a player-0 vertex v with
 * finite credit, the index k within v's out-edges (the edge offsets[v] + k of
 * the caller's arrays) of the first edge (v, u) with f(v) >= f(u) (-) w(v, u);
 * -1 for player-1 vertices and for vertices of W1 (credit EG_TOP).  Played
 * from v with initial credit f(v), these edges keep the energy >= 0 against
 * every player-1 strategy.  t_kernel (nullable) receives the kernel time in
 * seconds.  EG_EINVAL unless the last eg_solve / eg_solve_ex of g returned
 * EG_OK with no eg_set_measure since; EG_EDEVICE if some player-0 vertex with
 * finite credit has no such edge (the measure is not a fixpoint).  Serialised
 * with the solves of the context. */
int eg_strategy(eg_game* g, int32_t* choice, double* t_kernel);

/* The strongly connected components of the game graph and the levels of their
 * condensation, the order of the component schedule (the refinement proposed
 * in Sec. 6; see eg_config.scc_schedule), computed on the device at the first
 * call or schedule solve of g and kept with the game (21 bytes per vertex).
 * comp, level (n entries each, caller-owned host memory, caller's numbering):
 * comp[v] labels v's component (two vertices share a label exactly when each
 * reaches the other; labels are vertex ids of the device numbering, so they
 * equal the caller's ids only for games that are not renumbered); level[v] is
 * 0 for components with no edge leaving them, else one more than the largest
 * level among the components that v's component has edges into.  components,
 * levels (nullable): their counts.  EG_EINVAL on a null game or array.
 * Serialised with the solves of the context. */
int eg_components(eg_game* g, int32_t* comp, int32_t* level, uint32_t* components, uint32_t* levels);

/* Serving.  eg_submit copies the game into the context's pending queue and
 * returns at once with a ticket (EG_EBUSY if the queue is full, EG_EINVAL for
 * a malformed game, EG_ENOMEM if the game cannot fit even an empty budget).
 * A serving thread admits pending games while their device footprint fits the
 * HBM budget and a slot is free, and runs all admitted games together in one
 * batched device iteration; a game that arrives while others run joins them at
 * the next round.  eg_poll returns EG_OK with the credits (n entries) once the
 * game is done (the ticket is then retired), EG_PENDING before, or the
 * ticket's error.  eg_cancel drops a pending or running ticket.
 * eg_submit takes host or device pointers (desc->mem); device arrays are read
 * on the context's stream, which the call synchronises, and may be freed once
 * it returns.  After eg_ctx_destroy has started, eg_submit returns
 * EG_ECANCELED. */
int eg_submit(eg_ctx* ctx, const eg_game_desc* desc, eg_ticket* out);
int eg_poll(eg_ctx* ctx, eg_ticket t, int64_t* credits, eg_stats* stats);
int eg_cancel(eg_ctx* ctx, eg_ticket t);

/* As eg_poll, but blocks until the ticket is finished or timeout_s seconds
 * have passed (then EG_PENDING; timeout_s <= 0 waits without limit). */
int eg_wait(eg_ctx* ctx, eg_ticket t, int64_t* credits, eg_stats* stats, double timeout_s);

/* Batching: solve `count` games together in the batched device iteration
 * (resident games advance one round per launch together, or many rounds per
 * launch on their own once their active set is small; each is retired at its
 * own fixpoint) and block until all are done.  credits[i] receives game i's n
 * credits; stats (nullable) count entries.  The games must fit the context's
 * HBM budget one at a time; they are admitted as room frees up. */
int eg_solve_batch(eg_ctx* ctx, const eg_game_desc* games, int count, int64_t* const* credits, eg_stats* stats);

/* Message of the last failure on the calling thread ("" if none). */
const char* eg_last_error(eg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* EG_H */
