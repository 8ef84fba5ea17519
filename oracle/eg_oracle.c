/*
 * CPU oracle for the minimum-initial-credit problem on energy games
 * (Formisano, Gentilini, Vella, "Accelerating Energy Games Solvers on Modern
 * Architectures", arXiv 1710.03647).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this code.  It shares no code, header,
 * table or helper with the device solver; it builds its own predecessor lists.
 *
 * What it computes: the least energy progress measure f (Sec. 3.1, Def. 5 and
 * the properties listed after it), obtained by applying the lifting operator of
 * Def. 6 from the constant-0 function until nothing changes.  f(v) is the
 * minimum initial credit of v when finite, and TOP exactly on the vertices won
 * by player 1.
 *
 * Values live in N u {TOP}; TOP is represented by INT64_MAX, which keeps the
 * total order of Sec. 3.1 (x <= y iff x <= y as integers, or y = TOP) equal to
 * the integer order.  The codomain C_G holds the naturals up to a bound plus TOP
 * (Sec. 3.1); a value above the bound is TOP.  The bound is (n-1)*W by default
 * (mode 0), M_G = sum over v of max(0, max_e -w(e)) as printed in Sec. 3.1
 * (mode 1), or a caller-given value (mode 2).
 *
 * Iteration orders (all reach the same least fixpoint, since every one applies
 * the same monotone operator starting below it):
 *   ORC_FIFO   worklist taken first-in first-out (default).  Initial list as in
 *              Alg. 1 / Alg. 3 (player-0 vertices whose out-edges are all
 *              negative, player-1 vertices with some negative out-edge), in
 *              ascending id order; after a lift that changes f(v), every
 *              predecessor of v not already queued is appended (Alg. 3).
 *   ORC_LIFO   the same worklist taken last-in first-out.
 *   ORC_RANDOM the same worklist, element picked at random (seeded).
 *   ORC_JACOBI Alg. 2: sweep over all of V computing every new value from the
 *              previous sweep's values, until a sweep changes nothing.
 *   ORC_ROUNDS Alg. 3 run sequentially: rounds over the list L, lifts in place,
 *              L' = predecessors of the changed vertices (each once per round).
 *   ORC_ALG1   Alg. 1 with its per-vertex counters of satisfied out-edges for
 *              player-0 vertices and its predecessor filter.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TOP INT64_MAX

enum { ORC_FIFO = 0, ORC_LIFO = 1, ORC_RANDOM = 2, ORC_JACOBI = 3, ORC_ROUNDS = 4, ORC_ALG1 = 5 };

typedef struct {
  uint64_t lifts;          /* applications of the lifting operator */
  uint64_t relaxed_edges;  /* out-edges read by those lifts */
  uint64_t pushes;         /* insertions into the worklist */
  uint64_t changes;        /* lifts that raised f(v) */
  uint64_t rounds;         /* sweeps (Jacobi) or rounds (Alg. 3); 0 otherwise */
  int64_t bound;           /* the bound actually used */
} orc_stats;

/* a (-) b of Sec. 3.1: max(0, a - b) for finite a, TOP for TOP. */
static int64_t ominus(int64_t a, int64_t b) {
  if (a == ORC_TOP) return ORC_TOP;
  int64_t d = a - b;
  return d > 0 ? d : 0;
}

/* Membership in C_G: a finite value above the bound is TOP. */
static int64_t clamp_to_codomain(int64_t a, int64_t bound) {
  if (a != ORC_TOP && a > bound) return ORC_TOP;
  return a;
}

/* Def. 6: the value that delta(f, v) gives to v; reads f only. */
static int64_t lift_value(int32_t v, const int64_t *off, const int32_t *tgt, const int32_t *w,
                          const uint8_t *owner, const int64_t *f, int64_t bound) {
  int64_t acc = 0;
  int first = 1;
  for (int64_t e = off[v]; e < off[v + 1]; e++) {
    int64_t t = clamp_to_codomain(ominus(f[tgt[e]], (int64_t)w[e]), bound);
    if (first) {
      acc = t;
      first = 0;
    } else if (owner[v] == 0) {
      if (t < acc) acc = t; /* player 0: min */
    } else {
      if (t > acc) acc = t; /* player 1: max */
    }
  }
  return acc;
}

static uint64_t splitmix_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The bound of the codomain for the requested mode. */
int64_t orc_bound(int32_t n, const int64_t *off, const int32_t *w, int32_t W, int bound_mode,
                  int64_t explicit_bound) {
  if (bound_mode == 2) return explicit_bound;
  if (bound_mode == 1) {
    int64_t mg = 0;
    for (int32_t v = 0; v < n; v++) {
      int64_t worst = 0;
      for (int64_t e = off[v]; e < off[v + 1]; e++)
        if (-(int64_t)w[e] > worst) worst = -(int64_t)w[e];
      mg += worst;
    }
    return mg;
  }
  return (int64_t)(n - 1) * (int64_t)W;
}

/* Does v enter the initial list (Alg. 1 lines 1-2, Alg. 3 line 3)? */
static int initially_active(int32_t v, const int64_t *off, const int32_t *w, const uint8_t *owner) {
  int all_neg = 1, some_neg = 0;
  for (int64_t e = off[v]; e < off[v + 1]; e++) {
    if (w[e] < 0) some_neg = 1;
    else all_neg = 0;
  }
  return owner[v] == 0 ? all_neg : some_neg;
}

/*
 * Solve.  Inputs: CSR arena (off[n+1], tgt[m], w[m]), owner[v] in {0,1}
 * (1 = player 1), W >= max(0, max -w).  f_init (nullable): start from this
 * measure (TOP = INT64_MAX) with every vertex queued, instead of from 0 with the
 * initial list.  max_lifts: stop after this many lifts (0 = no limit).
 * Output f_out[n] (TOP = INT64_MAX).  Returns 0 at the fixpoint, 1 if stopped by
 * max_lifts (f_out is then the current, lower, measure), -1 on allocation failure.
 */
int orc_solve(int32_t n, const int64_t *off, const int32_t *tgt, const int32_t *w,
              const uint8_t *owner, int32_t W, int bound_mode, int64_t explicit_bound, int order,
              uint64_t seed, const int64_t *f_init, uint64_t max_lifts, int64_t *f_out,
              orc_stats *st) {
  orc_stats s;
  memset(&s, 0, sizeof s);
  const int64_t m = off[n];
  const int64_t bound = orc_bound(n, off, w, W, bound_mode, explicit_bound);
  s.bound = bound;
  int64_t *f = f_out;
  for (int32_t v = 0; v < n; v++) f[v] = f_init ? f_init[v] : 0;

  /* predecessor lists, one entry per edge (duplicates and self-loops kept) */
  int64_t *poff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *psrc = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int64_t *pedge = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t) + 4);
  uint8_t *inq = (uint8_t *)calloc((size_t)n, 1);
  int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *prev = (int64_t *)malloc((size_t)n * sizeof(int64_t) + 8);
  if (!poff || !psrc || !pedge || !fill || !queue || !inq || !cnt || !prev) {
    free(poff); free(psrc); free(pedge); free(fill); free(queue); free(inq); free(cnt); free(prev);
    return -1;
  }
  for (int32_t v = 0; v < n; v++)
    for (int64_t e = off[v]; e < off[v + 1]; e++) poff[tgt[e] + 1]++;
  for (int32_t u = 0; u < n; u++) poff[u + 1] += poff[u];
  for (int32_t v = 0; v < n; v++)
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int32_t u = tgt[e];
      int64_t slot = poff[u] + fill[u]++;
      psrc[slot] = v;
      pedge[slot] = e;
    }

  int status = 0;
  uint64_t rng = seed;

  if (order == ORC_JACOBI) {
    /* Alg. 2: every vertex lifted from the previous sweep's values */
    int more = 1;
    while (more) {
      if (max_lifts && s.lifts + (uint64_t)n > max_lifts) { status = 1; break; }
      more = 0;
      memcpy(prev, f, (size_t)n * sizeof(int64_t));
      for (int32_t v = 0; v < n; v++) {
        int64_t nv = lift_value(v, off, tgt, w, owner, prev, bound);
        s.lifts++;
        s.relaxed_edges += (uint64_t)(off[v + 1] - off[v]);
        if (nv != prev[v]) { f[v] = nv; s.changes++; more = 1; }
      }
      s.rounds++;
    }
  } else if (order == ORC_ROUNDS) {
    /* Alg. 3 executed sequentially: L' collects pre(v) of each changed v */
    int32_t *next = (int32_t *)malloc((size_t)n * sizeof(int32_t) + 4);
    uint64_t *stamp = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    if (!next || !stamp) { free(next); free(stamp); status = -1; goto done; }
    int64_t len = 0;
    for (int32_t v = 0; v < n; v++)
      if (f_init || initially_active(v, off, w, owner)) { queue[len++] = v; s.pushes++; }
    uint64_t r = 0;
    while (len > 0) {
      int64_t nlen = 0;
      r++;
      for (int64_t i = 0; i < len; i++) {
        if (max_lifts && s.lifts >= max_lifts) { status = 1; break; }
        int32_t v = queue[i];
        int64_t nv = lift_value(v, off, tgt, w, owner, f, bound);
        s.lifts++;
        s.relaxed_edges += (uint64_t)(off[v + 1] - off[v]);
        if (nv != f[v]) {
          f[v] = nv;
          s.changes++;
          for (int64_t k = poff[v]; k < poff[v + 1]; k++) {
            int32_t p = psrc[k];
            if (stamp[p] != r) { stamp[p] = r; next[nlen++] = p; s.pushes++; }
          }
        }
      }
      s.rounds++;
      if (status) break;
      int32_t *t = queue; queue = next; next = t;
      len = nlen;
    }
    free(next);
    free(stamp);
  } else if (order == ORC_ALG1) {
    /* Alg. 1: counters of satisfied out-edges for player-0 vertices */
    int64_t head = 0, tail = 0, size = 0; /* circular FIFO of capacity n */
    for (int32_t v = 0; v < n; v++) {
      int act = f_init ? 1 : initially_active(v, off, w, owner);
      if (act) { queue[tail] = v; tail = (tail + 1) % n; size++; inq[v] = 1; s.pushes++; }
      if (owner[v] == 0) {
        int64_t c = 0;
        if (!act)
          for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (f[v] >= clamp_to_codomain(ominus(f[tgt[e]], w[e]), bound)) c++;
        cnt[v] = c;
      }
    }
    while (size > 0) {
      if (max_lifts && s.lifts >= max_lifts) { status = 1; break; }
      int32_t v = queue[head]; head = (head + 1) % n; size--; inq[v] = 0;
      int64_t old = f[v];
      f[v] = lift_value(v, off, tgt, w, owner, f, bound);
      s.lifts++;
      s.relaxed_edges += (uint64_t)(off[v + 1] - off[v]);
      if (f[v] != old) s.changes++;
      if (owner[v] == 0) {
        int64_t c = 0;
        for (int64_t e = off[v]; e < off[v + 1]; e++)
          if (f[v] >= clamp_to_codomain(ominus(f[tgt[e]], w[e]), bound)) c++;
        cnt[v] = c;
      }
      for (int64_t k = poff[v]; k < poff[v + 1]; k++) {
        int32_t p = psrc[k];
        int64_t we = w[pedge[k]];
        if (!(f[p] < clamp_to_codomain(ominus(f[v], we), bound))) continue;
        int enq = 0;
        if (owner[p] == 0) {
          if (f[p] >= clamp_to_codomain(ominus(old, we), bound)) cnt[p]--;
          if (cnt[p] <= 0) enq = 1;
        } else {
          enq = 1;
        }
        if (enq && !inq[p]) { queue[tail] = p; tail = (tail + 1) % n; size++; inq[p] = 1; s.pushes++; }
      }
    }
  } else {
    /* worklist: FIFO (circular buffer), LIFO (stack) or random pick */
    int64_t head = 0, size = 0;
    for (int32_t v = 0; v < n; v++)
      if (f_init || initially_active(v, off, w, owner)) {
        queue[(head + size) % n] = v; size++; inq[v] = 1; s.pushes++;
      }
    while (size > 0) {
      if (max_lifts && s.lifts >= max_lifts) { status = 1; break; }
      int32_t v;
      if (order == ORC_FIFO) {
        v = queue[head]; head = (head + 1) % n; size--;
      } else if (order == ORC_LIFO) {
        v = queue[(head + size - 1) % n]; size--;
      } else {
        int64_t pick = (int64_t)(splitmix_next(&rng) % (uint64_t)size);
        int64_t a = (head + pick) % n, last = (head + size - 1) % n;
        v = queue[a]; queue[a] = queue[last]; size--;
      }
      inq[v] = 0;
      int64_t nv = lift_value(v, off, tgt, w, owner, f, bound);
      s.lifts++;
      s.relaxed_edges += (uint64_t)(off[v + 1] - off[v]);
      if (nv != f[v]) {
        f[v] = nv;
        s.changes++;
        for (int64_t k = poff[v]; k < poff[v + 1]; k++) {
          int32_t p = psrc[k];
          if (!inq[p]) { queue[(head + size) % n] = p; size++; inq[p] = 1; s.pushes++; }
        }
      }
    }
  }

done:
  free(poff); free(psrc); free(pedge); free(fill); free(queue); free(inq); free(cnt); free(prev);
  if (st) *st = s;
  return status;
}

/* Does f satisfy f(v) = delta(f, v)(v) at every v (a fixpoint of Def. 6)?
 * Returns the number of vertices where it does not. */
int64_t orc_count_unstable(int32_t n, const int64_t *off, const int32_t *tgt, const int32_t *w,
                           const uint8_t *owner, int64_t bound, const int64_t *f) {
  int64_t bad = 0;
  for (int32_t v = 0; v < n; v++)
    if (lift_value(v, off, tgt, w, owner, f, bound) != f[v]) bad++;
  return bad;
}

/* Player 0's positional strategy read off a progress measure f (Def. 5, first
 * condition; Lemma 1).  For v in V0 with f(v) finite, choice[v] is the least k
 * such that the edge e = off[v] + k satisfies f(v) >= f(target(e)) (-) w(e)
 * (TOP is above every finite value); -1 for player-1 vertices and where
 * f(v) = TOP.  When f is the least progress measure, following these edges
 * keeps the energy of every play from v >= 0 given the initial credit f(v).
 * Returns the number of V0 vertices with finite f(v) and no such edge (0 for
 * a progress measure); those get -1 as well. */
int64_t orc_strategy(int32_t n, const int64_t *off, const int32_t *tgt, const int32_t *w,
                     const uint8_t *owner, int64_t bound, const int64_t *f, int32_t *choice) {
  int64_t missing = 0;
  for (int32_t v = 0; v < n; v++) {
    choice[v] = -1;
    if (owner[v] != 0 || f[v] == ORC_TOP) continue;
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int64_t term = clamp_to_codomain(ominus(f[tgt[e]], (int64_t)w[e]), bound);
      if (term != ORC_TOP && term <= f[v]) {
        choice[v] = (int32_t)(e - off[v]);
        break;
      }
    }
    if (choice[v] < 0) missing++;
  }
  return missing;
}
