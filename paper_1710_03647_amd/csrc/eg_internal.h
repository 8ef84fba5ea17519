// Internal declarations of libeg: device layout of a game and the kernel
// launchers used by the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eg {

// Row starts are uint32 (m < 2^31); bit 31 of rs[v] carries the owner of v
// (1 = player 1, the max player), so one load yields both.
constexpr uint32_t OWNER_BIT = 0x80000000u;
constexpr uint32_t ROW_MASK = 0x7FFFFFFFu;

// ctrl[] words (uint32) and stats[] words (uint64) in device memory
enum Ctrl : int {
  C_CNT0 = 0,      // C_CNT0 + (r % 3): size of the active list of round r
  C_ROUNDS = 3,    // rounds with a non-empty active set
  C_DONE = 4,      // dense driver: blocks finished in the current round
  C_MODE = 5,      // dense driver: representation of the next round
  C_WORDS = 8
};
enum Stat : int { S_LIFTS = 0, S_EDGES = 1, S_PUSHES = 2, S_CHANGES = 3, S_WORDS = 4 };

// Everything a kernel needs to see of one game (passed by value).
struct DevGame {
  int32_t n;
  uint32_t m;
  const uint32_t* rs;       // n+1 row starts | owner bit
  const int2* edges;        // m {target, weight}
  const uint32_t* rev_off;  // n+1 predecessor-list starts (the paper's CSC)
  const int32_t* rev_src;   // m predecessor ids, one per edge
  void* f;                  // n values, int32 or int64 (vbits)
  uint32_t* stamp;          // n: stamp[v] == r  <=>  v is active in round r
  int32_t* wl0;             // n: active list of even rounds
  int32_t* wl1;             // n: active list of odd rounds
  uint32_t* ctrl;           // C_WORDS
  unsigned long long* stats;  // S_WORDS
  int64_t bound;            // B
  int64_t top;              // device encoding of TOP: B + P + 1, P = largest stored weight
};

// Layout and predecessor lists (eg_kernels.hip)
hipError_t launch_layout(const int64_t* off, const uint8_t* owner_bits, const int32_t* tgt,
                         const int32_t* w, int32_t n, uint32_t m, int32_t wclamp, uint32_t* rs,
                         int2* edges, hipStream_t s);
hipError_t launch_reverse_csr(const uint32_t* rs, const int2* edges, int32_t n, uint32_t m,
                              uint32_t* rev_off, int32_t* rev_src, uint32_t* cursor,
                              uint32_t* scan_tmp, size_t scan_tmp_words, hipStream_t s);
size_t scan_tmp_words(size_t count);

// Solve steps
hipError_t launch_init(const DevGame& g, int vbits, int h, int resume, hipStream_t s);
hipError_t launch_round(const DevGame& g, int vbits, int h, uint32_t r, int grid, hipStream_t s);
hipError_t launch_output(const DevGame& g, int vbits, int64_t* out, hipStream_t s);
hipError_t launch_input(const DevGame& g, int vbits, const int64_t* in, hipStream_t s);

int pick_h(double avg_deg);
int round_grid(int device);

}  // namespace eg
