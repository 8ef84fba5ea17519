// Serving runtime of libeg: request queue, admission by device footprint and
// the batched multi-game iteration.
#pragma once
#include <hip/hip_runtime.h>

#include "eg.h"

namespace eg {

struct Server;
Server* server_create(const eg_config& cfg, hipStream_t stream);
// Cancels every pending and running ticket (EG_ECANCELED), wakes the waiters,
// waits until no call holds a use of the server, then stops the serving
// thread and frees everything.
void server_destroy(Server* s);
// A use of the server by an API call in progress (server_destroy waits for
// every use to end).
void server_enter(Server* s);
void server_leave(Server* s);
// stream: where device-pointer inputs (EG_MEM_DEVICE) are read (synchronised)
int server_submit(Server* s, const eg_game_desc* desc, hipStream_t stream, eg_ticket* out);
int server_poll(Server* s, eg_ticket t, int64_t* credits, eg_stats* st);
int server_cancel(Server* s, eg_ticket t);
int server_wait(Server* s, eg_ticket t, int64_t* credits, eg_stats* st, double timeout_s);

void set_error(const char* msg);
const char* get_error();

}  // namespace eg
