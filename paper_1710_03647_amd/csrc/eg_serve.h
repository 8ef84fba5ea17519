// Serving runtime of libeg: request queue, admission by device footprint and
// the batched multi-game iteration.
#pragma once
#include <hip/hip_runtime.h>

#include "eg.h"

namespace eg {

struct Server;
Server* server_create(const eg_config& cfg, hipStream_t stream);
void server_destroy(Server* s);
int server_submit(Server* s, const eg_game_desc* desc, eg_ticket* out);
int server_poll(Server* s, eg_ticket t, int64_t* credits, eg_stats* st);
int server_cancel(Server* s, eg_ticket t);
int server_wait(Server* s, eg_ticket t, int64_t* credits, eg_stats* st, double timeout_s);

void set_error(const char* msg);
const char* get_error();

}  // namespace eg
