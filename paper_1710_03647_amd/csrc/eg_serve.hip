// Serving runtime (placeholder until the batched iteration lands).
#include "eg_serve.h"

namespace eg {

struct Server {};

Server* server_create(const eg_config&, hipStream_t) { return new Server(); }
void server_destroy(Server* s) { delete s; }
int server_submit(Server*, const eg_game_desc*, eg_ticket*) {
  set_error("serving is not available in this build");
  return EG_EINVAL;
}
int server_poll(Server*, eg_ticket, int64_t*, eg_stats*) {
  set_error("serving is not available in this build");
  return EG_ENOTFOUND;
}
int server_cancel(Server*, eg_ticket) {
  set_error("serving is not available in this build");
  return EG_ENOTFOUND;
}

}  // namespace eg
