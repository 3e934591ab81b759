// Placeholder serving entry points (replaced by the continuous-batching server).
#include "mdp.h"

extern "C" {
int mdp_server_create(size_t, int32_t, mdp_server **out) {
  if (out) *out = nullptr;
  return MDP_EINVAL;
}
int mdp_server_register(mdp_server *, mdp_handle *) { return MDP_EINVAL; }
int mdp_submit(mdp_server *, mdp_handle *, const double *, double *, int32_t, uint64_t *) { return MDP_EINVAL; }
int mdp_poll(mdp_server *, uint64_t, mdp_stats *) { return MDP_EINVAL; }
int mdp_server_destroy(mdp_server *) { return MDP_OK; }
}
