// hh_server.cpp -- request server (placeholder until the serving loop lands).
#include "hh_lib.h"

extern "C" {
hh_status hh_server_create(const hh_server_opts *, hh_server **out)
{
    if (out) *out = nullptr;
    return hh_fail(HH_ERR_ARG, "the request server is not built yet");
}
hh_status hh_submit(hh_server *, const hh_request *, uint64_t *) { return hh_fail(HH_ERR_ARG, "no server"); }
hh_status hh_poll(hh_server *, uint64_t, hh_result *) { return hh_fail(HH_ERR_TICKET, "no server"); }
hh_status hh_server_destroy(hh_server *) { return HH_OK; }
hh_status hh_server_query(hh_server *, hh_server_stats *) { return hh_fail(HH_ERR_ARG, "no server"); }
}
