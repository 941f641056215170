// Serving loop (continuous batching of diffusion-map eigensolves).
#include <string>

#include "op.hpp"

extern "C" {

hdm_status hdm_server_create(hdm_ctx, const hdm_server_cfg_t*, hdm_server*) { return HDM_EINTERNAL; }
hdm_status hdm_submit(hdm_server, const hdm_request_t*, uint64_t*) { return HDM_EINTERNAL; }
hdm_status hdm_poll(hdm_server, uint64_t, hdm_result_t*) { return HDM_EINTERNAL; }
hdm_status hdm_cancel(hdm_server, uint64_t) { return HDM_EINTERNAL; }
hdm_status hdm_server_stats(hdm_server, hdm_server_stats_t*) { return HDM_EINTERNAL; }
hdm_status hdm_server_destroy(hdm_server) { return HDM_EINTERNAL; }

}  // extern "C"
