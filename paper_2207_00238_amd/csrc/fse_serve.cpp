// fse_serve.cpp -- continuous-batching request server of libfse.
#include <hip/hip_runtime.h>

#include "../../include/fse.h"

extern "C" {

struct fse_server {
    int dummy;
};

fse_status_t fse_serve_create(const fse_serve_config_t* cfg, fse_server_t** server) {
    (void)cfg;
    (void)server;
    return FSE_ERR_UNSUPPORTED;
}
fse_status_t fse_serve_submit(fse_server_t* s, const fse_image_t* image, const fse_mask_t* mask,
                              const fse_params_t* p, fse_image_t* out, uint64_t* ticket) {
    (void)s; (void)image; (void)mask; (void)p; (void)out; (void)ticket;
    return FSE_ERR_UNSUPPORTED;
}
fse_status_t fse_serve_poll(fse_server_t* s, uint64_t ticket, int32_t* done, fse_request_stats_t* st) {
    (void)s; (void)ticket; (void)done; (void)st;
    return FSE_ERR_UNSUPPORTED;
}
fse_status_t fse_serve_wait(fse_server_t* s, uint64_t ticket, int64_t timeout_us, fse_request_stats_t* st) {
    (void)s; (void)ticket; (void)timeout_us; (void)st;
    return FSE_ERR_UNSUPPORTED;
}
fse_status_t fse_serve_destroy(fse_server_t* s) {
    (void)s;
    return FSE_ERR_UNSUPPORTED;
}
}
