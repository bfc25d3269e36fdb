// Serving entry points (continuous batching over many sessions).
#include "../../include/qtask.h"

extern "C" {
int qtask_server_opts_default(qtask_server_opts *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_create(const qtask_server_opts *, qtask_server_t *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_destroy(qtask_server_t) { return QTASK_E_UNSUPPORTED; }
int qtask_server_open(qtask_server_t, int, qtask_dtype, const qtask_opts *, uint64_t, uint64_t, const int32_t *,
                      const int32_t *, const int32_t *, const double *, const uint64_t *, int32_t *) {
    return QTASK_E_UNSUPPORTED;
}
int qtask_server_submit(qtask_server_t, int32_t, const qtask_edit *, int, uint64_t *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_wait(qtask_server_t, uint64_t, double, qtask_result *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_poll(qtask_server_t, uint64_t, int *, qtask_result *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_drain(qtask_server_t) { return QTASK_E_UNSUPPORTED; }
int qtask_server_session(qtask_server_t, int32_t, qtask_t *) { return QTASK_E_UNSUPPORTED; }
int qtask_server_usage(qtask_server_t, uint64_t *, int32_t *) { return QTASK_E_UNSUPPORTED; }
}
