// Continuous-batching server (in progress).
#include "runtime.hpp"

extern "C" {
int fastlec_es_server_create(const fastlec_es_options*, size_t, fastlec_es_server** out) {
    if (out) *out = nullptr;
    return FASTLEC_ERR_UNSUPPORTED;
}
int fastlec_es_server_submit(fastlec_es_server*, const fastlec_es_circuit*, uint64_t*) { return FASTLEC_ERR_UNSUPPORTED; }
int fastlec_es_server_poll(fastlec_es_server*, uint64_t, fastlec_es_result*, int) { return FASTLEC_ERR_UNSUPPORTED; }
int fastlec_es_server_stats_get(fastlec_es_server*, fastlec_es_server_stats*) { return FASTLEC_ERR_UNSUPPORTED; }
void fastlec_es_server_destroy(fastlec_es_server*) {}
}
