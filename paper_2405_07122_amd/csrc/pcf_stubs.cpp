// Temporary: serving and tuning entry points not yet built.
#include "../../include/pcfsort.h"
extern "C" {
int pcf_autotune(int, int, const char*) { return PCF_ERR_UNSUPPORTED; }
int pcf_load_tuning(const char*) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_create(const pcf_serve_config*, pcf_server**) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_submit(pcf_server*, int, const void*, size_t, int, uint64_t*) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_poll(pcf_server*, uint64_t, pcf_result*) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_wait(pcf_server*, uint64_t, uint32_t, pcf_result*) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_release(pcf_server*, uint64_t) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_get_stats(pcf_server*, pcf_serve_stats*) { return PCF_ERR_UNSUPPORTED; }
int pcf_serve_destroy(pcf_server*) { return PCF_ERR_UNSUPPORTED; }
}
