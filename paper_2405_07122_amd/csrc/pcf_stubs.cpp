// Tuning entry points not yet built.
#include "../../include/pcfsort.h"
extern "C" {
int pcf_autotune(int, int, const char*) { return PCF_ERR_UNSUPPORTED; }
int pcf_load_tuning(const char*) { return PCF_ERR_UNSUPPORTED; }
}
