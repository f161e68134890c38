// Status strings and version of libquadbox.
#include "qb_common.h"

extern "C" const char* qb_status_string(qb_status s)
{
    switch (s) {
        case QB_OK: return "ok";
        case QB_ERR_INVALID_ARG: return "invalid argument";
        case QB_ERR_CAPACITY: return "pair capacity exceeded";
        case QB_ERR_HIP: return "HIP runtime error";
        case QB_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" int32_t qb_version(void) { return 100; }
