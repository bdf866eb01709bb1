// Status strings and version of libsff.
#include "sff.h"

extern "C" const char* sff_status_string(int32_t status) {
    switch (status) {
        case SFF_OK: return "ok";
        case SFF_ERR_INVALID_ARG: return "invalid argument";
        case SFF_ERR_UNSUPPORTED: return "unsupported configuration";
        case SFF_ERR_HIP: return "HIP runtime error";
        case SFF_ERR_WORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

extern "C" int32_t sff_version(void) { return 301; }  // 0.3.1: sff_sift_sqrt

extern "C" int32_t sff_desc_channels(int32_t C) {
    if (C < 1 || C > 4) return 0;
    return C == 3 ? 4 : C;
}
