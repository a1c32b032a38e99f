// Status codes and error reporting of the C ABI.
#include "fpe_internal.h"

namespace fpe {
namespace {
thread_local std::string t_last_error;
}

void set_error(const std::string &msg) { t_last_error = msg; }

fpe_status fail(fpe_status s, const std::string &msg) {
    t_last_error = msg;
    return s;
}

fpe_status hip_fail(hipError_t e, const char *what) {
    t_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return FPE_ERR_HIP;
}

}  // namespace fpe

extern "C" const char *fpe_status_string(fpe_status s) {
    switch (s) {
        case FPE_OK: return "FPE_OK";
        case FPE_ERR_INVALID_ARG: return "FPE_ERR_INVALID_ARG";
        case FPE_ERR_NONFINITE: return "FPE_ERR_NONFINITE";
        case FPE_ERR_PRECISION: return "FPE_ERR_PRECISION";
        case FPE_ERR_WORKSPACE: return "FPE_ERR_WORKSPACE";
        case FPE_ERR_HIP: return "FPE_ERR_HIP";
        case FPE_ERR_UNSUPPORTED: return "FPE_ERR_UNSUPPORTED";
        default: return "FPE_ERR_UNKNOWN";
    }
}

extern "C" const char *fpe_last_error(void) { return fpe::t_last_error.c_str(); }

extern "C" int32_t fpe_abi_version(void) { return 3; }
