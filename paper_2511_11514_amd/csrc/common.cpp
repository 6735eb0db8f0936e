// Error reporting and version of libct.so.
#include <cstdarg>
#include <cstdio>

#include "ct_internal.h"

namespace ct {

static thread_local char g_msg[512] = "";

ct_status fail(ct_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = '\0'; }

ct_status refuse_capture(hipStream_t st, const char* what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CT_CHECK_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(CT_E_CAPTURE, "%s synchronises with the device and cannot run while its "
                                  "stream is being captured", what);
    return CT_OK;
}

}  // namespace ct

extern "C" const char* ct_last_error(void) { return ct::g_msg; }
extern "C" const char* ct_version(void) { return "ct 0.1.0 (gfx950)"; }
