// Error reporting, version and the velocity table of the C ABI.
#include <string>

#include "mdlg_internal.h"

namespace mdlg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mdlg_status fail(mdlg_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

}  // namespace mdlg

extern "C" const char* mdlg_last_error(void) { return mdlg::g_last_error.c_str(); }

extern "C" const char* mdlg_version(void) { return "mdlg-mi355x 0.1.0 (gfx950)"; }

extern "C" mdlg_status mdlg_velocity_table(int32_t* out) {
    if (!out) return mdlg::fail(MDLG_EINVAL, "mdlg_velocity_table: out is NULL");
    for (int i = 0; i < MDLG_NQ; ++i) {
        out[2 * i] = mdlg::kVel.v[i][0];
        out[2 * i + 1] = mdlg::kVel.v[i][1];
    }
    return MDLG_OK;
}
