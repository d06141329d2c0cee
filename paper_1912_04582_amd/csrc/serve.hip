// Serving entry points (continuous batching); see tk.h.
#include "tk_runtime.h"

extern "C" {

tk_status tk_serve_create(tk_ctx* ctx, size_t, tk_server** out) {
  if (out) *out = nullptr;
  return ctx_fail(ctx, TK_EINVAL, "serving is not available in this build");
}
tk_status tk_serve_submit(tk_server*, const tk_request*, uint64_t*) { return TK_EINVAL; }
tk_status tk_serve_poll(tk_server*, uint64_t, tk_result*) { return TK_EINVAL; }
tk_status tk_serve_destroy(tk_server*) { return TK_EINVAL; }

}  // extern "C"
