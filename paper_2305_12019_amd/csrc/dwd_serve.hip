// Serving loop (placeholder until the continuous-batching engine lands).
#include <hip/hip_runtime.h>

#include "dwd_solver.h"

using namespace dwd;

extern "C" dwd_status dwd_serve(const dwd_request* reqs, int32_t nreq, const dwd_serve_opts* opts,
                                dwd_response* out) {
  (void)reqs;
  (void)nreq;
  (void)opts;
  (void)out;
  return fail(DWD_E_INVALID, "dwd_serve: not built yet");
}
