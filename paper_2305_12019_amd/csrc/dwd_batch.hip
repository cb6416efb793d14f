// Batched solve over one shared X (placeholder: problems run one after the
// other on the shared set-up; the stepped-together path replaces it).
#include <hip/hip_runtime.h>

#include <vector>

#include "dwd_solver.h"

namespace dwd {

dwd_status solve_batch(Problem* P, int B, const dwd_params* p, double* W, dwd_info* info) {
  dwd_status worst = DWD_OK;
  for (int j = 0; j < B; ++j) {
    dwd_status s = solve_problem(P, &p[j], W ? W + (size_t)j * P->d : nullptr,
                                 info ? &info[j] : nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr);
    if (s < 0) return s;
    if (s == DWD_NOT_CONVERGED) worst = DWD_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace dwd
