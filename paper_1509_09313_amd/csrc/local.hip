// The other local NLS solvers of Algorithm 1 (MU, Eq. muupdate; HALS,
// Eq. halsupdate): the entry point and the per-k dispatch.  The kernels are
// in local_kernels.h, instantiated for every k in 1..64 by local_k*.hip.
#include "local_kernels.h"

namespace nmf {

int local_update_launch(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr, float* X,
                        int64_t ldx, hipStream_t s) {
  static const local::LaunchFn* table = [] {
    static local::LaunchFn t[64];
    local::fill_k1_44(t);
    local::fill_k45_56(t);
    local::fill_k57_64(t);
    return t;
  }();
  if (rows == 0) return NMF_OK;
  table[k - 1](solver, rows, G, R, ldr, X, ldx, s);
  return launch_status("local update");
}

}  // namespace nmf

extern "C" int nmf_local_update(int solver, int k, int64_t rows, const double* G, const float* R, int64_t ldr,
                                float* X, int64_t ldx, void* stream) {
  if (solver != NMF_SOLVER_HALS && solver != NMF_SOLVER_MU)
    return nmf::fail(NMF_EINVAL, "nmf_local_update: solver must be NMF_SOLVER_HALS or NMF_SOLVER_MU");
  if (!nmf::valid_k(k)) return nmf::fail(NMF_EINVAL, "nmf_local_update: k=%d outside [1,64]", k);
  if (rows < 0 || ldr < k || ldx < k) return nmf::fail(NMF_EINVAL, "nmf_local_update: bad sizes");
  if (rows > 0 && (!G || !R || !X)) return nmf::fail(NMF_EINVAL, "nmf_local_update: null pointer");
  return nmf::local_update_launch(solver, k, rows, G, R, ldr, X, ldx, nmf::as_stream(stream));
}
