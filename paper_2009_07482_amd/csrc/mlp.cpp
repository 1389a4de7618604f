// Learned cost model (placeholder until the MLP kernels land): any use reports unsupported.
#include "core.hpp"

namespace psc {
CostModel *mlp_cost_model(const psc_mlp *) {
  fail(PSC_ERR_UNSUPPORTED, "learned cost model not available in this build");
}
}  // namespace psc
