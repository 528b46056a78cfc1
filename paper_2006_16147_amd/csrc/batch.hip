// Multi-right-hand-side PCG: placeholder until the fused block V-cycle lands.
#include "internal.h"

namespace amg {

amg_status pcg_batch(amg_hierarchy *, int32_t, const double *, double *, double, int32_t,
                     amg_solve_info *) {
  return AMG_ERR_ARG;
}

}  // namespace amg
