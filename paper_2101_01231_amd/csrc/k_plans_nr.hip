// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3): two rows per lane (layout 3).
#include "plans_nr.hpp"

namespace ridg {

template <int D, int M>
struct launch_plans_2rowsL {
  static int run(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t, const PlanRec* plans,
                 const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    return launch_nr<PlanCfg2R<D, M>, D, M>(g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
  }
};

int launch_plans_2rows(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
            const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream) {
  return dispatch_dm<launch_plans_2rowsL>(d, M, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
}

}  // namespace ridg
