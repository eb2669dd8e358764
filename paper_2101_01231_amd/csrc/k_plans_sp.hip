// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3) with static pivots (layout 5):
// several rows per lane (the layout-4 geometry, or the layout-3 one at 2D order 4), FP64 or FP32
// with FP64-residual iterative refinement.
#include "plans_nr.hpp"

namespace ridg {

template <int D, int M>
struct launch_plans_spL {
  static int run(int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                 const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                 int64_t n_items, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    using C = PlanCfgSp<D, M>;
    if (n_items % C::S) return (int)hipErrorInvalidValue;  // the list is padded to whole wavefronts
    const int64_t per_block = (int64_t)C::WAVES * C::S;
    const int64_t blocks = (n_items + per_block - 1) / per_block;
    if (blocks == 0) return 0;
    if (precision == RIDG_FP32_REFINE)
      hipLaunchKernelGGL((predict_plans_sp_kernel<D, M, C::RPL, C::SEGW, true>), dim3((unsigned)blocks),
                         dim3(64 * C::WAVES), 0, (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items,
                         refine);
    else
      hipLaunchKernelGGL((predict_plans_sp_kernel<D, M, C::RPL, C::SEGW, false>), dim3((unsigned)blocks),
                         dim3(64 * C::WAVES), 0, (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items,
                         0);
    return (int)hipGetLastError();
  }
};

int launch_plans_sp(int d, int M, int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                    const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                    int64_t n_items, void* stream) {
  return dispatch_dm<launch_plans_spL>(d, M, precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items,
                                       stream);
}

}  // namespace ridg
