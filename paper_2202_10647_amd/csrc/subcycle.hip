// Sub-cycled explicit (RK4) integration of the windowed chain: the
// comparison baseline of adk_subcycle_step (see kernels.hpp).
#include <cmath>

#include "kernels.hpp"

namespace {

using Fn = hipError_t (*)(const adk_gas *, const double *, int64_t, double, double *, uint8_t *, double, int,
                          hipStream_t);
const Fn kSub[ADK_MAX_W + 1] = {nullptr,
                                adk::launch_subcycle<1>,
                                adk::launch_subcycle<2>,
                                adk::launch_subcycle<3>,
                                adk::launch_subcycle<4>,
                                adk::launch_subcycle<5>,
                                adk::launch_subcycle<6>,
                                adk::launch_subcycle<7>,
                                adk::launch_subcycle<8>};

}  // namespace

extern "C" int adk_subcycle_step(const adk_gas *gas, const void *E, int64_t ncells, double dt, void *pops,
                                 uint8_t *lo, const adk_window *win, int32_t nsub, hipStream_t stream)
{
    if (!gas || !win || ncells < 0 || nsub < 1) return ADK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ADK_EINVAL;
    if (!(win->eps >= 0.0) || !std::isfinite(win->eps)) return ADK_EINVAL;
    if (win->prec != ADK_F64 || win->layout != ADK_LAYOUT_COMPACT) return ADK_EINVAL;
    if (win->w < 1 || win->w > ADK_MAX_W || win->w > gas->Z) return ADK_ERANGE;
    if (ncells > 0 && (!E || !pops || !lo)) return ADK_EINVAL;
    if (ncells == 0) return ADK_OK;
    const hipError_t e = kSub[win->w](gas, (const double *)E, ncells, dt, (double *)pops, lo, win->eps, nsub, stream);
    if (e == hipSuccess) return ADK_OK;
    return e == hipErrorOutOfMemory ? ADK_ENOMEM : ADK_EDEVICE;
}
