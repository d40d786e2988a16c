// One precision x cells-per-lane instantiation of the batched plan kernel.
#include "kernels.hpp"

#ifndef ADK_PLAN_PREC
#error "define ADK_PLAN_PREC (f64 or mixed) and ADK_PLAN_CPL (1, 2 or 4)"
#endif

#define ADK_CAT2(a, b) a##b
#define ADK_CAT(a, b) ADK_CAT2(a, b)
#define ADK_POLICY_f64 adk::PolicyF64
#define ADK_POLICY_mixed adk::PolicyMixed
#define ADK_POLICY ADK_CAT(ADK_POLICY_, ADK_PLAN_PREC)
#define ADK_NAME(kind) ADK_CAT(ADK_CAT(ADK_CAT(ADK_CAT(adk_plan_, kind), _), ADK_CAT(ADK_PLAN_PREC, _)), ADK_PLAN_CPL)

hipError_t ADK_NAME(launch)(const adk::PlanArgs &a, int grid, const void *E, void *pops, uint8_t *lo, int64_t n,
                            const int32_t *perm, const adk::PlanTile *tiles, unsigned *ctr, hipStream_t st)
{
    return adk::launch_plan<ADK_POLICY, ADK_PLAN_CPL>(a, grid, E, pops, lo, n, perm, tiles, ctr, st);
}

int ADK_NAME(occupancy)() { return adk::plan_occupancy<ADK_POLICY, ADK_PLAN_CPL>(); }
