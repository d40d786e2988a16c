// One precision x widest-window instantiation of the batched plan kernel
// (cells per lane 1, 2 and 4).
#include "kernels.hpp"

#ifndef ADK_PLAN_PREC
#error "define ADK_PLAN_PREC (f64 or mixed) and ADK_PLAN_WMAX (1..6)"
#endif

#define ADK_CAT2(a, b) a##b
#define ADK_CAT(a, b) ADK_CAT2(a, b)
#define ADK_POLICY_f64 adk::PolicyF64
#define ADK_POLICY_mixed adk::PolicyMixed
#define ADK_POLICY ADK_CAT(ADK_POLICY_, ADK_PLAN_PREC)
#define ADK_NAME(kind, cpl)                                                                                  \
    ADK_CAT(ADK_CAT(ADK_CAT(ADK_CAT(ADK_CAT(ADK_CAT(adk_plan_, kind), _), ADK_CAT(ADK_PLAN_PREC, _)), ADK_PLAN_WMAX), \
                    _),                                                                                      \
            cpl)

#define ADK_PLAN_DEFINE(CPL)                                                                                 \
    hipError_t ADK_NAME(launch, CPL)(const adk::PlanArgs &a, const void *E, void *pops, uint8_t *lo, int64_t n, \
                                     const int32_t *perm, const adk::PlanTile *tiles, hipStream_t st)        \
    {                                                                                                        \
        return adk::launch_plan<ADK_POLICY, ADK_PLAN_WMAX, CPL>(a, E, pops, lo, n, perm, tiles, st);         \
    }

ADK_PLAN_DEFINE(1)
ADK_PLAN_DEFINE(2)
ADK_PLAN_DEFINE(4)
