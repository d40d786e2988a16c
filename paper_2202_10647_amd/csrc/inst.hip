// One precision x window-width instantiation of the step and chain-advance
// kernels.  Compiled once per (ADK_INST_PREC, ADK_INST_W) pair so that the
// instantiations build in parallel.
#include "kernels.hpp"

#ifndef ADK_INST_PREC
#error "define ADK_INST_PREC (f64 or mixed) and ADK_INST_W (1..8)"
#endif

#define ADK_CAT2(a, b) a##b
#define ADK_CAT(a, b) ADK_CAT2(a, b)
#define ADK_POLICY_f64 adk::PolicyF64
#define ADK_POLICY_mixed adk::PolicyMixed
#define ADK_POLICY ADK_CAT(ADK_POLICY_, ADK_INST_PREC)
#define ADK_NAME(kind) ADK_CAT(ADK_CAT(ADK_CAT(ADK_CAT(adk_, kind), _), ADK_CAT(ADK_INST_PREC, _)), ADK_INST_W)

hipError_t ADK_NAME(step)(const adk_gas *g, const void *E, int64_t n, double dt, void *pops, uint8_t *lo,
                          const adk_window *win, void *dne, hipStream_t st)
{
    return adk::launch_step<ADK_POLICY, ADK_INST_W>(g, E, n, dt, pops, lo, win, dne, st);
}

hipError_t ADK_NAME(advance)(const void *Wr, int64_t n, double dt, void *pops, hipStream_t st)
{
    return adk::launch_advance<ADK_POLICY, ADK_INST_W>(Wr, n, dt, pops, st);
}
