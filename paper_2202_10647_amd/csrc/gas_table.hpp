// Host-side gas object and table builder shared by the library's C++/HIP
// translation units.
#pragma once
#include <mutex>

#include "adkion.h"

// Opaque gas handle of the C ABI: per-level coefficients of Eq. (1) in log
// form (see gas_table.cpp), kept on the host and in device memory.
struct adk_gas {
    int32_t Z = 0;
    adk_constants consts{};
    int device = 0;
    int has_poly = 0;                  // some level averages over m
    double *d_coef = nullptr;          // device [Z][8]
    double h_coef[ADK_MAX_Z * 8] = {}; // host copy
    // field cutoff of the last time step used (see adk::field_cutoff)
    std::mutex cut_mu;
    double cut_dt = -1.0;
    double cut_E = 0.0;
    // per-level negligible-rate fields of the last step used by the surrogate
    double thr_dt = -1.0;
    float thr_E[ADK_MAX_Z] = {};
    // per-window identity fields of the last (step, width) of ionize_step
    double wcut_dt = -1.0;
    int wcut_w = 0;
    float wcut[ADK_MAX_Z + 1] = {};
};

namespace adk {

adk_constants resolve_constants(const adk_constants *consts);
int validate_desc(const adk_gas_desc *d, const adk_constants *consts);
void build_coeffs(const adk_gas_desc &d, const adk_constants &c, double *coef);
// |E| (GV/m) below which W dt < 1e-30 for every level of the gas.
double field_cutoff(const adk_gas &g, double dt);
// Per level k, the field (GV/m) below which W_k dt < theta on the rising
// branch of Eq. (1) (+inf if W_k dt < theta at every field, 0 if nowhere).
void level_thresholds(const adk_gas &g, double dt, double theta, float *thr);

}  // namespace adk
