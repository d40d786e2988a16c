// Host-side gas object and table builder shared by the library's C++/HIP
// translation units.
#pragma once
#include "adkion.h"

// Opaque gas handle of the C ABI: per-level coefficients of Eq. (1) in log
// form (see gas_table.cpp), kept on the host and in device memory.
struct adk_gas {
    int32_t Z;
    adk_constants consts;
    int device;
    double *d_coef;                 // device [Z][8]
    double h_coef[ADK_MAX_Z * 8];   // host copy
};

namespace adk {

adk_constants resolve_constants(const adk_constants *consts);
int validate_desc(const adk_gas_desc *d, const adk_constants *consts);
void build_coeffs(const adk_gas_desc &d, const adk_constants &c, double *coef);

}  // namespace adk
