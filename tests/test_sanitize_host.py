"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle (adk_oracle.c) and the library's host-side gas table and argument
validation (gas_table.cpp) are compiled with -fsanitize=address,undefined
into small drivers that run every entry point over ordinary and edge-case
inputs (zero, negative and non-finite fields, window indices past Z, the
full chain, the largest matrices, the adaptive window with forced tops,
invalid level tables).  Any out-of-bounds access, leak, overflow of a signed
integer or other undefined behaviour aborts the driver.  Host code only (no
device code is built with a sanitizer)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

ORACLE_DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
double orc_rate_lm(double, int, int, int, double, const double *);
double orc_level_rate(double, int, int, int, double, const double *);
void orc_rates(int, const double *, const int8_t *, const int8_t *, const double *, const double *, int64_t, int,
               int, double *);
void orc_expm(int, const double *, double *);
void orc_chain_advance(int, int64_t, const double *, double, double *);
void orc_ionize_step(int, const double *, const int8_t *, const int8_t *, const double *, int64_t, const double *,
                     double, int, double, int, double *, uint8_t *);
void orc_adaptive_step(int, const double *, const int8_t *, const int8_t *, const double *, int64_t,
                       const double *, double, int, int, double, double, double *, uint8_t *, uint8_t *,
                       const int *, int *, double *, double *, double *);
int main(void)
{
    const double c[3] = {4.13e16, 510.0, 27.21 / 2};
    enum { Z = 36, N = 97 };
    double U[Z];
    int8_t l[Z], m[Z];
    for (int k = 0; k < Z; ++k) { U[k] = 14.0 * pow(1.22, k); l[k] = (int8_t)(k % 3); m[k] = (int8_t)(k % 2 ? -1 : 0); }
    double E[N];
    for (int i = 0; i < N; ++i) E[i] = (i % 7 == 0) ? 0.0 : (i % 11 == 0 ? -300.0 : 10.0 * pow(1.08, i));
    E[5] = NAN; E[6] = INFINITY;
    double s = 0.0;
    for (int k = 0; k < Z; ++k) s += orc_rate_lm(U[k], k + 1, l[k], 0, 100.0, c) + orc_level_rate(U[k], k + 1, l[k], -1, 250.0, c);
    double *W = malloc(sizeof(double) * Z * N);
    orc_rates(Z, U, l, m, c, E, N, 0, Z, W);
    double M[72 * 72], T[72 * 72];
    for (int i = 0; i < 72 * 72; ++i) M[i] = 0.0;
    for (int i = 0; i + 1 < 72; ++i) { M[i * 72 + i] = -1e3 * (i + 1); M[(i + 1) * 72 + i] = 1e3 * (i + 1); }
    orc_expm(72, M, T);
    double *P = calloc((size_t)(Z + 1) * N, sizeof(double));
    uint8_t lo[N], wc[N];
    for (int w = 1; w <= Z; w += 7) {
        for (int i = 0; i < N; ++i) { lo[i] = (uint8_t)(i % 3 == 0 ? 200 : i % (Z + 1)); for (int r = 0; r <= w; ++r) P[r * N + i] = r == 0 ? 1.0 : 0.0; }
        orc_ionize_step(Z, U, l, m, c, N, E, 1.334e-16, w, 1e-8, 0, P, lo);
        for (int i = 0; i < N; ++i) lo[i] = (uint8_t)(i % (Z + 2));
        orc_ionize_step(Z, U, l, m, c, N, E, 1.334e-16, w, 1e-8, 1, P, lo);
        double *Wc = calloc((size_t)w * N, sizeof(double));
        for (int i = 0; i < w * N; ++i) Wc[i] = 1e16 * (i % 5);
        orc_chain_advance(w, N, Wc, 1e-16, P);
        free(Wc);
    }
    int ft[N], top[N];
    double lt[N], lb[N], *lk = malloc(sizeof(double) * (Z + 1) * N);
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < N; ++i) {
            lo[i] = (uint8_t)(i % (Z + 3));
            wc[i] = (uint8_t)(i % 40);
            ft[i] = pass == 2 ? (i % 4) : -1;
            for (int r = 0; r <= Z; ++r) P[r * N + i] = r == 0 ? 0.5 : (r == 1 ? 0.5 : 0.0);
        }
        orc_adaptive_step(Z, U, l, m, c, N, E, 1.334e-16, pass, Z, 1e-8, pass == 0 ? 0.0 : 1e-9, P, lo, wc,
                          pass == 2 ? ft : NULL, top, lt, lb, lk);
    }
    for (int i = 0; i < Z * N; ++i) s += isfinite(W[i]) ? W[i] * 0.0 : 0.0;
    free(W); free(P); free(lk);
    printf("ok %g %g\n", s, T[0]);
    return 0;
}
"""

GAS_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include "gas_table.hpp"
int main()
{
    adk_constants c{4.13e16, 510.0, 27.21 / 2};
    int bad = 0;
    // invalid tables: each must be rejected, none may fault
    double U[ADK_MAX_Z + 1];
    int8_t l[ADK_MAX_Z + 1], m[ADK_MAX_Z + 1];
    for (int k = 0; k <= ADK_MAX_Z; ++k) { U[k] = 13.6 * (k + 1); l[k] = (int8_t)(k % 4); m[k] = (int8_t)(k % 4 ? -1 : 0); }
    adk_gas_desc d{0, U, l, m};
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    d.Z = ADK_MAX_Z + 1;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    d.Z = 5; d.U_eV = nullptr;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    d.U_eV = U; U[2] = -1.0;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    U[2] = NAN;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    U[2] = 40.0; l[1] = 5;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    l[1] = 1; m[1] = 3;
    bad += adk::validate_desc(&d, &c) != ADK_OK;
    m[1] = -1;
    bad += adk_gas_coeffs(nullptr, &c, U) != ADK_OK;
    bad += adk_gas_coeffs(&d, &c, nullptr) != ADK_OK;
    // every size of a valid table: coefficients, field cutoff, level thresholds
    double coef[ADK_MAX_Z * 8];
    float thr[ADK_MAX_Z];
    double s = 0.0;
    for (int Z = 1; Z <= ADK_MAX_Z; ++Z) {
        adk_gas_desc g{Z, U, l, m};
        if (adk::validate_desc(&g, &c) != ADK_OK) return 2;
        if (adk_gas_coeffs(&g, nullptr, coef) != ADK_OK) return 3;
        adk_gas gas;
        gas.Z = Z;
        gas.consts = adk::resolve_constants(&c);
        adk::build_coeffs(g, gas.consts, gas.h_coef);
        for (double dt : {1e-18, 1.334e-16, 1e-14}) {
            s += adk::field_cutoff(gas, dt);
            adk::level_thresholds(gas, dt, 1e-9, thr);
            for (int k = 0; k < Z; ++k) s += std::isfinite(thr[k]) ? thr[k] : 0.0;
        }
        for (int k = 0; k < 8 * Z; ++k) s += coef[k] * 0.0;
    }
    std::printf("ok %d %g\n", bad, s);
    return bad == 9 ? 0 : 4;
}
"""


def _build_and_run(tmp_path, name, compiler, sources, extra):
    exe = str(tmp_path / name)
    r = subprocess.run([compiler, *SAN, *extra, "-o", exe, *sources], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "not supported" in r.stderr:
        pytest.skip("sanitizers not available to " + compiler)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    drv = tmp_path / "oracle_driver.c"
    drv.write_text(ORACLE_DRIVER)
    _build_and_run(tmp_path, "oracle_san", "gcc", [os.path.join(ROOT, "oracle", "adk_oracle.c"), str(drv)],
                   ["-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-lm"])


def test_gas_table_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are not available")
    drv = tmp_path / "gas_driver.cpp"
    drv.write_text(GAS_DRIVER)
    csrc = os.path.join(ROOT, "paper_2202_10647_amd", "csrc")
    _build_and_run(tmp_path, "gas_san", "g++", [os.path.join(csrc, "gas_table.cpp"), str(drv)],
                   ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    "-I", "/opt/rocm/include"])
