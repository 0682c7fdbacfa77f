// Host side of the interpreter core (core_host.cpp).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

#include "../../include/gp.h"
#include "gp_internal.h"
#include "runtime.h"

namespace gpx {

int core_variants();
int core_variant_t(int vi);        // case slots per lane
int core_variant_d(int vi);        // stack levels
int core_variant_nf(int vi);       // feature slots
int core_variant_arith(int vi);    // 1: no sin/cos/exp/log code
bool core_variant_bool(int vi);    // the Boolean function set (32-bit word slots)
bool core_variant_trees_only(int vi);   // no linear handlers (Boolean and trees-only arithmetic kernels)
int core_variant_ncv(int vi);      // VGPRs left to the compiled code
int core_reg_levels(int vi);       // register/stack levels before the features
// Variant for programs reading n_load features, needing `depth` stack levels,
// with a fraction transc_frac of sin/cos/exp/log instructions (has_transc:
// any at all), of the Boolean function set if `boolean`, and trees only if
// `trees_only` (then a kernel without linear handlers may be taken); -1 if
// none fits.
int pick_core_variant(int n_load, int depth, double transc_frac, bool has_transc, bool boolean = false,
                      bool trees_only = false);
// Locate the variant's handler table on the current device (one probe launch
// on stream s the first time).
gp_status core_ready(int vi, hipStream_t s);
// True if core_ready has found variant vi's handler table on the current device.
bool core_is_ready(int vi);
// Core instructions and per-program records of lowered programs.
gp_status core_translate(const ProgData& pd, int vi, std::vector<uint32_t>& code, std::vector<DevProg>& progs);
// The same with the handler table taken to start at `base` (no device needed).
gp_status core_translate_at(const ProgData& pd, int vi, uint64_t base, std::vector<uint32_t>& code,
                            std::vector<DevProg>& progs);

}  // namespace gpx
