// Refocus configuration choice: cached autotuned configurations, defaults.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "cpi.h"
#include "kernels.h"

namespace cpi {

// Configuration used by cpi_refocus: the cached autotuned one for this shape
// and device if any, else a default sized to fill the device.
RefocusConfig refocus_config_for(const cpi_geometry* g, int32_t n_alpha);
RefocusConfig default_refocus_config(const cpi_geometry* g, int32_t n_alpha);
// The column-sum kernel's default, taken where the row-lane kernel does not
// run the geometry or plane set.
RefocusConfig default_sep_config(const cpi_geometry* g, int32_t n_alpha);

// Times every supported configuration on the given inputs, caches the fastest
// and leaves its result in `out`.  Synchronises `st`.
cpi_status autotune_refocus(const float* gamma, const cpi_geometry* g, const double* alphas,
                            int32_t n_alpha, float* out, void* ws, size_t ws_bytes,
                            hipStream_t st, std::string* why);

// Enqueue a refocus (defined with the C ABI): `forced` overrides the
// configuration; `plain` selects the one-plane-per-launch kernel.
// Enqueue with an explicit column-sum or per-row configuration against a
// workspace that holds the tables and that configuration's partial sums only.
cpi_status refocus_enqueue_config(const float* gamma, const cpi_geometry* g, const double* alphas,
                                  int32_t n_alpha, float* out, void* workspace, size_t ws_bytes,
                                  hipStream_t st, const RefocusConfig& c);

cpi_status refocus_enqueue(const float* gamma, const cpi_geometry* g, const double* alphas,
                           int32_t n_alpha, float* out, void* workspace, size_t ws_bytes,
                           hipStream_t st, const RefocusConfig* forced, bool plain);

}  // namespace cpi
