// Host-side argument checks of the C ABI (g4d_checks.cpp): plain C++, no HIP.  Each returns
// G4D_OK or G4D_EINVAL and, on failure, writes a message into err[0..n_err).
#pragma once

#include <stddef.h>

#include "../../include/g4d.h"

namespace g4d {

// Gaussians (params: the parameter arrays must be present), views and settings of a render.
g4d_status check_args(const g4d_gaussians* g, const g4d_view* views, int32_t n_views,
                      const g4d_settings* s, bool params, char* err, size_t n_err);
// Extra channels of a channel render of g.
g4d_status check_channels_args(const g4d_gaussians* g, const g4d_channels* ch, char* err,
                               size_t n_err);
// A compact model.
g4d_status check_compact_args(const g4d_compact* c, char* err, size_t n_err);
// Extra channels E = n_features + depth + 2 flow (0 without channels).
int n_ext_of(const g4d_channels* ch);

}  // namespace g4d
