// Library-internal entry to the panel jets for callers that own their scratch
// (the boundary integral solves call it once per operator product).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vp.h"

namespace vp {

// vp_boundary_jets with caller-owned scratch ws of 3 n_pan q doubles (device)
// and arguments already validated; enqueues two launches on st.
vp_status boundary_jets_ws(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y, const double* dens,
                           int64_t n_tgt, const int32_t* pan, const double* u, int nder, double* out, hipStream_t st,
                           double* ws);

}  // namespace vp
