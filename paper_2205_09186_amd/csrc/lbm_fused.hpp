// lbm_fused.hpp -- single-pass fused step kernels (LDS-staged halos).
#pragma once

#include <hip/hip_runtime.h>
#include "lbm_kernels.hpp"

namespace lbm {

template <int LAT, int SCH>
inline bool fused_available(const Grid&) { return false; }

template <int LAT, int SCH>
inline void launch_fused_step(const double*, double*, double*, double*, const Grid&, const Eos&, double,
                              hipStream_t) {}

}  // namespace lbm
