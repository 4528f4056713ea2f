// Launcher of the network's row kernel with the batch gathered from data
// rows inside the kernel (used by rta_mlp_train_step_rows).
#pragma once

#include "rta_internal.h"

namespace rta {
// rows [B] (device): data row of each batch row, clamped to [0, n_data);
// rows == nullptr: batch row b is data row b.
hipError_t launch_mlp_rows_gather(const MlpDev& w, const float* x, const float* label, const float* log10e,
                                  const int64_t* rows, int64_t n_data, int B, int Bpad, float* out, bool train,
                                  hipStream_t st);
}  // namespace rta
