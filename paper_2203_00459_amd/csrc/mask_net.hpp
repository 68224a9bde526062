// Internal entry of the mask network shared with the ragged work lists.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fmbym_mask.h"

namespace fmbym {

// fmbym_mask_fwd with the scans given either packed (x + i n^2) or as a device
// table of image pointers (x_tab[i], x null).
int mask_forward(const fmbym_mask_desc* d, int images, int n, const float* x, const float* const* x_tab,
                 float* mask, void* act, size_t act_bytes, int training, hipStream_t s);

}  // namespace fmbym
