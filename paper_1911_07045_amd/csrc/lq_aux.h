// Internal declarations of the helpers outside the step kernels: the fixed
// workspace of the allocation-free minimizer.
#pragma once

#include <stdint.h>

#include "lqfire.h"

namespace lq {

// Device address of the fixed workspace of lq_minimize_noalloc on `device`
// (which must be current): looked up once per device, then cached.
int noalloc_workspace(int device, void** out);

}  // namespace lq
