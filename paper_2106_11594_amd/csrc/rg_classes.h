// Size classes of the register-resident batched kernel and their launcher.
#pragma once
#include "rg_internal.h"

#define RG_NUM_CLASSES 0
#define RG_MAX_FAMILIES (1 + RG_NUM_CLASSES)  // family 0 = generic global-state kernel

namespace rg {
// Class index for a stream of m regressors and capacity r_max, or -1 when the
// stream goes to the generic kernel.
int choose_class(int m, int r_max, int dtype);
template <typename T>
hipError_t launch_push_class(int cls, const PushArgs<T> &a, int num_cus, hipStream_t s);
}  // namespace rg
