// Batched launches: reset of the per-chunk segment counters.
#include "internal.hpp"

namespace fdas {

__global__ void k_batch_reset(int32_t *counters, int32_t n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

}  // namespace fdas
