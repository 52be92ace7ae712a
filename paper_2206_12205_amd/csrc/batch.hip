// Batched launches: the tile counter reset kernel.
#include "internal.hpp"

namespace fdas {

__global__ void k_batch_reset(int32_t *counter) {
    if (threadIdx.x == 0) counter[0] = 0;
}

}  // namespace fdas
