// Reverse-mode adjoint kernel (placeholder until the kernel lands).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace rich {

int adjoint_block_size() { return 256; }

hipError_t launch_adjoint(const DevScene &, const DevSource &, const AdjointArgs &, uint64_t, uint64_t, uint64_t, int,
                          hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace rich
