// Adjoint of the FSI evolution (placeholder until the adjoint kernels land).
#include "eed4.h"
#include "eed4_host.h"

namespace eed4 {
size_t backward_workspace(int, int, int, const eed4_params *) { return 0; }
}  // namespace eed4

extern "C" int eed4_backward(const float *, const uint8_t *, const float *, int, int, int,
                             const eed4_params *, int, const float *, float *, float *, float *,
                             void *, size_t, void *)
{
    return EED4_EINVAL;
}
