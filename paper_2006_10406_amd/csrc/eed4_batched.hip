// Batched uneven-size inpainting (placeholder until the persistent kernel lands).
#include "eed4.h"
#include "eed4_host.h"

extern "C" size_t eed4_batched_workspace_size(const eed4_image *, int, const eed4_params *)
{
    return 0;
}

extern "C" int eed4_inpaint_batched(const eed4_image *, int, const eed4_params *, void *, size_t,
                                    void *, eed4_stats *)
{
    return EED4_EINVAL;
}
