// Continuous-batching server replay (placeholder until the serving loop lands).
#include "../../include/rkmips.h"

extern "C" rkmips_status rkmips_serve_replay(rkmips_index*, const void*, const float*, int64_t, const int32_t*,
                                             const int64_t*, const rkmips_serve_params*, double*,
                                             rkmips_serve_stats*, rkmips_result**)
{
    return RKMIPS_EINVAL;
}
