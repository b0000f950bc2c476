// Size tier 0 of the fused RSAI(tol) kernel with the larger hash tables (a schedule
// choice of the autotuner), compiled with the unrolling of tier 0.
#include "rsai_tier_kernel.h"

namespace rsai {

void launch_tier0_h4(const TierArgs &a, int waves, hipStream_t s) { launch_tier<Tier0H4>(a, waves, s); }

}  // namespace rsai
