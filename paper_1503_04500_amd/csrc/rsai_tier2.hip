// Size tier 2 of the fused RSAI(tol) kernel (a wave per column, 2 rows x 32 columns
// per lane), compiled with the full unrolling of the register tiers.
#include "rsai_tier_kernel.h"

namespace rsai {

void launch_tier2(const TierArgs &a, int waves, hipStream_t s) { launch_tier<Tier2>(a, waves, s); }

}  // namespace rsai
