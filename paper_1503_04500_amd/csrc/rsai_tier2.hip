// Size tier 2 of the fused RSAI(tol) kernel. Its block (8 rows x 32 columns per
// lane) does not fit the register file even fully unrolled, so this file keeps the
// compiler's default unrolling.
#include "rsai_tier_kernel.h"

namespace rsai {

void launch_tier2(const TierArgs &a, int waves, hipStream_t s) { launch_tier<Tier2>(a, waves, s); }

}  // namespace rsai
