// Size tiers 0 and 1 of the fused RSAI(tol) kernel (tier 2 is in rsai_tier2.hip).
#include "rsai_tier_kernel.h"

namespace rsai {

const TierInfo kTiers[] = {
    {Tier0::G, Tier0::MMAX, Tier0::QMAX, Tier0::REC, Tier0::WPS},
    {Tier1::G, Tier1::MMAX, Tier1::QMAX, Tier1::REC, Tier1::WPS},
    {Tier2::G, Tier2::MMAX, Tier2::QMAX, Tier2::REC, Tier2::WPS},
};
const int kNumTiers = 3;
const int kPlainTier = 1;

void launch_tier_kernel(int tier, int hash4, const TierArgs &a, int waves, hipStream_t s) {
    switch (tier) {
        case 0:
            if (hash4) launch_tier0_h4(a, waves, s);
            else launch_tier<Tier0>(a, waves, s);
            break;
        case 1: launch_tier<Tier1>(a, waves, s); break;
        case 2: launch_tier2(a, waves, s); break;
        default: break;
    }
}

}  // namespace rsai
