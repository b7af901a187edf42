// One translation unit per coupled rank L (compiled with -DAP_RANK_L=<L>):
// the rank kernel instances of that L, for the launcher in k_ace_mixed.hip.
#include "ace_rank.h"

#ifndef AP_RANK_L
#error "k_ace_rank.hip is compiled once per coupled rank with -DAP_RANK_L=<L>"
#endif

namespace ap {

template <>
const void* rank_kernel<AP_RANK_L>(bool xo) {
  constexpr int L = AP_RANK_L;
  return xo ? (const void*)k_ace_rank<L, kMixRtw[L], L + 1, true>
            : (const void*)k_ace_rank<L, kMixRtw[L], L + 1, false>;
}

}  // namespace ap
