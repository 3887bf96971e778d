// Instantiates the iteration kernels of ranks 10, 12 (one of several
// translation units so that the ranks compile in parallel).
#include "copa_iter_impl.h"

namespace copa {
template struct RankOps<10>;
template struct RankOps<12>;
}  // namespace copa
