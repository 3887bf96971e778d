// Instantiates the iteration kernels of ranks 20, 24 (one of several
// translation units so that the ranks compile in parallel).
#include "copa_iter_impl.h"

namespace copa {
template struct RankOps<20>;
template struct RankOps<24>;
}  // namespace copa
