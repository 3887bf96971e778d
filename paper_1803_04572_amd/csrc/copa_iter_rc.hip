// Instantiates the iteration kernels of ranks 15, 16 (one of several
// translation units so that the ranks compile in parallel).
#include "copa_iter_impl.h"

namespace copa {
template struct RankOps<15>;
template struct RankOps<16>;
}  // namespace copa
