// Instantiates the iteration kernels of ranks 32 (one of several
// translation units so that the ranks compile in parallel).
#include "copa_iter_impl.h"

namespace copa {
template struct RankOps<32>;
}  // namespace copa
