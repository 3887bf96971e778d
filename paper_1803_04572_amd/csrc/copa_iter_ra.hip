// Instantiates the iteration kernels of ranks 1, 2, 3, 4, 5, 6, 7, 8 (one of several
// translation units so that the ranks compile in parallel).
#include "copa_iter_impl.h"

namespace copa {
template struct RankOps<1>;
template struct RankOps<2>;
template struct RankOps<3>;
template struct RankOps<4>;
template struct RankOps<5>;
template struct RankOps<6>;
template struct RankOps<7>;
template struct RankOps<8>;
}  // namespace copa
