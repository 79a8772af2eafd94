// Pair kernel instantiation for order 2.
#include "pair.hpp"

namespace mmvm {
template hipError_t launch_pair_M<2>(const DevTables&, const StageBufs&, int, bool, PairShape,
                                               hipStream_t);
}
