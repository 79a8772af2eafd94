// Pair kernel instantiation for order 0.
#include "pair.hpp"

namespace mmvm {
template hipError_t launch_pair_M<0>(const DevTables&, const StageBufs&, int, bool, PairShape,
                                               hipStream_t);
}
