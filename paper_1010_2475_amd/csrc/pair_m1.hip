// Pair kernel instantiation for order 1.
#include "pair.hpp"

namespace mmvm {
template hipError_t launch_pair_M<1>(const DevTables&, const StageBufs&, int, bool, PairShape,
                                               hipStream_t);
}
