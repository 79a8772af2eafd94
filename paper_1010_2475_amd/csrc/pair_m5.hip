// Pair kernel instantiation for order 5.
#include "pair.hpp"

namespace mmvm {
template hipError_t launch_pair_M<5>(const DevTables&, const StageBufs&, int, bool, PairShape,
                                               hipStream_t);
}
