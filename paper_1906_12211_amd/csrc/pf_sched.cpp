// Learned scheduler: placeholder until the MLP is built.
#include "pf_internal.h"

namespace pf {
std::vector<int32_t> learned_order(Index &, const uint32_t *, const uint64_t *, int64_t, hipStream_t) {
    throw Error(PF_EUNSUPPORTED, "learned scheduler not built");
}
} // namespace pf
