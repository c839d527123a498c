// The search kernels of k_search.hip instantiated for indexes whose table positions are
// stored in 3 bytes (pos_bytes = 3), in a translation unit of their own so that the two
// sets of kernels compile in parallel.
#define PF_SEARCH_KERNELS_ONLY
#include "k_search.hip"

namespace pf {

const void *search_kernel_pos3(int dt, int tile, bool shared) { return search_kernel_of<3>(dt, tile, shared); }

} // namespace pf
