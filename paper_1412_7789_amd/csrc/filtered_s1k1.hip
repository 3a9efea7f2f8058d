// Filtered-scan kernels of stride 1, prefix length 1 (see filtered.hpp).
#include "filtered.hpp"

namespace pfac {

dev::FilteredFn pick_filtered_s1k1(int kind, int segs) { return dev::pick_filter<1, 1>(kind, segs); }

}  // namespace pfac
