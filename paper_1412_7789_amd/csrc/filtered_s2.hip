// Filtered-scan kernels of stride 2 (see filtered.hpp).
#include "filtered.hpp"

namespace pfac {

dev::FilteredFn pick_filtered_s2(int kind, int segs) { return dev::pick_filter<3, 2>(kind, segs); }

}  // namespace pfac
