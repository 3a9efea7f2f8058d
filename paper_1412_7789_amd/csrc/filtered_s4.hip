// Filtered-scan kernels of stride 4 (see filtered.hpp).
#include "filtered.hpp"

namespace pfac {

dev::FilteredFn pick_filtered_s4(int kind, int segs) { return dev::pick_filter<3, 4>(kind, segs); }

}  // namespace pfac
