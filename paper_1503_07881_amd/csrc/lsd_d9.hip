// LSD radix sort passes on 9-bit digits (the pass kernels are in lsd.h).
#include "lsd.h"

namespace ringo {
template hipError_t launch_sort_part_rb<9>(const SortLaunch &, int, int, int, hipStream_t);
}  // namespace ringo
