// search_deg.hip -- one degree-array type of the search kernel per object
// (compiled with VC_DEG_BYTES = 1, 2 or 4), so the three instantiations
// build in parallel.
#include "search_worker.hpp"

#ifndef VC_DEG_BYTES
#error "compile with -DVC_DEG_BYTES=1, 2 or 4"
#endif

namespace vc {

#if VC_DEG_BYTES == 1
using DegT = uint8_t;
#define VC_SUFFIX(x) x##_d1
#elif VC_DEG_BYTES == 2
using DegT = uint16_t;
#define VC_SUFFIX(x) x##_d2
#else
using DegT = uint32_t;
#define VC_SUFFIX(x) x##_d4
#endif

hipError_t VC_SUFFIX(launch_search)(const SearchArgs& a, uint32_t workers, hipStream_t st) {
    return launch_t<DegT>(a, workers, st);
}
hipError_t VC_SUFFIX(search_occupancy)(uint32_t lds_bytes, int* bpc) {
    return occ_t<DegT>(lds_bytes, bpc);
}
hipError_t VC_SUFFIX(launch_search_init)(const SearchArgs& a, int best0, const uint32_t* kdeg,
                                          uint32_t blocks, hipStream_t st) {
    return init_t<DegT>(a, best0, kdeg, blocks, st);
}

}  // namespace vc
