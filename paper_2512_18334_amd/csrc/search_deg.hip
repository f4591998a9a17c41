// search_deg.hip -- one degree-array type of the search kernel per object
// (compiled with VC_DEG_BYTES = 1, 2 or 4, and VC_HL = 1 for the variant
// whose lists live in HBM), so the instantiations build in parallel.
#include "search_worker.hpp"

#ifndef VC_DEG_BYTES
#error "compile with -DVC_DEG_BYTES=1, 2 or 4"
#endif

namespace vc {

#ifndef VC_HL
#define VC_HL 0
#endif

#if VC_DEG_BYTES == 1
using DegT = uint8_t;
#if VC_HL
#define VC_SUFFIX(x) x##_d1h
#else
#define VC_SUFFIX(x) x##_d1
#endif
#elif VC_DEG_BYTES == 2
using DegT = uint16_t;
#if VC_HL
#define VC_SUFFIX(x) x##_d2h
#else
#define VC_SUFFIX(x) x##_d2
#endif
#else
using DegT = uint32_t;
#if VC_HL
#define VC_SUFFIX(x) x##_d4h
#else
#define VC_SUFFIX(x) x##_d4
#endif
#endif

hipError_t VC_SUFFIX(launch_search)(const SearchArgs& a, uint32_t workers, hipStream_t st) {
    return launch_t<DegT, VC_HL != 0>(a, workers, st);
}
hipError_t VC_SUFFIX(search_occupancy)(uint32_t lds_bytes, int* bpc) {
    return occ_t<DegT, VC_HL != 0>(lds_bytes, bpc);
}
#if !VC_HL
hipError_t VC_SUFFIX(launch_search_init)(const SearchArgs& a, int best0, const uint32_t* kdeg,
                                          uint32_t blocks, hipStream_t st) {
    return init_t<DegT>(a, best0, kdeg, blocks, st);
}
#endif

}  // namespace vc
