// root.hpp -- buffers and launchers of the root passes (root.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vc {

// device counters (uint32 slots of RootBufs::ctr)
enum {
    CTR_INVALID = 0,    // validation failure bits
    CTR_UNSORTED = 1,   // some row is not strictly increasing
    CTR_SROOT = 2,      // vertices the root reduction put in the cover
    CTR_FIRED = 4,      // rule firings of the last two rounds (2 slots)
    CTR_GLIVE = 6,      // greedy: live vertices seen this round (2 slots)
    CTR_GSIZE = 8,      // greedy cover size
    CTR_MAXDEG = 9,     // maximum degree of the induced subgraph
    CTR_CROWN_F = 10,   // crown: three rotating BFS frontier sizes
    CTR_CROWN_E = 13,   // crown: augmenting paths found this phase
    CTR_CROWN_M = 14,   // crown: vertices matched by the last proposal rounds
    CTR_CROWN_H = 15,   // crown: |H| of the last crown
    CTR_CROWN_I = 16,   // crown: |I| summed over the crowns of a solve
    CTR_ROUNDS = 17,    // reduction rounds run inside one workgroup (small graphs)
    CTR_COUNT = 24
};

struct RootGraph {
    uint32_t n;
    uint64_t nnz;
    const uint32_t* off;  // device
    const void* col;      // device
    uint32_t col_bytes;
    int sorted = 0;       // every row strictly increasing (known to the checks)
};

struct RootBufs {
    uint32_t* rdeg;      // [n]   root degrees (all ones = in the cover)
    uint32_t* gdeg;      // [n]   greedy working degrees
    uint8_t* gin;        // [n]   greedy cover flags
    uint8_t* addf;       // [n]   per-round selection flags
    uint8_t* newly;      // [n]   per-round newly covered flags
    uint32_t* flags;     // [n+1] scan input (live flags, cover flags)
    uint32_t* newid;     // [n+1] old -> new ids (also a scan output)
    uint32_t* oldid;     // [n]   new -> old ids
    uint32_t* kdeg;      // [n+1] degrees of the induced subgraph
    uint32_t* koff;      // [n+1] offsets of the induced subgraph
    void* kcol;          // [nnz] columns of the induced subgraph
    uint32_t* cover;     // [n]   final cover, ascending ids
    uint32_t* scan_tmp;  // [n / 2048 + 2]
    uint32_t* ctr;       // [CTR_COUNT]
    unsigned long long* hsum;
    uint32_t* cw = nullptr;  // [8n] crown workspace
    uint32_t* hm = nullptr;  // [16] pinned host words for the steps' read-backs
};

// The row check's symmetry hash is summed over HSUM_SLOTS 64-bit words (one
// word per wave would make every wave's atomic meet at one address); the
// caller provides and zeroes them (hsum), and the check folds them into
// hsum[0].
constexpr uint32_t HSUM_SLOTS = 64;

// hm: 4 words of pinned host memory for the read-back
hipError_t root_validate(const RootGraph& g, uint32_t* ctr, unsigned long long* hsum,
                         hipStream_t st, uint32_t* hm, uint32_t* bad_host,
                         int* sorted_host = nullptr);
hipError_t root_init(const RootGraph& g, const RootBufs& b, hipStream_t st);
hipError_t root_greedy(const RootGraph& g, const RootBufs& b, hipStream_t st, uint32_t* rounds);
// restart the greedy on the vertices the root rules left (gdeg from rdeg,
// the forced vertices already in the greedy cover)
hipError_t root_greedy_rest(const RootGraph& g, const RootBufs& b, hipStream_t st);
hipError_t root_reduce(const RootGraph& g, const RootBufs& b, int best0, hipStream_t st,
                       uint32_t max_rounds, uint32_t* rounds);
// keep_all: every input vertex keeps its id (isolated ones with degree 0)
hipError_t root_induce_a(const RootGraph& g, const RootBufs& b, hipStream_t st,
                         bool keep_all = false);
hipError_t root_induce_b(const RootGraph& g, const RootBufs& b, uint32_t np, uint32_t kcol_bytes,
                         hipStream_t st);
hipError_t root_cover(const RootGraph& g, const RootBufs& b, uint32_t np, int improved,
                      const uint32_t* root_bitmap, hipStream_t st);
// One crown reduction (crown.hip): H into the cover (counted in
// CTR_SROOT), I removed, their edges dropped.  *h_out = |H| (0: no crown).
hipError_t root_crown(const RootGraph& g, const RootBufs& b, hipStream_t st, uint32_t* h_out);
hipError_t scan_u32(const uint32_t* in, uint32_t N, uint32_t* out, uint32_t* tmp,
                    hipStream_t st);

}  // namespace vc
