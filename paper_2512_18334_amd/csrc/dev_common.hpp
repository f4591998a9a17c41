// dev_common.hpp -- wave64 primitives and scoped atomics shared by the
// libvc kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define VC_WAVE 64

namespace vc {

// ----------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return __popcll(m); }

__device__ __forceinline__ uint32_t shfl(uint32_t x, uint32_t src) {
    return (uint32_t)__shfl((int)x, (int)src, 64);
}

// Cross-lane scans with DPP: row_shr by 1, 2, 4, 8 inside each 16-lane row,
// then row_bcast 15 and 31 carry rows 0 -> 1, 2 -> 3 and rows 0-1 -> 2-3.
// Lanes without a source read `id` (0 for sums, 0 / ~0 for max / min).
#define VC_DPP_SCAN(x, op, id)                                                     \
    do {                                                                           \
        uint32_t _t;                                                               \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x111, 0xf, 0xf, false); x = op(x, _t); \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x112, 0xf, 0xf, false); x = op(x, _t); \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x114, 0xf, 0xf, false); x = op(x, _t); \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x118, 0xf, 0xf, false); x = op(x, _t); \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x142, 0xa, 0xf, false); x = op(x, _t); \
        _t = __builtin_amdgcn_update_dpp(id, x, 0x143, 0xc, 0xf, false); x = op(x, _t); \
    } while (0)

__device__ __forceinline__ uint32_t op_add(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint32_t op_max(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t op_min(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t op_or(uint32_t a, uint32_t b) { return a | b; }

// bitwise OR of a 64-bit value over the 64 lanes (wave-uniform result)
__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    VC_DPP_SCAN(lo, op_or, 0u);
    VC_DPP_SCAN(hi, op_or, 0u);
    // (readlane returns int: widen through uint32_t, never by sign extension)
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 63) << 32) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo, 63);
}

// inclusive prefix sum across the 64 lanes
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    VC_DPP_SCAN(x, op_add, 0u);
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
    VC_DPP_SCAN(x, op_add, 0u);
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
    VC_DPP_SCAN(x, op_max, 0u);
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    VC_DPP_SCAN(x, op_min, 0xFFFFFFFFu);
    return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    // exact modulo 2^64: the two low 16-bit fields cannot carry out of 32
    // bits over 64 lanes, the high word wraps exactly as the full sum does
    const uint64_t a = wave_sum((uint32_t)(x & 0xFFFFu));
    const uint64_t b = wave_sum((uint32_t)((x >> 16) & 0xFFFFu));
    const uint64_t c = wave_sum((uint32_t)(x >> 32));
    return a + (b << 16) + (c << 32);
}

// max of a 64-bit key: the largest high word, then the largest low word
// among the lanes that hold it
__device__ __forceinline__ uint64_t wave_max64(uint64_t x) {
    const uint32_t hi = wave_max((uint32_t)(x >> 32));
    const uint32_t lo = wave_max((uint32_t)(x >> 32) == hi ? (uint32_t)x : 0u);
    return ((uint64_t)hi << 32) | lo;
}

// Order LDS traffic between the lanes of one wave (a worker is one wave and
// the whole workgroup).  The LDS executes a wave's instructions in issue
// order, so no wait is needed in hardware; the wavefront-scope fences keep
// the compiler from moving LDS accesses across this point or forwarding a
// lane's own store to a later load that another lane may have overwritten.
// Unlike a workgroup barrier, it does not wait for global memory traffic.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ atomics
// Agent scope = the whole GPU (all XCDs).  Relaxed operations are used for
// counters whose value is the only data; acquire/release only where a
// payload (node, cover bitmap) is published to another worker.

__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acquire(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_relaxed(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_relaxed(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t add_relaxed(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_acq_rel(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_release(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int min_relaxed(int* p, int v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void fence_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
__device__ __forceinline__ void fence_seq() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
}
__device__ __forceinline__ bool cas_acquire(int* p, int expect, int desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_ACQUIRE,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_relaxed64(uint64_t* p, uint64_t expect, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent accesses for data that crosses workers (worklist payloads,
// cover bitmaps): relaxed agent-scope atomic loads and stores, which compile
// to global_load/store with the device-scope cache policy, so a reader on
// another XCD never sees a stale cached copy.
__device__ __forceinline__ void st_coh(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_coh64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every memory operation this wave issued has completed.  With
// all cross-worker data moved by coherent accesses, this is the ordering
// point between writing a payload and publishing it (and between the two
// halves of a registry update), without the whole-cache write-back and
// invalidate an agent-scope fence costs on a multi-XCD part.
__device__ __forceinline__ void order_point() {
    // compiler fences on both sides: no memory access of any lane moves
    // across the wait
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// idle wait: short sleeps first, then 63 x 64 clocks (about 1.7 us) per
// round (longer sleeps, up to 8 x that, made the blocks-and-hubs search 4%
// slower: idle workers picked up donated nodes later)
__device__ __forceinline__ void backoff(uint32_t& spins) {
    if (spins < 4) {
        __builtin_amdgcn_s_sleep(2);
    } else {
        __builtin_amdgcn_s_sleep(63);
    }
    ++spins;
}

// ----------------------------------------------- packed degrees in LDS
// A degree array of element type D (uint8/uint16/uint32) lives in LDS as
// 32-bit words; element v is bits [8*sizeof(D)*(v%per), +8*sizeof(D)) of
// word v/per.  The all-ones value marks "in the cover"; 0 marks a vertex
// with no remaining edge; anything else is the live degree.

template <typename D>
struct Deg {
    static constexpr uint32_t per = 4u / sizeof(D);
    static constexpr uint32_t bits = 8u * sizeof(D);
    static constexpr uint32_t IN = (uint32_t)(D)(~(D)0);

    __device__ static __forceinline__ uint32_t get(const D* a, uint32_t v) {
        return (uint32_t)a[v];
    }
    __device__ static __forceinline__ void set(D* a, uint32_t v, uint32_t x) {
        a[v] = (D)x;
    }
    __device__ static __forceinline__ bool live(uint32_t d) {
        return d != 0u && d != IN;
    }
    // atomic decrement of a live entry (never underflows: callers only
    // decrement once per live edge)
    __device__ static __forceinline__ void dec(D* a, uint32_t v) {
        uint32_t* w = reinterpret_cast<uint32_t*>(a);
        atomicSub(&w[v / per], 1u << ((v % per) * bits));
    }
    // atomically mark v as in the cover; true if it was not marked before
    __device__ static __forceinline__ bool mark_in(D* a, uint32_t v) {
        uint32_t* w = reinterpret_cast<uint32_t*>(a);
        uint32_t sh = (v % per) * bits;
        uint32_t old = atomicOr(&w[v / per], IN << sh);
        return ((old >> sh) & IN) != IN;
    }
};

// ------------------------------------------------------------- row check
// One wave checks one adjacency row, entries [o0, o1), of vertex v in a graph
// of ni vertices.  Lanes stride the row: every entry must be below ni and
// differ from v, and each adds its signed pair hash to the lane's *hs (the
// callers' symmetry test).  A row that is not strictly increasing is then
// checked for repeats with an open-addressing table in LDS: ROWCHK_CHUNK
// entries at a time are inserted (a repeat inside the chunk meets its twin),
// and the rest of the row is looked up against them.  tbl is this wave's
// ROWCHK_TBL words of LDS.  Returns ROWCHK_ENTRY and/or ROWCHK_REPEAT, the
// same on every lane, plus ROWCHK_UNSORTED when the row is not strictly
// increasing.
// (4 waves of a block take 16 KB: the validation runs beside a resident
// search kernel, which leaves 32 KB of LDS per CU to the side stream)
constexpr uint32_t ROWCHK_TBL = 1024u;    // LDS words per wave
constexpr uint32_t ROWCHK_CHUNK = 512u;   // entries per pass (load <= 1/2)
constexpr uint32_t ROWCHK_EMPTY = 0xFFFFFFFFu;
constexpr uint32_t ROWCHK_ENTRY = 1u;     // an entry out of range or equal to v
constexpr uint32_t ROWCHK_REPEAT = 2u;    // an entry repeated in the row
constexpr uint32_t ROWCHK_UNSORTED = 4u;  // the row is not strictly increasing

__device__ __forceinline__ uint32_t rowchk_slot(uint32_t w) {
    return (w * 0x9E3779B1u) >> 22;  // 10 bits: ROWCHK_TBL slots
}

static_assert(4u * 4u * ROWCHK_TBL <= 16384u, "row-check LDS exceeds the serving reserve");
static_assert(ROWCHK_TBL == 1024u, "rowchk_slot yields 10 bits");

template <typename Col, typename Hash>
__device__ __forceinline__ uint32_t wave_row_check(uint32_t v, uint32_t ni, uint32_t o0,
                                                   uint32_t o1, Col col, Hash hash,
                                                   uint32_t* tbl, uint64_t* hs) {
    const uint32_t l = threadIdx.x & 63u;
    uint32_t bad = 0;
    bool unsorted = false;
    uint64_t acc = 0;
    for (uint32_t e = o0 + l; e < o1; e += 64u) {
        const uint32_t w = col(e);
        if (w >= ni || w == v) bad |= ROWCHK_ENTRY;
        if (e > o0 && col(e - 1u) >= w) unsorted = true;
        acc += hash(v, w);
    }
    *hs += acc;
    if (ballot(unsorted) != 0ull) {
        for (uint32_t c0 = o0; c0 < o1; c0 += ROWCHK_CHUNK) {
            const uint32_t c1 = o1 - c0 > ROWCHK_CHUNK ? c0 + ROWCHK_CHUNK : o1;
            for (uint32_t i = l; i < ROWCHK_TBL; i += 64u) tbl[i] = ROWCHK_EMPTY;
            wave_sync();
            for (uint32_t e = c0 + l; e < c1; e += 64u) {
                const uint32_t w = col(e);
                if (w == ROWCHK_EMPTY) continue;  // out of range: flagged above
                uint32_t h = rowchk_slot(w);
                for (uint32_t p = 0; p < ROWCHK_TBL; ++p) {
                    const uint32_t prev = atomicCAS(&tbl[h], ROWCHK_EMPTY, w);
                    if (prev == ROWCHK_EMPTY) break;
                    if (prev == w) {
                        bad |= ROWCHK_REPEAT;
                        break;
                    }
                    h = (h + 1u) & (ROWCHK_TBL - 1u);
                }
            }
            wave_sync();
            for (uint32_t e = c1 + l; e < o1; e += 64u) {
                const uint32_t w = col(e);
                uint32_t h = rowchk_slot(w);
                for (uint32_t p = 0; p < ROWCHK_TBL; ++p) {
                    const uint32_t t = tbl[h];
                    if (t == ROWCHK_EMPTY) break;
                    if (t == w) {
                        bad |= ROWCHK_REPEAT;
                        break;
                    }
                    h = (h + 1u) & (ROWCHK_TBL - 1u);
                }
            }
            wave_sync();  // lookups done before the next chunk clears tbl
            if (ballot(bad & ROWCHK_REPEAT) != 0ull) break;
        }
    }
    uint32_t out = 0;
    if (ballot(unsorted) != 0ull) out |= ROWCHK_UNSORTED;
    if (ballot(bad & ROWCHK_ENTRY) != 0ull) out |= ROWCHK_ENTRY;
    if (ballot(bad & ROWCHK_REPEAT) != 0ull) out |= ROWCHK_REPEAT;
    return out;
}

}  // namespace vc
