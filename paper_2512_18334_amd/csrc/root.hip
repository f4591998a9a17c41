// root.hip -- grid-wide passes over the input graph before the search:
// CSR validation, degrees, the greedy initial bound (Sec. II-B), the root
// reduction to a fixpoint (Sec. IV-B), inducing the subgraph on the
// remaining vertices with narrow column ids, and assembling the final cover.
// These kernels stream the CSR from HBM; each is a grid-stride loop with one
// vertex per thread.
#include <algorithm>

#include "dev_common.hpp"
#include "internal.hpp"
#include "root.hpp"

namespace vc {

constexpr uint32_t RIN = 0xFFFFFFFFu;  // root degree array: in the cover

__device__ __forceinline__ bool rlive(uint32_t d) { return d != 0u && d != RIN; }

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// one atomic per wave: every lane of the block must call this
__device__ __forceinline__ void wave_atomic_add(uint32_t* p, uint32_t x) {
    x = wave_sum(x);
    if ((threadIdx.x & 63u) == 0 && x) atomicAdd(p, x);
}

// one atomic per 256-thread block: in a round where most vertices change,
// one atomic per wave on a single counter serialises (16K of them for a
// million vertices); every thread of the block must call it
__device__ __forceinline__ void block_atomic_add(uint32_t* p, uint32_t x) {
    __shared__ uint32_t part[4];
    x = wave_sum(x);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(p, t);
    }
}

// LDS of the root-step kernels.  They also run on a served context's side
// stream beside its resident search, which leaves 32 KB of LDS per CU to
// them, so none may take more than 16 KB per block (a kernel that could not
// be placed would wait for the resident search forever); each is launched
// with 256 threads, which its __launch_bounds__ states, except the
// one-workgroup kernels of small graphs (1,024 threads, a few words of LDS).
constexpr uint32_t SIDE_LDS_MAX = 16384u;
static_assert(sizeof(uint32_t) * 4u * ROWCHK_TBL <= SIDE_LDS_MAX, "k_check_rows table");
static_assert(sizeof(uint32_t) * 4u <= SIDE_LDS_MAX, "block_atomic_add partial sums");

#define GRID_LOOP(i, n)                                                        \
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (n);          \
         i += gridDim.x * blockDim.x)

// one wave per vertex (its lanes stride the row), so a hub's row costs one
// pass instead of one thread walking it alone
#define WAVE_LOOP(v, n)                                                        \
    for (uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < (n);   \
         v += (gridDim.x * blockDim.x) >> 6)

// ------------------------------------------------------------- validation

// offsets: off[0] == 0, non-decreasing, off[n] == nnz
__global__ void __launch_bounds__(256) k_check_offsets(uint32_t n, uint64_t nnz, const uint32_t* off, uint32_t* ctr) {
    GRID_LOOP(v, n) {
        if (off[v] > off[v + 1]) atomicOr(&ctr[CTR_INVALID], 1u);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (off[0] != 0u || (uint64_t)off[n] != nnz) atomicOr(&ctr[CTR_INVALID], 2u);
    }
}

// Rows: ids < n, no self-loop, no repeated entry, symmetric.  The entries
// of 64 consecutive rows are contiguous in the CSR, so a wave walks them flat,
// 64 entries per step with one coalesced load: each entry finds its row by
// the marks its row's start leaves in 64 words of LDS (an inclusive
// max-scan), and compares itself with the entry before it (the lane to its
// left, or the last entry of the previous step).  Rows that are not strictly
// increasing are then checked for repeats one by one (a lane per short row,
// the whole wave per long row).  Symmetry: the signed sum of a hash of each
// unordered pair over all entries vanishes when every entry has its mirror
// (an asymmetric graph passes only on a hash collision).
template <typename C>
__global__ void __launch_bounds__(256) k_check_rows(uint32_t n, const uint32_t* off, const C* col,
                                                    uint32_t* ctr, unsigned long long* hsum) {
    // (16 KB: the row marks use the first 64 words of the wave's repeat
    // table, which is only needed after the flat walk of a block of rows)
    __shared__ uint32_t tbl_all[4 * ROWCHK_TBL];
    uint32_t* tbl = tbl_all + (threadIdx.x >> 6) * ROWCHK_TBL;
    uint32_t* MK = tbl;
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    auto hash = [](uint32_t v, uint32_t w) -> uint64_t {
        const uint64_t a = v < w ? v : w, b = v < w ? w : v;
        const uint64_t h = mix64(a * 0x9E3779B97F4A7C15ull + b);
        return v < w ? h : (0ull - h);
    };
    // the offsets check ran before on the same stream: with bad offsets the
    // rows are not walked (their bounds could lie outside the columns)
    if (ctr[CTR_INVALID]) return;
    auto cl = [col](uint32_t e) -> uint32_t { return (uint32_t)col[e]; };
    uint64_t acc = 0;
    uint32_t bad = 0;
    bool uns = false;
    for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
        const uint32_t v = base + l;
        const uint32_t last = (n - base < 64u ? n - base : 64u) - 1u;  // last row's lane
        const uint32_t r0 = v < n ? off[v] : 0u, r1 = v < n ? off[v + 1] : 0u;
        const uint32_t start = __builtin_amdgcn_readfirstlane(r0);
        const uint32_t end = __builtin_amdgcn_readlane(r1, last);
        bool row_uns = false;  // this lane's row is not strictly increasing
        uint32_t carry = 0, wprev = 0;
        // the columns of the next two chunks are loaded ahead, so three
        // loads per wave are in flight while a chunk is checked
        uint32_t wa = start + l < end ? cl(start + l) : 0u;
        uint32_t wb = start + 64u + l < end ? cl(start + 64u + l) : 0u;
        for (uint32_t t0 = start; t0 < end; t0 += 64u) {
            const uint32_t e2 = t0 + 128u + l;
            const uint32_t wc = e2 < end ? cl(e2) : 0u;
            wave_sync();  // the previous step's reads of MK are done
            MK[l] = 0u;
            wave_sync();
            if (v < n && r1 > r0 && r0 >= t0 && r0 - t0 < 64u) MK[r0 - t0] = l + 1u;
            wave_sync();  // every row start is marked
            uint32_t own = MK[l];
            VC_DPP_SCAN(own, op_max, 0u);
            own = own > carry ? own : carry;
            carry = __builtin_amdgcn_readlane(own, 63);
            const uint32_t jr = own - 1u;  // lane of this entry's row
            const uint32_t e = t0 + l;
            const bool ok = e < end;
            const uint32_t w = ok ? wa : 0u;
            wa = wb;
            wb = wc;
            const uint32_t rv = base + jr;
            const uint32_t rs = shfl(r0, jr);
            // the entry before, in CSR order
            uint32_t p = shfl(w, l ? l - 1u : 0u);
            if (l == 0) p = wprev;
            wprev = __builtin_amdgcn_readlane(w, 63);
            bool unsorted_here = false;
            if (ok) {
                if (w >= n) {
                    bad |= 4u;
                } else {
                    if (w == rv) bad |= 8u;
                    acc += hash(rv, w);
                }
                if (e > rs && p >= w) unsorted_here = true;
            }
            // tell the row's lane
            uint64_t um = ballot(unsorted_here);
            while (um) {
                const uint32_t k = (uint32_t)__builtin_ctzll(um);
                um &= um - 1ull;
                if (l == shfl(jr, k)) row_uns = true;
            }
        }
        wave_sync();  // the marks are read before the repeat table is reused
        // repeats, in the rows that are not increasing
        if (row_uns) uns = true;
        const bool longrow = row_uns && r1 - r0 > 32u;
        if (row_uns && !longrow)
            for (uint32_t e = r0; e < r1; ++e)
                for (uint32_t f = e + 1; f < r1; ++f)
                    if (col[e] == col[f]) bad |= 16u;
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j2 = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            uint64_t unused = 0;
            const uint32_t r = wave_row_check(base + j2, n, shfl(r0, j2), shfl(r1, j2), cl, hash,
                                              tbl, &unused);
            if (r & ROWCHK_REPEAT) bad |= 16u;
        }
    }
    if (bad) atomicOr(&ctr[CTR_INVALID], bad);
    if (ballot(uns) != 0ull && l == 0) atomicOr(&ctr[CTR_UNSORTED], 1u);
    acc = wave_sum64(acc);
    if (l == 0 && acc) atomicAdd(&hsum[wave % HSUM_SLOTS], (unsigned long long)acc);
}

// hsum[0] = the sum of the HSUM_SLOTS partial hash sums (one wave)
__global__ void __launch_bounds__(64) k_hsum_fold(unsigned long long* hsum) {
    const uint32_t l = threadIdx.x;
    uint64_t x = l < HSUM_SLOTS ? (uint64_t)hsum[l] : 0ull;
    x = wave_sum64(x);
    if (l == 0) hsum[0] = (unsigned long long)x;
}

// ------------------------------------------------------------- degrees

__global__ void __launch_bounds__(256) k_init(uint32_t n, const uint32_t* off, uint32_t* rdeg, uint32_t* gdeg,
                       uint8_t* gin, uint8_t* addf, uint8_t* newly) {
    GRID_LOOP(v, n) {
        uint32_t d = off[v + 1] - off[v];
        rdeg[v] = d;
        gdeg[v] = d;
        gin[v] = 0;
        addf[v] = 0;
        newly[v] = 0;
    }
}

// ------------------------------------------------------------- greedy
// Parallel max-degree greedy: each round takes every vertex whose key
// (degree, then lower id) beats all its live neighbours' keys; these form
// an independent set, so taking them together is well defined.

template <typename C>
__global__ void __launch_bounds__(256) k_greedy_select(uint32_t n, const uint32_t* off, const C* col,
                                const uint32_t* gdeg, uint8_t* sel, uint32_t* ctr_live) {
    // 64 consecutive vertices per wave, one per lane; a row longer than 32
    // entries is walked by the whole wave together (hubs take one pass)
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    uint32_t live = 0;
    for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
        const uint32_t v = base + l;
        const uint32_t d = v < n ? gdeg[v] : 0u;
        const uint32_t r0 = v < n ? off[v] : 0u, r1 = v < n ? off[v + 1] : 0u;
        const uint64_t kv = ((uint64_t)d << 32) | (uint32_t)~v;
        const bool longrow = d != 0u && r1 - r0 > 32u;
        bool top = d != 0u;
        if (d != 0u) ++live;
        if (d != 0u && !longrow) {
            for (uint32_t e = r0; e < r1 && top; ++e) {
                const uint32_t u = (uint32_t)col[e];
                const uint32_t du = gdeg[u];
                if (du && (((uint64_t)du << 32) | (uint32_t)~u) > kv) top = false;
            }
        }
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t a = shfl(r0, j), b = shfl(r1, j);
            const uint32_t vj = shfl(v, j), dj = shfl(d, j);
            const uint64_t kj = ((uint64_t)dj << 32) | (uint32_t)~vj;
            bool beaten = false;
            for (uint32_t e = a + l; e < b; e += 64) {
                const uint32_t u = (uint32_t)col[e];
                const uint32_t du = gdeg[u];
                if (du && (((uint64_t)du << 32) | (uint32_t)~u) > kj) beaten = true;
            }
            const bool any = ballot(beaten) != 0ull;
            if (l == j) top = !any;
        }
        if (top) sel[v] = 1;
    }
    wave_atomic_add(ctr_live, live);
}

template <typename C>
__global__ void __launch_bounds__(256) k_greedy_apply(uint32_t n, const uint32_t* off, const C* col, uint32_t* gdeg,
                               uint8_t* sel, uint8_t* gin, const uint32_t* ctr_live,
                               uint32_t* ctr_size) {
    if (*ctr_live == 0) return;
    const uint32_t l = threadIdx.x & 63u;
    uint32_t taken = 0;
    WAVE_LOOP(v, n) {
        if (!sel[v]) continue;
        // selected vertices are never adjacent (strict local maxima), so
        // every neighbour still has the edge to v: no underflow
        const uint32_t r1 = off[v + 1];
        for (uint32_t e = off[v] + l; e < r1; e += 64) {
            const uint32_t u = (uint32_t)col[e];
            if (gdeg[u]) atomicSub(&gdeg[u], 1u);
        }
        if (l == 0) {
            sel[v] = 0;
            gin[v] = 1;
            gdeg[v] = 0;
            ++taken;
        }
    }
    wave_atomic_add(ctr_size, taken);
}

// the greedy restarted on what the root rules left: working degrees of the
// live vertices only, and the vertices the rules forced already in its cover
__global__ void __launch_bounds__(256) k_greedy_rest(uint32_t n, const uint32_t* rdeg, uint32_t* gdeg, uint8_t* gin) {
    GRID_LOOP(v, n) {
        const uint32_t d = rdeg[v];
        gdeg[v] = rlive(d) ? d : 0u;
        gin[v] = d == RIN ? 1 : 0;
    }
}

// ------------------------------------------------------------- root reduce
// One round = decide (rules on the state before the round, with the same
// tie-breaks as the search kernel), mark (flags -> in the cover), remove
// edges.  The bound is best0 - |S_root| - 1.

// is {u, w} an edge: the shorter row is searched, by bisection when every
// row is strictly increasing (power-law graphs pair hubs with long rows)
template <typename C>
__device__ __forceinline__ bool r_adjacent(const uint32_t* off, const C* col, uint32_t u,
                                           uint32_t w, int sorted) {
    uint32_t a = u, b = w;
    if (off[w + 1] - off[w] < off[u + 1] - off[u]) { a = w; b = u; }
    uint32_t lo = off[a], hi = off[a + 1];
    if (sorted) {
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            const uint32_t x = (uint32_t)col[mid];
            if (x == b) return true;
            if (x < b) lo = mid + 1u;
            else hi = mid;
        }
        return false;
    }
    for (uint32_t e = lo; e < hi; ++e)
        if ((uint32_t)col[e] == b) return true;
    return false;
}

template <typename C>
__global__ void __launch_bounds__(256) k_reduce_decide(uint32_t n, const uint32_t* off, const C* col,
                                const uint32_t* rdeg, uint8_t* addf, uint32_t* ctr,
                                uint32_t round, int best0, int sorted) {
    // the previous round fired nothing: the fixpoint is reached (this
    // round's count stays 0, so the rest of the group does nothing either)
    if (round > 0 && ctr[CTR_FIRED + ((round + 1u) & 1u)] == 0) return;
    const int s = (int)ctr[CTR_SROOT];
    const int64_t b = (int64_t)best0 - s - 1;
    uint32_t fired = 0;
    if (s >= best0) return;
    GRID_LOOP(v, n) {
        const uint32_t d = rdeg[v];
        if (!rlive(d)) continue;
        if ((int64_t)d > b) {
            addf[v] = 1;
            ++fired;
            continue;
        }
        if (d > 2u) continue;
        uint32_t u = NONE, w = NONE, got = 0;
        for (uint32_t e = off[v]; e < off[v + 1] && got < d; ++e) {
            uint32_t x = (uint32_t)col[e];
            if (rlive(rdeg[x])) {
                if (got == 0) u = x; else w = x;
                ++got;
            }
        }
        if (got < d) continue;
        if (d == 1u) {
            if (!(rdeg[u] == 1u && u < v)) {
                addf[u] = 1;
                ++fired;
            }
        } else if (r_adjacent(off, col, u, w, sorted)) {
            if (!(rdeg[u] == 2u && u < v) && !(rdeg[w] == 2u && w < v)) {
                addf[u] = 1;
                addf[w] = 1;
                ++fired;
            }
        }
    }
    block_atomic_add(&ctr[CTR_FIRED + (round & 1u)], fired);
}

__global__ void __launch_bounds__(256) k_reduce_mark(uint32_t n, uint32_t* rdeg, uint8_t* addf, uint8_t* newly,
                              uint32_t* ctr, uint32_t round) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_FIRED + ((round + 1u) & 1u)] = 0;
    if (ctr[CTR_FIRED + (round & 1u)] == 0) return;
    uint32_t added = 0;
    GRID_LOOP(v, n) {
        if (!addf[v]) continue;
        addf[v] = 0;
        if (rlive(rdeg[v])) {
            rdeg[v] = RIN;
            newly[v] = 1;
            ++added;
        }
    }
    block_atomic_add(&ctr[CTR_SROOT], added);
}

// Remove the edges of the vertices marked this round: a lane per marked
// vertex walks a short row, the whole wave a row longer than 16 entries.
template <typename C>
__global__ void __launch_bounds__(256) k_reduce_remove(uint32_t n, const uint32_t* off,
                                                       const C* col, uint32_t* rdeg,
                                                       uint8_t* newly, const uint32_t* ctr,
                                                       uint32_t round) {
    if (ctr[CTR_FIRED + (round & 1u)] == 0) return;  // nothing was marked
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
        const uint32_t v = base + l;
        const bool nw = v < n && newly[v];
        uint32_t r0 = 0, r1 = 0;
        if (nw) {
            newly[v] = 0;
            r0 = off[v];
            r1 = off[v + 1];
        }
        const bool longrow = nw && r1 - r0 > 16u;
        if (nw && !longrow) {
            for (uint32_t e = r0; e < r1; ++e) {
                const uint32_t u = (uint32_t)col[e];
                if (rlive(rdeg[u])) atomicSub(&rdeg[u], 1u);
            }
        }
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t a = shfl(r0, j), b = shfl(r1, j);
            for (uint32_t e = a + l; e < b; e += 64u) {
                const uint32_t u = (uint32_t)col[e];
                if (rlive(rdeg[u])) atomicSub(&rdeg[u], 1u);
            }
        }
    }
}

// ------------------------------------------------------------- small graphs
// Graphs of at most SMALL_N vertices run the rounds of the reduction, and
// of the greedy, inside one workgroup: the phases of a round (decide, mark,
// remove; select, apply) are separated by barriers instead of launches, and
// the host checks nothing between rounds.  Each phase does what the kernel
// of the same name does for the whole grid, on the same state.
constexpr uint32_t SMALL_N = 4096;
constexpr uint32_t SMALL_T = 1024;

template <typename C>
__global__ void __launch_bounds__(SMALL_T) k_reduce_small(uint32_t n, const uint32_t* off,
                                                          const C* col, uint32_t* rdeg,
                                                          uint8_t* addf, uint8_t* newly,
                                                          uint32_t* ctr, int best0, int sorted,
                                                          uint32_t max_rounds) {
    __shared__ uint32_t sh_fired, sh_added;
    __shared__ int sh_s;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t l = tid & 63u, wave = tid >> 6, waves = nt >> 6;
    if (tid == 0) sh_s = (int)ctr[CTR_SROOT];
    uint32_t r = 0;
    for (; r < max_rounds; ++r) {
        if (tid == 0) {
            sh_fired = 0;
            sh_added = 0;
        }
        __syncthreads();
        const int s = sh_s;
        if (s >= best0) break;
        const int64_t bnd = (int64_t)best0 - s - 1;
        // decide (on the state before the round)
        uint32_t fired = 0;
        for (uint32_t v = tid; v < n; v += nt) {
            const uint32_t d = rdeg[v];
            if (!rlive(d)) continue;
            if ((int64_t)d > bnd) {
                addf[v] = 1;
                ++fired;
                continue;
            }
            if (d > 2u) continue;
            uint32_t u = NONE, w = NONE, got = 0;
            for (uint32_t e = off[v]; e < off[v + 1] && got < d; ++e) {
                const uint32_t x = (uint32_t)col[e];
                if (rlive(rdeg[x])) {
                    if (got == 0) u = x; else w = x;
                    ++got;
                }
            }
            if (got < d) continue;
            if (d == 1u) {
                if (!(rdeg[u] == 1u && u < v)) {
                    addf[u] = 1;
                    ++fired;
                }
            } else if (r_adjacent(off, col, u, w, sorted)) {
                if (!(rdeg[u] == 2u && u < v) && !(rdeg[w] == 2u && w < v)) {
                    addf[u] = 1;
                    addf[w] = 1;
                    ++fired;
                }
            }
        }
        if (fired) atomicAdd(&sh_fired, fired);
        __syncthreads();
        if (sh_fired == 0) break;
        // mark
        uint32_t added = 0;
        for (uint32_t v = tid; v < n; v += nt) {
            if (!addf[v]) continue;
            addf[v] = 0;
            if (rlive(rdeg[v])) {
                rdeg[v] = RIN;
                newly[v] = 1;
                ++added;
            }
        }
        if (added) atomicAdd(&sh_added, added);
        __syncthreads();
        if (tid == 0) sh_s += (int)sh_added;
        // remove: a lane per marked vertex, the wave for a long row
        for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
            const uint32_t v = base + l;
            const bool nw = v < n && newly[v];
            uint32_t r0 = 0, r1 = 0;
            if (nw) {
                newly[v] = 0;
                r0 = off[v];
                r1 = off[v + 1];
            }
            const bool longrow = nw && r1 - r0 > 16u;
            if (nw && !longrow) {
                for (uint32_t e = r0; e < r1; ++e) {
                    const uint32_t u = (uint32_t)col[e];
                    if (rlive(rdeg[u])) atomicSub(&rdeg[u], 1u);
                }
            }
            uint64_t m = ballot(longrow);
            while (m) {
                const uint32_t j = (uint32_t)__builtin_ctzll(m);
                m &= m - 1ull;
                const uint32_t a = shfl(r0, j), b = shfl(r1, j);
                for (uint32_t e = a + l; e < b; e += 64u) {
                    const uint32_t u = (uint32_t)col[e];
                    if (rlive(rdeg[u])) atomicSub(&rdeg[u], 1u);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        ctr[CTR_SROOT] = (uint32_t)sh_s;
        ctr[CTR_ROUNDS] += r;
    }
}

template <typename C>
__global__ void __launch_bounds__(SMALL_T) k_greedy_small(uint32_t n, const uint32_t* off,
                                                          const C* col, uint32_t* gdeg,
                                                          uint8_t* sel, uint8_t* gin,
                                                          uint32_t* ctr) {
    __shared__ uint32_t sh_live, sh_taken;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t l = tid & 63u, wave = tid >> 6, waves = nt >> 6;
    uint32_t total = 0;
    for (uint32_t round = 0; round <= 4u * n + 8u; ++round) {
        if (tid == 0) {
            sh_live = 0;
            sh_taken = 0;
        }
        __syncthreads();
        // select: every live vertex whose (degree, lower id) beats all its
        // live neighbours' (rows longer than 32 entries by the whole wave)
        uint32_t live = 0;
        for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
            const uint32_t v = base + l;
            const uint32_t d = v < n ? gdeg[v] : 0u;
            const uint32_t r0 = v < n ? off[v] : 0u, r1 = v < n ? off[v + 1] : 0u;
            const uint64_t kv = ((uint64_t)d << 32) | (uint32_t)~v;
            const bool longrow = d != 0u && r1 - r0 > 32u;
            bool top = d != 0u;
            if (d != 0u) ++live;
            if (d != 0u && !longrow) {
                for (uint32_t e = r0; e < r1 && top; ++e) {
                    const uint32_t u = (uint32_t)col[e];
                    const uint32_t du = gdeg[u];
                    if (du && (((uint64_t)du << 32) | (uint32_t)~u) > kv) top = false;
                }
            }
            uint64_t m = ballot(longrow);
            while (m) {
                const uint32_t j = (uint32_t)__builtin_ctzll(m);
                m &= m - 1ull;
                const uint32_t a = shfl(r0, j), b = shfl(r1, j);
                const uint32_t vj = shfl(v, j), dj = shfl(d, j);
                const uint64_t kj = ((uint64_t)dj << 32) | (uint32_t)~vj;
                bool beaten = false;
                for (uint32_t e = a + l; e < b; e += 64) {
                    const uint32_t u = (uint32_t)col[e];
                    const uint32_t du = gdeg[u];
                    if (du && (((uint64_t)du << 32) | (uint32_t)~u) > kj) beaten = true;
                }
                const bool any = ballot(beaten) != 0ull;
                if (l == j) top = !any;
            }
            if (top) sel[v] = 1;
        }
        if (live) atomicAdd(&sh_live, live);
        __syncthreads();
        if (sh_live == 0) break;
        // apply: the selected vertices form an independent set
        uint32_t taken = 0;
        for (uint32_t v = wave; v < n; v += waves) {
            if (!sel[v]) continue;
            const uint32_t r1 = off[v + 1];
            for (uint32_t e = off[v] + l; e < r1; e += 64) {
                const uint32_t u = (uint32_t)col[e];
                if (gdeg[u]) atomicSub(&gdeg[u], 1u);
            }
            if (l == 0) {
                sel[v] = 0;
                gin[v] = 1;
                gdeg[v] = 0;
                ++taken;
            }
        }
        if (taken) atomicAdd(&sh_taken, taken);
        __syncthreads();
        total += sh_taken;
    }
    if (tid == 0) ctr[CTR_GSIZE] += total;
}

// ------------------------------------------------------------- scan
// Exclusive prefix sum, three passes: per-block totals, one block scans the
// totals, per-block scan plus its offset.  2048 items per 256-thread block.

constexpr uint32_t SCAN_T = 256, SCAN_PER = 8, SCAN_ITEMS = SCAN_T * SCAN_PER;
static_assert(sizeof(uint32_t) * (SCAN_T / 64u) <= SIDE_LDS_MAX, "scan partial sums");

template <typename T>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* sh, uint32_t* total) {
    const uint32_t w = threadIdx.x >> 6, l = threadIdx.x & 63u;
    uint32_t incl = wave_incl_scan(x);
    if (l == 63) sh[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t i = 0; i < SCAN_T / 64; ++i) {
        if (i < w) pre += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return pre + incl - x;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scan_totals(const T* in, uint32_t N, uint32_t* sums) {
    __shared__ uint32_t sh[SCAN_T / 64];
    const uint32_t base = blockIdx.x * SCAN_ITEMS + threadIdx.x * SCAN_PER;
    uint32_t x = 0;
    for (uint32_t j = 0; j < SCAN_PER; ++j)
        if (base + j < N) x += (uint32_t)in[base + j];
    uint32_t tot;
    block_excl_scan<T>(x, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_sums(uint32_t* sums, uint32_t nb) {
    __shared__ uint32_t sh[SCAN_T / 64];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += SCAN_T) {
        uint32_t i = base + threadIdx.x;
        uint32_t x = i < nb ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan<uint32_t>(x, sh, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scan_apply(const T* in, uint32_t N, const uint32_t* sums, uint32_t* out,
                             uint32_t nb) {
    __shared__ uint32_t sh[SCAN_T / 64];
    const uint32_t base = blockIdx.x * SCAN_ITEMS + threadIdx.x * SCAN_PER;
    uint32_t v[SCAN_PER];
    uint32_t x = 0;
    for (uint32_t j = 0; j < SCAN_PER; ++j) {
        v[j] = base + j < N ? (uint32_t)in[base + j] : 0u;
        x += v[j];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<T>(x, sh, &tot) + sums[blockIdx.x];
    for (uint32_t j = 0; j < SCAN_PER; ++j) {
        if (base + j < N) out[base + j] = ex;
        ex += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[N] = sums[nb];
}

// ------------------------------------------------------------- induce

__global__ void __launch_bounds__(256) k_live_flags(uint32_t n, const uint32_t* rdeg, uint32_t* flag, int keep_all) {
    GRID_LOOP(v, n) flag[v] = (keep_all || rlive(rdeg[v])) ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_induce_deg(uint32_t n, const uint32_t* rdeg, const uint32_t* newid,
                             uint32_t* kdeg, uint32_t* oldid, uint32_t* ctr, int keep_all) {
    uint32_t mx = 0;
    GRID_LOOP(v, n) {
        uint32_t d = rdeg[v];
        if (!rlive(d)) {
            if (!keep_all) continue;
            d = 0;
        }
        const uint32_t i = newid[v];
        kdeg[i] = d;
        oldid[i] = v;
        mx = d > mx ? d : mx;
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63u) == 0 && mx) atomicMax(&ctr[CTR_MAXDEG], mx);
}

template <typename C, typename CO>
__global__ void __launch_bounds__(256) k_induce_cols(uint32_t np, const uint32_t* off, const C* col,
                              const uint32_t* rdeg, const uint32_t* newid,
                              const uint32_t* oldid, const uint32_t* koff, CO* kcol) {
    // 64 consecutive new vertices per wave, one per lane; a row longer than
    // 32 entries is compacted by the whole wave (ballot + mbcnt keep order)
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t base = wave * 64u; base < np; base += waves * 64u) {
        const uint32_t i = base + l;
        uint32_t r0 = 0, r1 = 0;
        if (i < np) {
            const uint32_t v = oldid[i];
            r0 = off[v];
            r1 = off[v + 1];
        }
        const bool longrow = r1 - r0 > 32u;
        if (i < np && !longrow) {
            uint32_t pos = koff[i];
            const uint32_t end = koff[i + 1];
            for (uint32_t e = r0; e < r1 && pos < end; ++e) {
                const uint32_t u = (uint32_t)col[e];
                if (rlive(rdeg[u])) kcol[pos++] = (CO)newid[u];
            }
        }
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t a = shfl(r0, j), b = shfl(r1, j);
            uint32_t pos = koff[base + j];
            const uint32_t end = koff[base + j + 1];
            for (uint32_t c = a; c < b; c += 64u) {
                const uint32_t e = c + l;
                uint32_t u = 0;
                bool keep = false;
                if (e < b) {
                    u = (uint32_t)col[e];
                    keep = rlive(rdeg[u]);
                }
                const uint64_t km = ballot(keep);
                const uint32_t at = pos + mbcnt(km);
                if (keep && at < end) kcol[at] = (CO)newid[u];
                pos += (uint32_t)__builtin_popcountll(km);
            }
        }
    }
}

// ------------------------------------------------------------- cover

// flags[v] = 1 for the final cover: root-forced vertices plus the kernel
// cover (mapped back) when the search improved on the greedy bound, else the
// greedy cover itself.
__global__ void __launch_bounds__(256) k_cover_base(uint32_t n, const uint32_t* rdeg, const uint8_t* gin,
                             int improved, uint32_t* flags) {
    GRID_LOOP(v, n) flags[v] = improved ? (rdeg[v] == RIN ? 1u : 0u) : (uint32_t)gin[v];
}

__global__ void __launch_bounds__(256) k_cover_kernel(uint32_t np, const uint32_t* oldid, const uint32_t* bitmap,
                               uint32_t* flags) {
    GRID_LOOP(i, np) {
        if ((bitmap[i >> 5] >> (i & 31u)) & 1u) flags[oldid[i]] = 1u;
    }
}

__global__ void __launch_bounds__(256) k_cover_list(uint32_t n, const uint32_t* flags, const uint32_t* pos,
                             uint32_t* out) {
    GRID_LOOP(v, n) {
        if (flags[v]) out[pos[v]] = v;
    }
}

// ============================================================ launchers

static inline uint32_t grid_for(uint64_t n, uint32_t t = 256) {
    uint64_t b = (n + t - 1) / t;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (uint32_t)b;
}

// blocks of 256 threads for one wave per vertex
static inline uint32_t grid_for_waves(uint64_t n) {
    uint64_t b = (n + 3) / 4;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (uint32_t)b;
}

hipError_t root_validate(const RootGraph& g, uint32_t* ctr, unsigned long long* hsum,
                         hipStream_t st, uint32_t* hm, uint32_t* bad_host, int* sorted_host) {
    hipError_t e;
    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, g.nnz,
                       g.off, ctr);
    if ((e = hipGetLastError())) return e;
    uint32_t bad = 0;
    // (the row check returns at once when the offsets were bad)
    if (g.col_bytes == 2)
        hipLaunchKernelGGL(k_check_rows<uint16_t>, dim3(grid_for(g.n)), dim3(256), 0, st, g.n,
                           g.off, (const uint16_t*)g.col, ctr, hsum);
    else
        hipLaunchKernelGGL(k_check_rows<uint32_t>, dim3(grid_for(g.n)), dim3(256), 0, st, g.n,
                           g.off, (const uint32_t*)g.col, ctr, hsum);
    hipLaunchKernelGGL(k_hsum_fold, dim3(1), dim3(64), 0, st, hsum);
    if ((e = hipGetLastError())) return e;
    if ((e = hipMemcpyAsync(&hm[0], ctr + CTR_INVALID, 4, hipMemcpyDeviceToHost, st))) return e;
    if ((e = hipMemcpyAsync(&hm[1], ctr + CTR_UNSORTED, 4, hipMemcpyDeviceToHost, st))) return e;
    if ((e = hipMemcpyAsync(&hm[2], hsum, 8, hipMemcpyDeviceToHost, st))) return e;
    if ((e = hipStreamSynchronize(st))) return e;
    bad = hm[0];
    const uint32_t uns = hm[1];
    if (hm[2] != 0u || hm[3] != 0u) bad |= 64u;
    *bad_host = bad;
    if (sorted_host) *sorted_host = !bad && uns == 0;
    return hipSuccess;
}

hipError_t root_init(const RootGraph& g, const RootBufs& b, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, g.off, b.rdeg, b.gdeg,
                       b.gin, b.addf, b.newly);
    return hipGetLastError();
}

template <typename C>
static hipError_t greedy_t(const RootGraph& g, const RootBufs& b, hipStream_t st,
                           uint32_t* rounds) {
    const C* col = (const C*)g.col;
    hipError_t e;
    if (g.n <= SMALL_N) {
        hipLaunchKernelGGL(k_greedy_small<C>, dim3(1), dim3(SMALL_T), 0, st, g.n, g.off, col,
                           b.gdeg, b.addf, b.gin, b.ctr);
        *rounds = 0;
        return hipGetLastError();
    }
    const uint32_t wgrid = grid_for_waves(g.n);
    for (uint32_t r = 0;; r += 4) {
        for (uint32_t j = 0; j < 4; ++j) {
            uint32_t* live = b.ctr + CTR_GLIVE + ((r + j) & 1u);
            if ((e = hipMemsetAsync(live, 0, 4, st))) return e;
            hipLaunchKernelGGL(k_greedy_select<C>, dim3(wgrid), dim3(256), 0, st, g.n, g.off, col,
                               b.gdeg, b.addf, live);
            hipLaunchKernelGGL(k_greedy_apply<C>, dim3(wgrid), dim3(256), 0, st, g.n, g.off, col,
                               b.gdeg, b.addf, b.gin, live, b.ctr + CTR_GSIZE);
        }
        if ((e = hipGetLastError())) return e;
        if ((e = hipMemcpyAsync(&b.hm[4], b.ctr + CTR_GLIVE + ((r + 3) & 1u), 4,
                                hipMemcpyDeviceToHost, st)))
            return e;
        if ((e = hipStreamSynchronize(st))) return e;
        const uint32_t live = b.hm[4];
        if (live == 0 || r > 4 * g.n + 8) {
            *rounds = r + 4;
            return hipSuccess;
        }
    }
}

hipError_t root_greedy_rest(const RootGraph& g, const RootBufs& b, hipStream_t st) {
    hipLaunchKernelGGL(k_greedy_rest, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, b.rdeg, b.gdeg,
                       b.gin);
    return hipGetLastError();
}

hipError_t root_greedy(const RootGraph& g, const RootBufs& b, hipStream_t st, uint32_t* rounds) {
    return g.col_bytes == 2 ? greedy_t<uint16_t>(g, b, st, rounds)
                            : greedy_t<uint32_t>(g, b, st, rounds);
}

template <typename C>
static hipError_t reduce_t(const RootGraph& g, const RootBufs& b, int best0, hipStream_t st,
                           uint32_t max_rounds, uint32_t* rounds) {
    const C* col = (const C*)g.col;
    hipError_t e;
    if (g.n <= SMALL_N) {
        // (rounds are counted in ctr[CTR_ROUNDS])
        hipLaunchKernelGGL(k_reduce_small<C>, dim3(1), dim3(SMALL_T), 0, st, g.n, g.off, col,
                           b.rdeg, b.addf, b.newly, b.ctr, best0, g.sorted, max_rounds);
        *rounds = 0;
        return hipGetLastError();
    }
    // decide and mark end with one atomic per block on a single counter:
    // at most 1024 blocks, so a round where most blocks fire does not
    // serialise thousands of them
    const uint32_t grid = std::min<uint32_t>(grid_for(g.n), 1024u);
    uint32_t r = 0;
    for (;;) {
        // eight rounds per host check: rounds after the fixpoint return at
        // once on the device
        for (uint32_t j = 0; j < 8; ++j, ++r) {
            hipLaunchKernelGGL(k_reduce_decide<C>, dim3(grid), dim3(256), 0, st, g.n, g.off, col,
                               b.rdeg, b.addf, b.ctr, r, best0, g.sorted);
            hipLaunchKernelGGL(k_reduce_mark, dim3(grid), dim3(256), 0, st, g.n, b.rdeg, b.addf,
                               b.newly, b.ctr, r);
            hipLaunchKernelGGL(k_reduce_remove<C>, dim3(grid), dim3(256), 0, st, g.n, g.off, col,
                               b.rdeg, b.newly, b.ctr, r);
        }
        if ((e = hipGetLastError())) return e;
        if ((e = hipMemcpyAsync(&b.hm[5], b.ctr + CTR_FIRED + ((r - 1) & 1u), 4,
                                hipMemcpyDeviceToHost, st)))
            return e;
        if ((e = hipStreamSynchronize(st))) return e;
        const uint32_t fired = b.hm[5];
        if (fired == 0 || r >= max_rounds) break;
    }
    *rounds = r;
    return hipSuccess;
}

hipError_t root_reduce(const RootGraph& g, const RootBufs& b, int best0, hipStream_t st,
                       uint32_t max_rounds, uint32_t* rounds) {
    return g.col_bytes == 2 ? reduce_t<uint16_t>(g, b, best0, st, max_rounds, rounds)
                            : reduce_t<uint32_t>(g, b, best0, st, max_rounds, rounds);
}

hipError_t scan_u32(const uint32_t* in, uint32_t N, uint32_t* out, uint32_t* tmp,
                    hipStream_t st) {
    const uint32_t nb = (N + SCAN_ITEMS - 1) / SCAN_ITEMS ? (N + SCAN_ITEMS - 1) / SCAN_ITEMS : 1;
    hipLaunchKernelGGL(k_scan_totals<uint32_t>, dim3(nb), dim3(SCAN_T), 0, st, in, N, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply<uint32_t>, dim3(nb), dim3(SCAN_T), 0, st, in, N, tmp, out, nb);
    return hipGetLastError();
}

hipError_t root_induce_a(const RootGraph& g, const RootBufs& b, hipStream_t st, bool keep_all) {
    hipLaunchKernelGGL(k_live_flags, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, b.rdeg, b.flags,
                       (int)keep_all);
    hipError_t e = scan_u32(b.flags, g.n, b.newid, b.scan_tmp, st);
    if (e) return e;
    hipLaunchKernelGGL(k_induce_deg, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, b.rdeg, b.newid,
                       b.kdeg, b.oldid, b.ctr, (int)keep_all);
    return hipGetLastError();
}

hipError_t root_induce_b(const RootGraph& g, const RootBufs& b, uint32_t np, uint32_t kcol_bytes,
                         hipStream_t st) {
    hipError_t e = scan_u32(b.kdeg, np, b.koff, b.scan_tmp, st);
    if (e) return e;
    const uint32_t grid = grid_for(np);
    if (g.col_bytes == 2) {
        if (kcol_bytes == 2)
            hipLaunchKernelGGL((k_induce_cols<uint16_t, uint16_t>), dim3(grid), dim3(256), 0, st,
                               np, g.off, (const uint16_t*)g.col, b.rdeg, b.newid, b.oldid, b.koff,
                               (uint16_t*)b.kcol);
        else
            hipLaunchKernelGGL((k_induce_cols<uint16_t, uint32_t>), dim3(grid), dim3(256), 0, st,
                               np, g.off, (const uint16_t*)g.col, b.rdeg, b.newid, b.oldid, b.koff,
                               (uint32_t*)b.kcol);
    } else {
        if (kcol_bytes == 2)
            hipLaunchKernelGGL((k_induce_cols<uint32_t, uint16_t>), dim3(grid), dim3(256), 0, st,
                               np, g.off, (const uint32_t*)g.col, b.rdeg, b.newid, b.oldid, b.koff,
                               (uint16_t*)b.kcol);
        else
            hipLaunchKernelGGL((k_induce_cols<uint32_t, uint32_t>), dim3(grid), dim3(256), 0, st,
                               np, g.off, (const uint32_t*)g.col, b.rdeg, b.newid, b.oldid, b.koff,
                               (uint32_t*)b.kcol);
    }
    return hipGetLastError();
}

hipError_t root_cover(const RootGraph& g, const RootBufs& b, uint32_t np, int improved,
                      const uint32_t* root_bitmap, hipStream_t st) {
    hipLaunchKernelGGL(k_cover_base, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, b.rdeg, b.gin,
                       improved, b.flags);
    if (improved && np)
        hipLaunchKernelGGL(k_cover_kernel, dim3(grid_for(np)), dim3(256), 0, st, np, b.oldid,
                           root_bitmap, b.flags);
    hipError_t e = scan_u32(b.flags, g.n, b.newid, b.scan_tmp, st);
    if (e) return e;
    hipLaunchKernelGGL(k_cover_list, dim3(grid_for(g.n)), dim3(256), 0, st, g.n, b.flags, b.newid,
                       b.cover);
    return hipGetLastError();
}

}  // namespace vc
