// Crown reduction at the root (Sec. IV-B names it among the root rules; the
// construction is the classic one of Chor, Fellows and Juedes / Abu-Khzam et
// al.): a maximal matching M1; O = the vertices M1 leaves unmatched (an
// independent set, M1 being maximal); a maximum matching M2 between O and
// N(O); if M2 leaves some of O unmatched, the alternating closure from those
// vertices gives I (in O) and H = N(I), which M2 matches into I.  Some
// minimum cover contains H and avoids I, so H goes into the cover and I is
// removed: MVC(G) = |H| + MVC(G - H - I).
//
// On the GPU: M1 by rounds of mutual proposals (each vertex proposes to its
// unmatched neighbour of least hashed key; at least the globally least key
// with an unmatched neighbour pairs up every round).  M2 by phases of a
// level-synchronous BFS over alternating paths from every M2-free vertex of
// O at once: a vertex of N(O) is claimed once (its BFS parent), a matched
// one hands the search to its partner, and a free one ends an augmenting
// path, one per BFS root.  Those paths are vertex-disjoint and are flipped
// in parallel.  A phase that finds no path proves M2 maximum, and what it
// visited is the crown: H = the claimed vertices of N(O), I = the free
// vertices of O plus the partners of H.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_common.hpp"
#include "internal.hpp"
#include "root.hpp"

namespace vc {

namespace {

constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint32_t RIN32 = 0xFFFFFFFFu;  // root degree array: in the cover

__device__ __forceinline__ bool c_live(uint32_t d) { return d != 0u && d != RIN32; }

__device__ __forceinline__ uint64_t mm_key(uint32_t u) {
    uint32_t h = u;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return ((uint64_t)h << 32) | u;  // distinct for distinct u
}

#define C_GRID_LOOP(i, n) \
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

// append `val` to list[] where pred holds (one atomic per wave)
__device__ __forceinline__ void wave_push(bool pred, uint32_t val, uint32_t* list,
                                          uint32_t* count) {
    const uint64_t m = ballot(pred);
    if (!m) return;
    const uint32_t leader = (uint32_t)__builtin_ctzll(m);
    uint32_t base = 0;
    if ((threadIdx.x & 63u) == leader) base = atomicAdd(count, (uint32_t)__builtin_popcountll(m));
    base = shfl(base, leader);
    if (pred) list[base + mbcnt(m)] = val;
}

__global__ void k_mm_init(uint32_t n, uint32_t* mate, uint32_t* prop) {
    C_GRID_LOOP(v, n) {
        mate[v] = NONE32;
        prop[v] = NONE32;
    }
}

// prop[v] = the unmatched live neighbour of least key (rows longer than 32
// entries are scanned by the whole wave)
template <typename C>
__global__ void k_mm_propose(uint32_t n, const uint32_t* off, const C* col, const uint32_t* rdeg,
                             const uint32_t* mate, uint32_t* prop) {
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t base = wave * 64u; base < n; base += waves * 64u) {
        const uint32_t v = base + l;
        const bool act = v < n && c_live(rdeg[v]) && mate[v] == NONE32;
        const uint32_t r0 = act ? off[v] : 0u, r1 = act ? off[v + 1] : 0u;
        const bool longrow = r1 - r0 > 32u;
        if (act && !longrow) {
            uint64_t best = ~0ull;
            for (uint32_t e = r0; e < r1; ++e) {
                const uint32_t u = (uint32_t)col[e];
                if (c_live(rdeg[u]) && mate[u] == NONE32) {
                    const uint64_t k = mm_key(u);
                    best = k < best ? k : best;
                }
            }
            prop[v] = best == ~0ull ? NONE32 : (uint32_t)best;
        }
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t a = shfl(r0, j), b = shfl(r1, j);
            uint64_t best = ~0ull;
            for (uint32_t e = a + l; e < b; e += 64u) {
                const uint32_t u = (uint32_t)col[e];
                if (c_live(rdeg[u]) && mate[u] == NONE32) {
                    const uint64_t k = mm_key(u);
                    best = k < best ? k : best;
                }
            }
            best = ~wave_max64(~best);
            if (l == 0) prop[base + j] = best == ~0ull ? NONE32 : (uint32_t)best;
        }
    }
}

// mutual proposals become matched pairs; *matched counts matched vertices
__global__ void k_mm_accept(uint32_t n, const uint32_t* rdeg, uint32_t* mate, const uint32_t* prop,
                            uint32_t* matched) {
    uint32_t cnt = 0;
    C_GRID_LOOP(v, n) {
        if (!c_live(rdeg[v]) || mate[v] != NONE32) continue;
        const uint32_t u = prop[v];
        if (u != NONE32 && prop[u] == v) {
            mate[v] = u;
            ++cnt;
        }
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63u) == 0 && cnt) atomicAdd(matched, cnt);
}

// start of a phase: clear the BFS marks; the M2-free vertices of O are the
// roots of the first frontier
__global__ void k_cr_phase_init(uint32_t n, const uint32_t* rdeg, const uint32_t* mate1,
                                const uint32_t* mate2, uint32_t* parent, uint32_t* rootof,
                                uint32_t* rootdone, uint32_t* front, uint32_t* count) {
    const uint32_t stride = gridDim.x * blockDim.x;
    // whole waves run the loop (wave_push needs every lane)
    for (uint32_t base = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u; base < n; base += stride) {
        const uint32_t v = base + (threadIdx.x & 63u);
        bool root = false;
        if (v < n) {
            parent[v] = NONE32;
            rootdone[v] = 0u;
            root = c_live(rdeg[v]) && mate1[v] == NONE32 && mate2[v] == NONE32;
            if (root) rootof[v] = v;
        }
        wave_push(root, v, front, count);
    }
}

// One BFS level.  cnt[lvl % 3] holds the size of `in`; the next frontier
// goes to `out` and cnt[(lvl + 1) % 3]; cnt[(lvl + 2) % 3] is cleared for the
// level after.  An M2-free vertex reached ends a path (one per root).
template <typename C>
__global__ void k_cr_level(const uint32_t* off, const C* col, const uint32_t* rdeg,
                           const uint32_t* mate2, uint32_t* parent, uint32_t* rootof,
                           uint32_t* rootdone, const uint32_t* in, uint32_t* out, uint32_t* cnt,
                           uint32_t lvl, uint32_t* ends, uint32_t* nends) {
    const uint32_t nin = cnt[lvl % 3u];
    uint32_t* nout = &cnt[(lvl + 1u) % 3u];
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(lvl + 2u) % 3u] = 0u;
    C_GRID_LOOP(i, nin) {
        const uint32_t x = in[i];
        const uint32_t r = rootof[x];
        if (__hip_atomic_load(&rootdone[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
        for (uint32_t e = off[x]; e < off[x + 1]; ++e) {
            const uint32_t y = (uint32_t)col[e];
            if (!c_live(rdeg[y])) continue;
            if (atomicCAS(&parent[y], NONE32, x) != NONE32) continue;
            const uint32_t m = mate2[y];
            if (m == NONE32) {
                if (atomicCAS(&rootdone[r], 0u, 1u) == 0u) ends[atomicAdd(nends, 1u)] = y;
                break;
            }
            rootof[m] = r;
            out[atomicAdd(nout, 1u)] = m;
        }
    }
}

// flip every found augmenting path (vertex-disjoint: one per BFS root)
__global__ void k_cr_augment(uint32_t n, const uint32_t* ends, const uint32_t* nends,
                             const uint32_t* parent, uint32_t* mate2) {
    C_GRID_LOOP(i, *nends) {
        uint32_t y = ends[i];
        for (uint32_t step = 0; step < n; ++step) {
            const uint32_t x = parent[y];
            const uint32_t ny = mate2[x];
            mate2[y] = x;
            mate2[x] = y;
            if (ny == NONE32) break;
            y = ny;
        }
    }
}

// The last phase found no path: its visited vertices of N(O) are H (into
// the cover), their partners and the M2-free vertices of O are I (removed).
__global__ void k_cr_apply(uint32_t n, uint32_t* rdeg, const uint32_t* mate1,
                           const uint32_t* mate2, const uint32_t* parent, uint8_t* newly,
                           uint32_t* ctr) {
    uint32_t h = 0, i = 0;
    C_GRID_LOOP(v, n) {
        if (parent[v] != NONE32) {
            rdeg[v] = RIN32;
            newly[v] = 1;
            ++h;
            const uint32_t m = mate2[v];  // matched: the phase found no path
            if (m != NONE32) {
                rdeg[m] = 0u;
                ++i;
            }
        } else if (c_live(rdeg[v]) && mate1[v] == NONE32 && mate2[v] == NONE32) {
            rdeg[v] = 0u;
            ++i;
        }
    }
    h = wave_sum(h);
    i = wave_sum(i);
    if ((threadIdx.x & 63u) == 0) {
        if (h) {
            atomicAdd(&ctr[CTR_SROOT], h);
            atomicAdd(&ctr[CTR_CROWN_H], h);
        }
        if (i) atomicAdd(&ctr[CTR_CROWN_I], i);
    }
}

template <typename C>
__global__ void k_cr_remove(uint32_t n, const uint32_t* off, const C* col, uint32_t* rdeg,
                            uint8_t* newly) {
    const uint32_t l = threadIdx.x & 63u;
    for (uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < n;
         v += (gridDim.x * blockDim.x) >> 6) {
        if (!newly[v]) continue;
        for (uint32_t e = off[v] + l; e < off[v + 1]; e += 64u) {
            const uint32_t u = (uint32_t)col[e];
            if (c_live(rdeg[u])) atomicSub(&rdeg[u], 1u);
        }
        if (l == 0) newly[v] = 0;
    }
}

inline uint32_t c_grid(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (uint32_t)b;
}

template <typename C>
hipError_t crown_t(const RootGraph& g, const RootBufs& b, hipStream_t st, uint32_t* h_out) {
    *h_out = 0;
    const uint32_t n = g.n;
    const C* col = (const C*)g.col;
    uint32_t* mate1 = b.cw;
    uint32_t* mate2 = b.cw + (size_t)n;  // the proposals while M1 is built
    uint32_t* parent = b.cw + 2ull * n;
    uint32_t* rootof = b.cw + 3ull * n;
    uint32_t* rootdone = b.cw + 4ull * n;
    uint32_t* front[2] = {b.cw + 5ull * n, b.cw + 6ull * n};
    uint32_t* ends = b.cw + 7ull * n;
    uint32_t* cnt = b.ctr + CTR_CROWN_F;  // 3 rotating frontier counts
    uint32_t* nends = b.ctr + CTR_CROWN_E;
    uint32_t* matched = b.ctr + CTR_CROWN_M;
    const uint32_t grid = c_grid(n);
    const uint32_t wgrid = c_grid(64ull * n);  // one wave per vertex
    hipError_t e;
    uint32_t* host = b.hm + 8;  // pinned read-back words

    // ---- M1: maximal matching by mutual proposals
    hipLaunchKernelGGL(k_mm_init, dim3(grid), dim3(256), 0, st, n, mate1, mate2);
    for (uint32_t round = 0;; round += 4) {
        if ((e = hipMemsetAsync(matched, 0, 4, st))) return e;
        for (uint32_t j = 0; j < 4; ++j) {
            hipLaunchKernelGGL(k_mm_propose<C>, dim3(grid), dim3(256), 0, st, n, g.off, col, b.rdeg,
                               mate1, mate2);
            hipLaunchKernelGGL(k_mm_accept, dim3(grid), dim3(256), 0, st, n, b.rdeg, mate1, mate2,
                               matched);
        }
        if ((e = hipGetLastError())) return e;
        if ((e = hipMemcpyAsync(&host[0], matched, 4, hipMemcpyDeviceToHost, st))) return e;
        if ((e = hipStreamSynchronize(st))) return e;
        if (host[0] == 0) break;  // four rounds without a new pair: maximal
        if (round > n) return hipErrorUnknown;  // at least one pair per round
    }

    // ---- M2: maximum matching between O and N(O), phase by phase
    hipLaunchKernelGGL(k_mm_init, dim3(grid), dim3(256), 0, st, n, mate2, ends);
    for (uint32_t phase = 0;; ++phase) {
        if (phase > n) return hipErrorUnknown;  // each phase grows M2
        if ((e = hipMemsetAsync(cnt, 0, 5 * 4, st))) return e;  // counts, ends, matched
        hipLaunchKernelGGL(k_cr_phase_init, dim3(grid), dim3(256), 0, st, n, b.rdeg, mate1, mate2,
                           parent, rootof, rootdone, front[0], &cnt[0]);
        if ((e = hipMemcpyAsync(&host[0], &cnt[0], 4, hipMemcpyDeviceToHost, st))) return e;
        if ((e = hipStreamSynchronize(st))) return e;
        if (host[0] == 0) return hipGetLastError();  // M2 covers O: no crown
        // BFS levels, four per look at the frontier size (an empty frontier
        // makes the remaining levels of the four no-ops)
        uint32_t lvl = 0;
        for (;;) {
            for (uint32_t j = 0; j < 4; ++j, ++lvl)
                hipLaunchKernelGGL(k_cr_level<C>, dim3(grid), dim3(256), 0, st, g.off, col, b.rdeg,
                                   mate2, parent, rootof, rootdone, front[lvl & 1u],
                                   front[(lvl + 1u) & 1u], cnt, lvl, ends, nends);
            if ((e = hipGetLastError())) return e;
            if ((e = hipMemcpyAsync(&host[0], &cnt[lvl % 3u], 4, hipMemcpyDeviceToHost, st)))
                return e;
            if ((e = hipMemcpyAsync(&host[1], nends, 4, hipMemcpyDeviceToHost, st))) return e;
            if ((e = hipStreamSynchronize(st))) return e;
            if (host[0] == 0) break;
            if (lvl > 2u * n + 8u) return hipErrorUnknown;  // every vertex enters once
        }
        if (host[1] == 0) break;  // no augmenting path: M2 is maximum
        hipLaunchKernelGGL(k_cr_augment, dim3(c_grid(host[1])), dim3(256), 0, st, n, ends, nends,
                           parent, mate2);
    }

    // ---- the last phase's search is the crown
    if ((e = hipMemsetAsync(b.ctr + CTR_CROWN_H, 0, 4, st))) return e;
    hipLaunchKernelGGL(k_cr_apply, dim3(grid), dim3(256), 0, st, n, b.rdeg, mate1, mate2, parent,
                       b.newly, b.ctr);
    hipLaunchKernelGGL(k_cr_remove<C>, dim3(wgrid), dim3(256), 0, st, n, g.off, col, b.rdeg,
                       b.newly);
    if ((e = hipGetLastError())) return e;
    if ((e = hipMemcpyAsync(&host[2], b.ctr + CTR_CROWN_H, 4, hipMemcpyDeviceToHost, st)))
        return e;
    if ((e = hipStreamSynchronize(st))) return e;
    *h_out = host[2];
    return hipSuccess;
}

}  // namespace

hipError_t root_crown(const RootGraph& g, const RootBufs& b, hipStream_t st, uint32_t* h_out) {
    return g.col_bytes == 2 ? crown_t<uint16_t>(g, b, st, h_out)
                            : crown_t<uint32_t>(g, b, st, h_out);
}

}  // namespace vc
