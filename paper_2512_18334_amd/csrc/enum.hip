// Enumeration of the minimal vertex covers of size <= k: the PVC variant
// that Sec. III-E describes (enumerate per component, then combine the
// components' covers whose sizes fit) and the paper leaves unbuilt.  All
// covers of size <= k are the supersets of these.
//
// Steps, all on the device:
//   1. connected components by min-label propagation with pointer jumping;
//      component ids by a scan of the roots; a local id (0..63) per vertex;
//   2. per component, one wave: adjacency masks, a greedy matching (a lower
//      bound lb_c on its cover size); the component's budget is
//      k - sum of the other components' lb (a cover of the whole graph within
//      k leaves no more room than that);
//   3. per component, one wave enumerates its minimal covers within the
//      budget (twice: counting by size, then writing the masks): branch on
//      the lowest vertex u with an uncovered edge, u in the cover, or u out
//      for good and N(u) in (dropped if N(u) meets a vertex kept out); keep
//      a leaf when every cover vertex has a neighbour outside;
//   4. ways[c][b] = number of ways to pick one cover from each of components
//      c.. with total size <= b (saturating); the count is ways[0][k];
//   5. cover t of the combined list is unranked component by component.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "ctx.hpp"
#include "dev_common.hpp"
#include "internal.hpp"
#include "root.hpp"
#include "vc.h"

namespace vc {

namespace {

constexpr uint32_t EN_NONE = 0xFFFFFFFFu;
constexpr uint32_t EN_MAXC = 64;                 // vertices per component
constexpr uint64_t EN_LIST_MAX = 1ull << 26;     // component covers kept
constexpr uint64_t EN_WAYS_MAX = 1ull << 26;     // (components + 1) x (k + 1)
constexpr uint64_t EN_SAT = ~0ull;

#define EN_GRID_LOOP(i, n) \
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

__device__ __forceinline__ uint64_t rl64(uint64_t x, uint32_t j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)j);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (a == 0 || b == 0) return 0;
    return b > EN_SAT / a ? EN_SAT : a * b;
}
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
    return a > EN_SAT - b ? EN_SAT : a + b;
}

// ---------------------------------------------------------------- labels

__global__ void k_en_label_init(uint32_t n, const uint32_t* off, uint32_t* label) {
    EN_GRID_LOOP(v, n) label[v] = off[v + 1] > off[v] ? v : EN_NONE;
}

template <typename C>
__global__ void k_en_label_prop(uint32_t n, const uint32_t* off, const C* col, uint32_t* label,
                                uint32_t* changed) {
    uint32_t ch = 0;
    EN_GRID_LOOP(v, n) {
        const uint32_t lv = label[v];
        if (lv == EN_NONE) continue;
        uint32_t m = lv;
        for (uint32_t e = off[v]; e < off[v + 1]; ++e) {
            const uint32_t lu = label[(uint32_t)col[e]];
            m = lu < m ? lu : m;
        }
        m = label[m] < m ? label[m] : m;  // pointer jumping
        if (m < lv) {
            atomicMin(&label[v], m);
            ++ch;
        }
    }
    ch = wave_sum(ch);
    if ((threadIdx.x & 63u) == 0 && ch) atomicAdd(changed, ch);
}

__global__ void k_en_roots(uint32_t n, const uint32_t* label, uint32_t* flag) {
    EN_GRID_LOOP(v, n) flag[v] = label[v] == v ? 1u : 0u;
}

// local id of every vertex in its component; size of every component
__global__ void k_en_local(uint32_t n, const uint32_t* label, const uint32_t* rank,
                           uint32_t* loc, uint32_t* csize, uint32_t* maxsize) {
    uint32_t mx = 0;
    EN_GRID_LOOP(v, n) {
        const uint32_t lv = label[v];
        if (lv == EN_NONE) continue;
        const uint32_t c = rank[lv];
        const uint32_t i = atomicAdd(&csize[c], 1u);
        loc[v] = i;
        mx = i + 1u > mx ? i + 1u : mx;
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63u) == 0 && mx) atomicMax(maxsize, mx);
}

__global__ void k_en_place(uint32_t n, const uint32_t* label, const uint32_t* rank,
                           const uint32_t* loc, const uint32_t* coff, uint32_t* verts) {
    EN_GRID_LOOP(v, n) {
        const uint32_t lv = label[v];
        if (lv == EN_NONE) continue;
        verts[coff[rank[lv]] + loc[v]] = v;
    }
}

// ------------------------------------------------------------ per component

// lane i < nc: local vertex i's adjacency mask
template <typename C>
__device__ __forceinline__ uint64_t en_adj(const uint32_t* off, const C* col, const uint32_t* loc,
                                           const uint32_t* verts, uint32_t base, uint32_t nc) {
    const uint32_t l = threadIdx.x & 63u;
    uint64_t a = 0;
    if (l < nc) {
        const uint32_t v = verts[base + l];
        for (uint32_t e = off[v]; e < off[v + 1]; ++e) a |= 1ull << loc[(uint32_t)col[e]];
    }
    return a;
}

// greedy maximal matching size: a lower bound on the component's cover
template <typename C>
__global__ void __launch_bounds__(64) k_en_lb(uint32_t ncomp, const uint32_t* off, const C* col,
                                              const uint32_t* loc, const uint32_t* verts,
                                              const uint32_t* coff, uint32_t* lb, uint32_t* lbsum) {
    for (uint32_t c = blockIdx.x; c < ncomp; c += gridDim.x) {
        const uint32_t base = coff[c], nc = coff[c + 1] - base;
        const uint64_t adj = en_adj(off, col, loc, verts, base, nc);
        uint64_t matched = 0;
        uint32_t m = 0;
        for (uint32_t i = 0; i < nc; ++i) {
            if ((matched >> i) & 1ull) continue;
            const uint64_t a = rl64(adj, i) & ~matched;
            if (a) {
                matched |= (1ull << i) | (1ull << __builtin_ctzll(a));
                ++m;
            }
        }
        if (threadIdx.x == 0) {
            lb[c] = m;
            atomicAdd(lbsum, m);
        }
    }
}

// Enumerate the component's minimal covers within its budget, split over
// 2^L threads per component (L <= 22): thread j replays the first L branch
// decisions from the bits of j (bit d: 0 = u in, 1 = u out and N(u) in), then walks
// the subtree below with a private stack.  A path that ends above depth L
// (a leaf, a cut or a dropped branch) belongs to the one j whose remaining
// bits are zero, so nothing is counted twice.  write == 0: cnt[c * 64 + s]
// counts the covers of size s; write == 1: each cover's mask goes to
// list[loff[c] + cur[c]++].
__device__ __forceinline__ uint32_t en_first_uncovered(const uint64_t* adj, uint64_t in,
                                                       uint64_t full) {
    for (uint64_t cand = ~in & full; cand; cand &= cand - 1ull) {
        const uint32_t v = (uint32_t)__builtin_ctzll(cand);
        if (adj[v] & ~in) return v;
    }
    return EN_NONE;
}

__device__ __forceinline__ bool en_minimal(const uint64_t* adj, uint64_t in) {
    for (uint64_t x = in; x; x &= x - 1ull)
        if ((adj[__builtin_ctzll(x)] & ~in) == 0ull) return false;
    return true;
}

template <typename C>
__global__ void __launch_bounds__(256) k_en_enum(uint32_t ncomp, uint32_t L, const uint32_t* off,
                                                 const C* col, const uint32_t* loc,
                                                 const uint32_t* verts, const uint32_t* coff,
                                                 const uint32_t* lb, const uint32_t* lbsum,
                                                 int64_t k, int write, unsigned long long* cnt,
                                                 uint32_t* cur, const uint32_t* loff,
                                                 uint64_t* list, uint64_t node_limit,
                                                 uint32_t* err) {
    __shared__ uint64_t adj[EN_MAXC];
    const uint32_t per = (1u << L) > 256u ? (1u << L) / 256u : 1u;  // blocks per component
    const uint32_t c = blockIdx.x / per;
    if (c >= ncomp) return;
    const uint32_t base = coff[c], nc = coff[c + 1] - base;
    if (threadIdx.x < EN_MAXC) {
        uint64_t a = 0;
        if (threadIdx.x < nc) {
            const uint32_t v = verts[base + threadIdx.x];
            for (uint32_t e = off[v]; e < off[v + 1]; ++e) a |= 1ull << loc[(uint32_t)col[e]];
        }
        adj[threadIdx.x] = a;
    }
    __syncthreads();
    const uint32_t j = (blockIdx.x % per) * 256u + threadIdx.x;
    if (j >= (1u << L)) return;
    const int64_t budget = k - ((int64_t)*lbsum - (int64_t)lb[c]);
    if (budget < 0) return;
    const uint64_t full = nc >= 64u ? ~0ull : ((1ull << nc) - 1ull);
    auto emit = [&](uint64_t in, uint32_t size) {
        if (write) {
            const uint32_t pos = atomicAdd(&cur[c], 1u);
            list[(uint64_t)loff[c] + pos] = in;
        } else {
            atomicAdd(&cnt[(uint64_t)c * 64u + size], 1ull);
        }
    };
    uint64_t in = 0, out = 0;
    uint32_t size = 0;
    // the prefix
    for (uint32_t d = 0; d < L; ++d) {
        const uint32_t u = en_first_uncovered(adj, in, full);
        if (u == EN_NONE) {
            if ((j >> d) == 0u && en_minimal(adj, in)) emit(in, size);
            return;
        }
        if (((j >> d) & 1u) == 0u) {
            in |= 1ull << u;
            ++size;
            if ((int64_t)size > budget) return;
        } else {
            const uint64_t au = adj[u];
            if (au & out) return;
            size += (uint32_t)__builtin_popcountll(au & ~in);
            if ((int64_t)size > budget) return;
            in |= au;
            out |= 1ull << u;
        }
    }
    // the subtree below, depth first (a path holds at most nc pending
    // "u out" branches, one per vertex put in the cover on it)
    uint64_t st_in[EN_MAXC], st_out[EN_MAXC];
    uint32_t st_size[EN_MAXC];
    uint32_t sp = 0;
    uint64_t nodes = 0;
    for (;;) {
        if (node_limit && ++nodes > node_limit) {
            atomicOr(err, 1u);
            return;
        }
        const uint32_t u = en_first_uncovered(adj, in, full);
        bool pop = false;
        if (u == EN_NONE) {
            if (en_minimal(adj, in)) emit(in, size);
            pop = true;
        } else {
            const uint64_t au = adj[u];
            if ((au & out) == 0ull) {
                const uint32_t sb = size + (uint32_t)__builtin_popcountll(au & ~in);
                if ((int64_t)sb <= budget && sp < EN_MAXC) {
                    st_in[sp] = in | au;
                    st_out[sp] = out | (1ull << u);
                    st_size[sp] = sb;
                    ++sp;
                }
            }
            in |= 1ull << u;
            ++size;
            if ((int64_t)size > budget) pop = true;
        }
        if (pop) {
            if (sp == 0) return;
            --sp;
            in = st_in[sp];
            out = st_out[sp];
            size = st_size[sp];
        }
    }
}

// per component: its number of covers (the list length) and the total
__global__ void k_en_tot(uint32_t ncomp, const unsigned long long* cnt, uint32_t* tot,
                         unsigned long long* all) {
    EN_GRID_LOOP(c, ncomp) {
        unsigned long long t = 0;
        for (uint32_t s = 0; s < 64; ++s) t += cnt[(uint64_t)c * 64u + s];
        tot[c] = t > EN_LIST_MAX ? (uint32_t)(EN_LIST_MAX + 1u) : (uint32_t)t;
        atomicAdd(all, t);
    }
}

// ways[c * (k + 1) + b]: choices of one cover from each of components c..
// with total size <= b; one wave, components from the last to the first
__global__ void __launch_bounds__(64) k_en_ways(uint32_t ncomp, uint32_t k, const uint64_t* cnt,
                                                uint64_t* ways) {
    const uint32_t l = threadIdx.x;
    const uint64_t w = (uint64_t)k + 1u;
    for (uint32_t b = l; b <= k; b += 64) ways[(uint64_t)ncomp * w + b] = 1ull;
    __syncthreads();
    for (int64_t c = (int64_t)ncomp - 1; c >= 0; --c) {
        for (uint32_t b = l; b <= k; b += 64) {
            uint64_t sum = 0;
            for (uint32_t s = 0; s < 64 && s <= b; ++s) {
                const uint64_t cs = cnt[(uint64_t)c * 64u + s];
                if (cs) sum = sat_add(sum, sat_mul(cs, ways[(uint64_t)(c + 1) * w + (b - s)]));
            }
            ways[(uint64_t)c * w + b] = sum;
        }
        __syncthreads();
    }
}

// cover t of the combined list, for t < nout: ids ascending in out[t * k ..]
__global__ void k_en_unrank(uint64_t nout, uint32_t ncomp, uint32_t k, const uint64_t* ways,
                            const uint32_t* loff, const uint64_t* list, const uint32_t* coff,
                            const uint32_t* verts, uint32_t* out, uint32_t* sizes) {
    const uint64_t w = (uint64_t)k + 1u;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nout;
         t += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t r = t;
        uint32_t b = k, len = 0;
        uint32_t* o = out + t * k;
        for (uint32_t c = 0; c < ncomp; ++c) {
            for (uint32_t i = loff[c]; i < loff[c + 1]; ++i) {
                const uint64_t x = list[i];
                const uint32_t s = (uint32_t)__builtin_popcountll(x);
                if (s > b) continue;
                const uint64_t wc = ways[(uint64_t)(c + 1) * w + (b - s)];
                if (r < wc) {
                    for (uint64_t y = x; y; y &= y - 1ull) {
                        // insertion keeps the ids ascending
                        uint32_t v = verts[coff[c] + (uint32_t)__builtin_ctzll(y)];
                        uint32_t p = len++;
                        while (p > 0 && o[p - 1] > v) {
                            o[p] = o[p - 1];
                            --p;
                        }
                        o[p] = v;
                    }
                    b -= s;
                    break;
                }
                r -= wc;
            }
        }
        sizes[t] = len;
    }
}

inline uint32_t en_grid(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(b, 1), 4096);
}

template <typename C>
vc_status enum_t(vc_ctx* c, const RootGraph& g, uint32_t k, uint64_t max_covers, uint32_t* covers,
                 uint32_t* sizes, uint64_t* count) {
    hipStream_t s = c->stream;
    const uint32_t n = g.n;
    const C* col = (const C*)g.col;
    const uint32_t grid = en_grid(n);
    DevBuf* B = c->en;
    // ctr: 0 changed, 1 max component size, 2 sum of lb, 3 error bits,
    // 4-5 covers of all components (64-bit)
    HIPCHK(ensure(c->pool, B[0], 64));
    uint32_t* ctr = (uint32_t*)B[0].p;
    HIPCHK(ensure(c->pool, B[1], 4ull * n));        // label
    HIPCHK(ensure(c->pool, B[2], 4ull * (n + 1)));  // root flags, then component sizes
    HIPCHK(ensure(c->pool, B[3], 4ull * (n + 1)));  // rank of each root
    HIPCHK(ensure(c->pool, B[4], 4ull * n));        // local ids
    HIPCHK(ensure(c->pool, B[5], 4ull * n));        // vertices by component
    HIPCHK(ensure(c->pool, B[6], 4ull * (n / 2048 + 4)));  // scan scratch
    uint32_t *label = (uint32_t*)B[1].p, *flag = (uint32_t*)B[2].p, *rank = (uint32_t*)B[3].p;
    uint32_t *loc = (uint32_t*)B[4].p, *verts = (uint32_t*)B[5].p, *tmp = (uint32_t*)B[6].p;
    HIPCHK(hipMemsetAsync(ctr, 0, 64, s));
    hipLaunchKernelGGL(k_en_label_init, dim3(grid), dim3(256), 0, s, n, g.off, label);
    for (uint32_t it = 0;; it += 8) {
        HIPCHK(hipMemsetAsync(ctr, 0, 4, s));
        for (uint32_t j = 0; j < 8; ++j)
            hipLaunchKernelGGL(k_en_label_prop<C>, dim3(grid), dim3(256), 0, s, n, g.off, col,
                               label, ctr);
        HIPCHK(hipGetLastError());
        uint32_t ch = 0;
        HIPCHK(hipMemcpyAsync(&ch, ctr, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ch == 0) break;
        if (it > n + 8u) return VC_EDEVICE;  // labels only decrease
    }
    hipLaunchKernelGGL(k_en_roots, dim3(grid), dim3(256), 0, s, n, label, flag);
    HIPCHK(scan_u32(flag, n, rank, tmp, s));
    uint32_t ncomp = 0;
    HIPCHK(hipMemcpyAsync(&ncomp, rank + n, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ncomp == 0) return VC_EDEVICE;  // an edge makes a component
    uint32_t* csize = flag;  // roots are ranked: reuse the flags as sizes
    HIPCHK(hipMemsetAsync(csize, 0, 4ull * (ncomp + 1), s));
    hipLaunchKernelGGL(k_en_local, dim3(grid), dim3(256), 0, s, n, label, rank, loc, csize,
                       ctr + 1);
    uint32_t maxsize = 0;
    HIPCHK(hipMemcpyAsync(&maxsize, ctr + 1, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (maxsize > EN_MAXC) return VC_ERANGE;
    HIPCHK(ensure(c->pool, B[7], 4ull * (ncomp + 1)));  // component offsets
    uint32_t* coff = (uint32_t*)B[7].p;
    HIPCHK(scan_u32(csize, ncomp, coff, tmp, s));
    hipLaunchKernelGGL(k_en_place, dim3(grid), dim3(256), 0, s, n, label, rank, loc, coff, verts);
    // lower bounds, then counts by size
    HIPCHK(ensure(c->pool, B[8], 4ull * ncomp + 4ull * (ncomp + 1)));  // lb, totals
    uint32_t* lb = (uint32_t*)B[8].p;
    uint32_t* tot = lb + ncomp;
    HIPCHK(ensure(c->pool, B[9], 8ull * 64u * ncomp));
    uint64_t* cnt = (uint64_t*)B[9].p;
    const uint32_t cgrid = std::min<uint32_t>(ncomp, 65535u);
    hipLaunchKernelGGL(k_en_lb<C>, dim3(cgrid), dim3(64), 0, s, ncomp, g.off, col, loc, verts,
                       coff, lb, ctr + 2);
    const uint64_t nl = c->opts.node_limit;
    // 2^L threads per component, about 2^24 threads in all: most prefixes
    // end early (cut or dropped), and the deeper the split, the more evenly
    // the surviving subtrees spread over the threads
    uint32_t L = 4;
    while (L < 22 && ((uint64_t)ncomp << (L + 1)) <= (1ull << 24)) ++L;
    const uint32_t per = (1u << L) > 256u ? (1u << L) / 256u : 1u;
    const uint64_t eblocks = (uint64_t)ncomp * per;
    if (eblocks > 0x7FFFFFFFull) return VC_ERANGE;
    HIPCHK(hipMemsetAsync(cnt, 0, 8ull * 64u * ncomp, s));
    hipLaunchKernelGGL(k_en_enum<C>, dim3((uint32_t)eblocks), dim3(256), 0, s, ncomp, L, g.off, col,
                       loc, verts, coff, lb, ctr + 2, (int64_t)k, 0,
                       (unsigned long long*)cnt, (uint32_t*)nullptr, (const uint32_t*)nullptr,
                       (uint64_t*)nullptr, nl, ctr + 3);
    hipLaunchKernelGGL(k_en_tot, dim3(en_grid(ncomp)), dim3(256), 0, s, ncomp,
                       (const unsigned long long*)cnt, tot,
                       reinterpret_cast<unsigned long long*>(ctr + 4));
    HIPCHK(hipGetLastError());
    // list offsets (the component lists stay below 2^26 entries in all)
    HIPCHK(ensure(c->pool, B[10], 4ull * (ncomp + 1)));
    uint32_t* loff = (uint32_t*)B[10].p;
    HIPCHK(scan_u32(tot, ncomp, loff, tmp, s));
    uint32_t hdr[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(&hdr[0], ctr + 3, 12, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hdr[0] & 1u) return VC_ETIMEDOUT;
    const uint64_t nlist = (uint64_t)hdr[1] | ((uint64_t)hdr[2] << 32);
    if ((hdr[0] & 2u) || nlist > EN_LIST_MAX) return VC_ERANGE;
    const uint64_t wsz = ((uint64_t)ncomp + 1u) * ((uint64_t)k + 1u);
    if (wsz > EN_WAYS_MAX) return VC_ERANGE;
    HIPCHK(ensure(c->pool, B[11], 8ull * (nlist ? nlist : 1) + 8ull * wsz));
    uint64_t* list = (uint64_t*)B[11].p;
    uint64_t* ways = list + (nlist ? nlist : 1);
    if (nlist) {
        uint32_t* cur = tot;  // the totals are in loff now: reuse as cursors
        HIPCHK(hipMemsetAsync(cur, 0, 4ull * ncomp, s));
        hipLaunchKernelGGL(k_en_enum<C>, dim3((uint32_t)eblocks), dim3(256), 0, s, ncomp, L, g.off,
                           col, loc, verts, coff, lb, ctr + 2, (int64_t)k, 1,
                           (unsigned long long*)cnt, cur, loff, list, nl, ctr + 3);
    }
    hipLaunchKernelGGL(k_en_ways, dim3(1), dim3(64), 0, s, ncomp, k, cnt, ways);
    HIPCHK(hipGetLastError());
    uint64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, ways + k, 8, hipMemcpyDeviceToHost, s));  // ways[0][k]
    HIPCHK(hipStreamSynchronize(s));
    *count = total;
    const uint64_t nout = std::min<uint64_t>(total, max_covers);
    if (nout && k) {
        HIPCHK(ensure(c->pool, B[12], 4ull * nout * k + 4ull * nout));
        uint32_t* dout = (uint32_t*)B[12].p;
        uint32_t* dsz = dout + nout * k;
        hipLaunchKernelGGL(k_en_unrank, dim3(en_grid(nout)), dim3(256), 0, s, nout, ncomp, k, ways,
                           loff, list, coff, verts, dout, dsz);
        HIPCHK(hipGetLastError());
        if (covers) HIPCHK(hipMemcpyAsync(covers, dout, 4ull * nout * k, hipMemcpyDeviceToHost, s));
        if (sizes) HIPCHK(hipMemcpyAsync(sizes, dsz, 4ull * nout, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } else if (nout && sizes) {
        memset(sizes, 0, 4ull * nout);  // k = 0: the only cover is empty
    }
    return VC_OK;
}

}  // namespace

}  // namespace vc

extern "C" vc_status vc_param_enum(vc_ctx* c, const vc_csr* g, uint32_t k, uint64_t max_covers,
                                   uint32_t* covers, uint32_t* sizes, uint64_t* count) {
    if (!c || !g || !count) return VC_EINVAL;
    if (max_covers && ((k && !covers) || !sizes)) return VC_EINVAL;
    if (vc::server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    vc::pool_reset(c);
    vc::RootGraph rg;
    vc_status st = vc::stage_input(c, g, &rg);
    if (st) return st;
    if (g->n == 0 || g->nnz == 0) {
        // no edge: the empty set is the one minimal cover
        *count = 1;
        if (max_covers && sizes) sizes[0] = 0;
        return VC_OK;
    }
    uint64_t cnt = 0;
    st = g->col_bytes == 2
             ? vc::enum_t<uint16_t>(c, rg, k, max_covers, covers, sizes, &cnt)
             : vc::enum_t<uint32_t>(c, rg, k, max_covers, covers, sizes, &cnt);
    if (st) return st;
    *count = cnt;
    return VC_OK;
}
