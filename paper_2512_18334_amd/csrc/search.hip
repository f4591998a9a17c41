// search.hip -- the persistent component-aware branch-and-reduce search.
//
// One 64-lane wave is one worker (Sec. II-C: prior work uses thread blocks;
// on gfx950 a wave64 needs no block barriers and many more workers fit).
// Each worker keeps the node it is solving in LDS: the degree array (in the
// narrow type chosen after the root reduction, Sec. IV-D) plus a compacted
// list of the live vertices (ballot/mbcnt compaction instead of the paper's
// [lo, hi] window, Sec. IV-C), so rules, stopping tests and the component
// search touch live vertices only.  Pending nodes go to the worker's private
// stack in HBM or, when other workers are idle, to a shared bounded MPMC
// worklist (Sec. II-C).  Branches on components (Alg. 2) are registered in a
// registry in HBM; the last descendant to finish does the post-processing
// (Sec. III-C).
#include "dev_common.hpp"
#include "internal.hpp"
#include "vc.h"

namespace vc {

__device__ __forceinline__ uint32_t uni(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ int uni(int x) {
    return (int)__builtin_amdgcn_readfirstlane((uint32_t)x);
}
__device__ __forceinline__ uint64_t uni(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Visit every CSR entry of the rows of list[0..cnt): lane t of a 64-wide
// chunk of the flattened rows finds its row by a binary search over the
// lanes' exclusive prefix sums (load-balanced expansion).  f(ok, v, w) is
// called by all lanes in lock-step; ok is false on padding lanes.
template <typename C, typename F>
__device__ __forceinline__ void for_rows(const uint32_t* off, const C* col,
                                         const uint32_t* list, uint32_t cnt, F&& f) {
    const uint32_t l = lane();
    for (uint32_t base = 0; base < cnt; base += 64) {
        uint32_t i = base + l;
        uint32_t v = 0, r0 = 0, len = 0;
        if (i < cnt) {
            v = list[i];
            r0 = off[v];
            len = off[v + 1] - r0;
        }
        uint32_t incl = wave_incl_scan(len);
        uint32_t excl = incl - len;
        uint32_t total = shfl(incl, 63);
        for (uint32_t t0 = 0; t0 < total; t0 += 64) {
            uint32_t t = t0 + l;
            uint32_t j = 0;
#pragma unroll
            for (uint32_t step = 32; step >= 1; step >>= 1) {
                uint32_t c = j + step;
                uint32_t ec = shfl(excl, c & 63u);
                if (c < 64u && ec <= t) j = c;
            }
            uint32_t vj = shfl(v, j);
            uint32_t e = shfl(r0, j) + (t - shfl(excl, j));
            bool ok = t < total;
            uint32_t w = ok ? (uint32_t)col[e] : 0u;
            f(ok, vj, w);
        }
    }
}

template <typename D, typename C>
struct Worker {
    using DG = Deg<D>;
    const SearchArgs& A;
    D* deg;
    uint32_t *L, *Q, *R, *VB, *PB, *misc;
    const uint32_t* off;
    const C* col;
    uint32_t n, n_pad, bw;
    // node state (wave-uniform)
    uint32_t nl;    // live vertices in L
    int s;          // |S| in scope
    int scope;      // registry entry of the scope
    int best;       // scope bound used at this node
    uint64_t e2;    // sum of live degrees = 2|E|
    uint64_t key;   // max over live v of (deg << 32 | ~v): v_max, lowest id on ties
    bool known_connected;
    // worker state
    uint8_t* stack;
    uint32_t top;
    uint64_t nodes, cbr, comps, dons, pushes, nodes_flushed;

    __device__ Worker(const SearchArgs& a, uint8_t* lds) : A(a) {
        deg = reinterpret_cast<D*>(lds);
        L = reinterpret_cast<uint32_t*>(lds + a.lds_L);
        Q = reinterpret_cast<uint32_t*>(lds + a.lds_Q);
        R = reinterpret_cast<uint32_t*>(lds + a.lds_R);
        VB = reinterpret_cast<uint32_t*>(lds + a.lds_VB);
        PB = reinterpret_cast<uint32_t*>(lds + a.lds_PB);
        misc = reinterpret_cast<uint32_t*>(lds + a.lds_misc);
        off = a.off;
        col = reinterpret_cast<const C*>(a.col);
        n = a.n;
        n_pad = a.n_pad;
        bw = (n_pad + 31u) / 32u;
        stack = a.stacks + (size_t)blockIdx.x * a.stack_depth * a.slot_bytes;
        top = 0;
        nodes = cbr = comps = dons = pushes = nodes_flushed = 0;
        known_connected = false;
    }

    // ------------------------------------------------------- live list

    // rebuild L from the whole degree array
    __device__ void build_live() {
        const uint32_t l = lane();
        uint32_t cnt = 0;
        uint64_t sum = 0, k = 0;
        for (uint32_t base = 0; base < n; base += 64) {
            uint32_t v = base + l;
            uint32_t d = v < n ? DG::get(deg, v) : 0u;
            bool lv = DG::live(d);
            uint64_t m = ballot(lv);
            if (lv) {
                L[cnt + mbcnt(m)] = v;
                sum += d;
                uint64_t kk = ((uint64_t)d << 32) | (uint32_t)~v;
                k = kk > k ? kk : k;
            }
            cnt += popc(m);
        }
        nl = cnt;
        e2 = wave_sum64(sum);
        key = wave_max64(k);
        wave_sync();
    }

    // drop vertices that left the graph from L (in place), refresh e2 / key
    __device__ void recompact() {
        const uint32_t l = lane();
        uint32_t cnt = 0;
        uint64_t sum = 0, k = 0;
        for (uint32_t base = 0; base < nl; base += 64) {
            uint32_t i = base + l;
            uint32_t v = i < nl ? L[i] : 0u;
            uint32_t d = i < nl ? DG::get(deg, v) : 0u;
            bool lv = DG::live(d);
            uint64_t m = ballot(lv);
            if (lv) {
                L[cnt + mbcnt(m)] = v;
                sum += d;
                uint64_t kk = ((uint64_t)d << 32) | (uint32_t)~v;
                k = kk > k ? kk : k;
            }
            cnt += popc(m);
        }
        nl = cnt;
        e2 = wave_sum64(sum);
        key = wave_max64(k);
        wave_sync();
    }

    // Put the vertices of list[0..cnt) into the cover (duplicates allowed):
    // mark them, then remove their edges.  Returns how many were new.
    __device__ uint32_t take_list(uint32_t* list, uint32_t cnt) {
        const uint32_t l = lane();
        uint32_t nn = 0;
        for (uint32_t base = 0; base < cnt; base += 64) {
            uint32_t i = base + l;
            uint32_t v = i < cnt ? list[i] : 0u;
            bool isnew = i < cnt && DG::mark_in(deg, v);
            uint64_t m = ballot(isnew);
            if (isnew) list[nn + mbcnt(m)] = v;
            nn += popc(m);
        }
        wave_sync();
        for_rows(off, col, list, nn, [&](bool ok, uint32_t, uint32_t w) {
            if (ok && DG::live(DG::get(deg, w))) DG::dec(deg, w);
        });
        wave_sync();
        s += (int)nn;
        return nn;
    }

    // ------------------------------------------------------- reduce

    __device__ bool adjacent(uint32_t u, uint32_t w) {
        uint32_t a = u, b = w;
        uint32_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
        if (lb < la) { a = w; b = u; }
        for (uint32_t e = off[a]; e < off[a + 1]; ++e)
            if ((uint32_t)col[e] == b) return true;
        return false;
    }

    // Reduction rules of Sec. II-B to a joint fixpoint.  Applied in parallel
    // in two kinds of rounds: (1) every vertex of degree > best-|S|-1 at
    // once (each is in every cover of size < best); (2) degree-one and
    // degree-two-triangle rules at once, where a degree-one vertex whose
    // neighbour also has degree one defers to the lower id, and of the
    // degree-two vertices of one triangle only the lowest id fires, so the
    // joint effect equals some sequential order.  Returns false if pruned.
    __device__ bool reduce() {
        const uint32_t l = lane();
        bool changed_any = false;
        for (;;) {
            if (s >= best) return false;
            const int64_t b = (int64_t)best - s - 1;
            // (1) high degree
            uint32_t cnt = 0;
            for (uint32_t base = 0; base < nl; base += 64) {
                uint32_t i = base + l;
                uint32_t v = i < nl ? L[i] : 0u;
                bool f = i < nl && (int64_t)DG::get(deg, v) > b;
                uint64_t m = ballot(f);
                if (f) R[cnt + mbcnt(m)] = v;
                cnt += popc(m);
            }
            wave_sync();
            if (cnt) {
                take_list(R, cnt);
                recompact();
                changed_any = true;
                continue;
            }
            // (2) degree one / degree-two triangle
            for (uint32_t base = 0; base < nl; base += 64) {
                uint32_t i = base + l;
                uint32_t v = i < nl ? L[i] : 0u;
                uint32_t d = i < nl ? DG::get(deg, v) : 0u;
                uint32_t u = NONE, w = NONE;
                bool add_u = false, add_w = false;
                if (d == 1u || d == 2u) {
                    uint32_t got = 0;
                    for (uint32_t e = off[v]; e < off[v + 1] && got < d; ++e) {
                        uint32_t x = (uint32_t)col[e];
                        if (DG::live(DG::get(deg, x))) {
                            if (got == 0) u = x; else w = x;
                            ++got;
                        }
                    }
                    if (got < d) {
                        // inconsistent input (not a simple symmetric graph): no rule
                    } else if (d == 1u) {
                        add_u = !(DG::get(deg, u) == 1u && u < v);
                    } else if (adjacent(u, w)) {
                        add_u = !(DG::get(deg, u) == 2u && u < v) &&
                                !(DG::get(deg, w) == 2u && w < v);
                        add_w = add_u;
                    }
                }
                uint64_t m1 = ballot(add_u);
                if (add_u) R[cnt + mbcnt(m1)] = u;
                cnt += popc(m1);
                uint64_t m2 = ballot(add_w);
                if (add_w) R[cnt + mbcnt(m2)] = w;
                cnt += popc(m2);
            }
            wave_sync();
            if (cnt) {
                take_list(R, cnt);
                recompact();
                changed_any = true;
                continue;
            }
            break;
        }
        if (changed_any) known_connected = false;
        return true;
    }

    // ------------------------------------------------------- components

    // Breadth-first searches from the lowest-position unvisited live vertex
    // until all live vertices are visited (Sec. III-B).  Q receives the
    // vertices grouped by component, R[0..nc] the group boundaries, PB the
    // parity of each vertex's BFS level.  Returns nc.
    __device__ uint32_t find_components() {
        const uint32_t l = lane();
        for (uint32_t i = l; i < bw; i += 64) {
            VB[i] = 0u;
            PB[i] = 0u;
        }
        wave_sync();
        uint32_t qn = 0, nc = 0, sp = 0;
        while (qn < nl) {
            uint32_t seed = NONE;
            while (seed == NONE) {
                uint32_t i = sp + l;
                uint32_t v = i < nl ? L[i] : 0u;
                bool unv = i < nl && !((VB[v >> 5] >> (v & 31u)) & 1u);
                uint64_t m = ballot(unv);
                if (m) {
                    uint32_t first = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                    seed = shfl(v, first);
                    sp += first + 1u;
                } else {
                    sp += 64u;
                }
            }
            R[nc++] = qn;
            if (l == 0) {
                VB[seed >> 5] |= 1u << (seed & 31u);
                Q[qn] = seed;
            }
            ++qn;
            wave_sync();
            uint32_t fa = qn - 1, fb = qn, level = 0;
            while (fa < fb) {
                const bool odd = ((level + 1u) & 1u) != 0u;
                for_rows(off, col, Q + fa, fb - fa, [&](bool ok, uint32_t, uint32_t w) {
                    bool nw = false;
                    if (ok && DG::live(DG::get(deg, w))) {
                        uint32_t bit = 1u << (w & 31u);
                        uint32_t old = atomicOr(&VB[w >> 5], bit);
                        nw = !(old & bit);
                        if (nw && odd) atomicOr(&PB[w >> 5], bit);
                    }
                    uint64_t m = ballot(nw);
                    if (nw) Q[qn + mbcnt(m)] = w;
                    qn += popc(m);
                });
                wave_sync();
                fa = fb;
                fb = qn;
                ++level;
                if (nc == 1 && qn == nl) break;  // one component: stop early
            }
        }
        R[nc] = qn;
        wave_sync();
        return nc;
    }

    // ------------------------------------------------------- node I/O

    // Write a slot: header (stamp = worklist position, or 0 on the private
    // stack), the degree array src (n_pad elements in LDS) and the trailer.
    // Worklist slots (coh) are written with coherent stores; private stack
    // slots are written and read by this worker only and use plain stores.
    __device__ void write_slot(uint8_t* slot, int ss, int sc, uint32_t bv, uint32_t live,
                               uint32_t stamp, const D* src, bool coh) {
        const uint32_t l = lane();
        uint32_t hw = 0;  // header word l (8 words)
        if (l == 0) hw = (uint32_t)ss;
        if (l == 1) hw = (uint32_t)sc;
        if (l == 2) hw = bv;
        if (l == 3) hw = live;
        if (l == 4) hw = stamp;
        uint32_t* h = reinterpret_cast<uint32_t*>(slot);
        uint32_t* tr = reinterpret_cast<uint32_t*>(slot + A.slot_bytes - 16u);
        const uint32_t nw = (n_pad * (uint32_t)sizeof(D)) / 8u;
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(src);
        uint64_t* d8 = reinterpret_cast<uint64_t*>(slot + sizeof(SlotHdr));
        if (coh) {
            if (l < 8) st_coh(&h[l], hw);
            if (l < 4) st_coh(&tr[l], l == 0 ? stamp : 0u);
            for (uint32_t i = l; i < nw; i += 64) st_coh64(&d8[i], s8[i]);
        } else {
            if (l < 8) h[l] = hw;
            if (l < 4) tr[l] = l == 0 ? stamp : 0u;
            for (uint32_t i = l; i < nw; i += 64) d8[i] = s8[i];
        }
    }

    __device__ void store_slot(uint8_t* slot, int ss, int sc, uint32_t bv, uint32_t stamp,
                               bool coh) {
        write_slot(slot, ss, sc, bv, nl, stamp, deg, coh);
    }

    // copy a private-stack node into LDS; returns its pending branch vertex
    __device__ uint32_t copy_slot(const uint8_t* slot) {
        const uint32_t l = lane();
        const SlotHdr h = *reinterpret_cast<const SlotHdr*>(slot);
        const uint4* src = reinterpret_cast<const uint4*>(slot + sizeof(SlotHdr));
        uint4* dst = reinterpret_cast<uint4*>(deg);
        const uint32_t nv = (n_pad * (uint32_t)sizeof(D)) / 16u;
        for (uint32_t i = l; i < nv; i += 64) dst[i] = src[i];
        s = uni(h.s);
        scope = uni(h.scope);
        uint32_t bv = uni(h.branch_v);
        wave_sync();
        return bv;
    }

    // copy a worklist node into LDS with coherent loads; returns the stamps
    // (header, trailer) through st0/st1 and the pending branch vertex
    __device__ uint32_t copy_slot_coh(const uint8_t* slot, uint32_t& st0, uint32_t& st1) {
        const uint32_t l = lane();
        const uint32_t* h = reinterpret_cast<const uint32_t*>(slot);
        const uint32_t* tr = reinterpret_cast<const uint32_t*>(slot + A.slot_bytes - 16u);
        uint32_t hw = l < 8 ? ld_coh(&h[l]) : 0u;
        uint32_t t0 = l == 0 ? ld_coh(&tr[0]) : 0u;
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(slot + sizeof(SlotHdr));
        uint64_t* d8 = reinterpret_cast<uint64_t*>(deg);
        const uint32_t nw = (n_pad * (uint32_t)sizeof(D)) / 8u;
        for (uint32_t i = l; i < nw; i += 64) d8[i] = ld_coh64(&s8[i]);
        s = (int)shfl(hw, 0);
        scope = (int)shfl(hw, 1);
        const uint32_t bv = shfl(hw, 2);
        st0 = shfl(hw, 4);
        st1 = shfl(t0, 0);
        s = uni(s);
        scope = uni(scope);
        st0 = uni(st0);
        st1 = uni(st1);
        wave_sync();
        return uni(bv);
    }

    // start on a node copied into LDS: live list, then the pending N(v)
    __device__ void begin_node(uint32_t bv) {
        build_live();
        known_connected = false;
        if (bv != NONE) take_neighbours(bv);
    }

    // the N(v) branch: every live neighbour of v goes into the cover
    __device__ void take_neighbours(uint32_t v) {
        const uint32_t l = lane();
        uint32_t cnt = 0;
        const uint32_t r0 = off[v], r1 = off[v + 1];
        for (uint32_t e0 = r0; e0 < r1; e0 += 64) {
            uint32_t e = e0 + l;
            uint32_t w = e < r1 ? (uint32_t)col[e] : 0u;
            bool lv = e < r1 && DG::live(DG::get(deg, w));
            uint64_t m = ballot(lv);
            if (lv) R[cnt + mbcnt(m)] = w;
            cnt += popc(m);
        }
        wave_sync();
        take_list(R, cnt);
        recompact();
    }

    // ------------------------------------------------------- worklist

    __device__ bool hungry() {
        if (A.flags & VC_OPT_NO_LOAD_BALANCE) return false;
        int idle = 0;
        uint64_t h = 0, t = 0;
        if (lane() == 0) {
            idle = ld_relaxed(&A.ctl->idle);
            h = ld_relaxed(&A.ctl->wl_head);
            t = ld_relaxed(&A.ctl->wl_tail);
        }
        idle = uni(idle);
        uint64_t q = uni(t) - uni(h);
        return (uint64_t)idle > q + A.donate_slack;
    }

    // reserve a worklist position (UINT64_MAX when full)
    __device__ uint64_t wl_reserve() {
        uint64_t res = ~0ull;
        if (lane() == 0) {
            const uint64_t cap = A.wl_cap;
            uint64_t pos = ld_relaxed(&A.ctl->wl_tail);
            for (int tries = 0; tries < 256; ++tries) {
                uint64_t seq = ld_relaxed(&A.wl_seq[pos % cap]);
                int64_t diff = (int64_t)(seq - pos);
                if (diff == 0) {
                    if (cas_relaxed64(&A.ctl->wl_tail, pos, pos + 1)) {
                        res = pos;
                        break;
                    }
                    pos = ld_relaxed(&A.ctl->wl_tail);
                } else if (diff < 0) {
                    break;  // full
                } else {
                    pos = ld_relaxed(&A.ctl->wl_tail);
                }
            }
        }
        return uni(res);
    }

    __device__ void wl_publish(uint64_t pos) {
        wave_sync();
        if (lane() == 0) {
            add_relaxed(&A.ctl->outstanding, 1);
            st_release(&A.wl_seq[pos % A.wl_cap], pos + 1);
        }
        ++dons;
    }

    // take one node from the worklist into LDS; false if it looked empty
    __device__ bool wl_take() {
        uint64_t res = ~0ull;
        if (lane() == 0) {
            const uint64_t cap = A.wl_cap;
            uint64_t pos = ld_relaxed(&A.ctl->wl_head);
            for (int tries = 0; tries < 64; ++tries) {
                uint64_t seq = ld_relaxed(&A.wl_seq[pos % cap]);
                int64_t diff = (int64_t)(seq - (pos + 1));
                if (diff == 0) {
                    if (cas_relaxed64(&A.ctl->wl_head, pos, pos + 1)) {
                        fence_acquire();
                        res = pos;
                        break;
                    }
                    pos = ld_relaxed(&A.ctl->wl_head);
                } else if (diff < 0) {
                    break;  // empty
                } else {
                    pos = ld_relaxed(&A.ctl->wl_head);
                }
            }
        }
        res = uni(res);
        if (res == ~0ull) return false;
        wave_sync();
        const uint8_t* slot = A.wl_slots + (size_t)(res % A.wl_cap) * A.slot_bytes;
        const uint32_t want = (uint32_t)res;
        uint32_t s0 = 0, s1 = 0;
        uint32_t bv = copy_slot_coh(slot, s0, s1);
        for (uint32_t tries = 0; !(s0 == want && s1 == want) && tries < 100000; ++tries) {
            // an old copy of the slot was read: count it and read again
            if (lane() == 0) {
                if (tries == 0) add_relaxed(&A.ctl->stale, 1ull);
                fence_acquire();
            }
            wave_sync();
            bv = copy_slot_coh(slot, s0, s1);
        }
        if (lane() == 0) st_release(&A.wl_seq[res % A.wl_cap], res + A.wl_cap);
        begin_node(bv);
        return true;
    }

    // Place a pending node: the shared worklist when others are idle, else
    // the own stack; the caller fills the slot through fill(slot).
    template <typename Fill>
    __device__ bool push_node(Fill&& fill) {
        ++pushes;
        if (hungry()) {
            uint64_t pos = wl_reserve();
            if (pos != ~0ull) {
                fill(A.wl_slots + (size_t)(pos % A.wl_cap) * A.slot_bytes, (uint32_t)pos, true);
                wl_publish(pos);
                return true;
            }
        }
        if (top < A.stack_depth) {
            fill(stack + (size_t)top * A.slot_bytes, 0u, false);
            ++top;
            return true;
        }
        uint64_t pos = wl_reserve();
        if (pos != ~0ull) {
            fill(A.wl_slots + (size_t)(pos % A.wl_cap) * A.slot_bytes, (uint32_t)pos, true);
            wl_publish(pos);
            return true;
        }
        fail(VC_ENOMEM);
        return false;
    }

    __device__ void fail(int code) {
        if (lane() == 0) {
            atomicCAS(&A.ctl->err, 0, code);
            st_relaxed(&A.ctl->done, 1);
        }
    }

    // ------------------------------------------------------- registry

    __device__ int scope_best(int e) {
        int b = 0;
        if (lane() == 0) b = ld_relaxed(&A.reg[e].best);
        return uni(b);
    }
    __device__ int reg_field(const int* p) {
        int b = 0;
        if (lane() == 0) b = ld_relaxed(p);
        return uni(b);
    }

    __device__ void lock(int e) {
        if (lane() == 0) {
            uint32_t spins = 0;
            while (!cas_acquire(&A.reg[e].lock, 0, 1)) backoff(spins);
        }
        wave_sync();
    }
    __device__ void unlock(int e) {
        wave_sync();
        if (lane() == 0) st_release(&A.reg[e].lock, 0);
    }

    __device__ uint32_t* bitmap(int e) { return A.bitmaps + (size_t)e * A.bm_words; }

    // registry entries are only ever accessed with atomics
    __device__ void init_entry(int e, int best_or_sum, int live, int up, int cover_size,
                               int nchild, int size) {
        RegEntry* r = &A.reg[e];
        st_relaxed(&r->best, best_or_sum);
        st_relaxed(&r->live, live);
        st_relaxed(&r->up, up);
        st_relaxed(&r->lock, 0);
        st_relaxed(&r->cover_size, cover_size);
        st_relaxed(&r->nchild, nchild);
        st_relaxed(&r->size, size);
        st_relaxed(&r->pad, 0);
    }

    // write the IN marks of the LDS degree array as bitmap words
    __device__ void write_in_bitmap(uint32_t* bm) {
        const uint32_t l = lane();
        for (uint32_t wi = l; wi < A.bm_words; wi += 64) {
            uint32_t bits = 0;
            const uint32_t v0 = wi * 32u;
            for (uint32_t j = 0; j < 32u; ++j) {
                uint32_t v = v0 + j;
                if (v < n && DG::get(deg, v) == DG::IN) bits |= 1u << j;
            }
            st_coh(&bm[wi], bits);
        }
    }

    // Offer `val` (attained by the cover in LDS, or assembled from the
    // children of parent entry `from` when from >= 0) as a new Best of scope
    // entry e.  Returns true if it improved and the cover was written.
    __device__ bool improve(int e, int val, int from) {
        int old = 0;
        if (lane() == 0) old = min_relaxed(&A.reg[e].best, val);
        old = uni(old);
        if (val >= old) return false;
        lock(e);
        int cs = reg_field(&A.reg[e].cover_size);
        bool wrote = false;
        if (val < cs) {
            uint32_t* dst = bitmap(e);
            if (from < 0) {
                write_in_bitmap(dst);
            } else {
                const int nch = reg_field(&A.reg[from].nchild);
                for (uint32_t wi = lane(); wi < A.bm_words; wi += 64) {
                    uint32_t x = ld_coh(&bitmap(from)[wi]);
                    for (int c = 1; c <= nch; ++c) x |= ld_coh(&bitmap(from + c)[wi]);
                    st_coh(&dst[wi], x);
                }
            }
            wave_sync();
            if (lane() == 0) st_relaxed(&A.reg[e].cover_size, val);
            wrote = true;
        }
        unlock(e);
        if (A.pvc && e == 0 && val <= A.k) {
            if (lane() == 0) st_relaxed(&A.ctl->done, 1);
        }
        return wrote;
    }

    // A node of scope e has finished.  Walk the registry chain: the last
    // descendant of a component adds its Best to the parent's Sum; the last
    // component of a parent offers Sum to the ancestor's Best and finishes
    // the parent node in the ancestor's scope (Sec. III-C).
    __device__ void complete(int e, bool wrote) {
        while (e != 0) {
            int old = 0;
            if (lane() == 0) {
                old = wrote ? add_release(&A.reg[e].live, -1)
                            : add_relaxed(&A.reg[e].live, -1);
            }
            old = uni(old);
            if (old != 1) return;
            if (lane() == 0) fence_acquire();
            const int p = reg_field(&A.reg[e].up);
            const int cb = reg_field(&A.reg[e].best);
            if (lane() == 0) {
                add_relaxed(&A.reg[p].best, cb);
                old = add_acq_rel(&A.reg[p].live, -1);
            }
            old = uni(old);
            if (old != 1) return;
            wave_sync();
            const int sum = reg_field(&A.reg[p].best);
            const int a = reg_field(&A.reg[p].up);
            wrote = improve(a, sum, p);
            e = a;
        }
    }

    // ------------------------------------------------------- node handling

    __device__ void count_node() {
        ++nodes;
        if (A.node_limit && nodes - nodes_flushed >= 256) {
            uint64_t tot = 0;
            if (lane() == 0) tot = add_relaxed(&A.ctl->nodes, nodes - nodes_flushed);
            tot = uni(tot) + (nodes - nodes_flushed);
            nodes_flushed = nodes;
            if (tot > A.node_limit) fail(VC_ETIMEDOUT);
        }
    }

    __device__ bool stop_requested() {
        int d = 0;
        if (lane() == 0) d = ld_relaxed(&A.ctl->done);
        return uni(d) != 0;
    }

    // vertex branch on v_max: the G - N(v) child is pushed (lazily, as the
    // current state plus v), the G - v child continues here
    __device__ bool vertex_branch() {
        const uint32_t v = ~(uint32_t)(key & 0xFFFFFFFFull);
        if (scope != 0 && lane() == 0) add_relaxed(&A.reg[scope].live, 1);
        const int ss = s, sc = scope;
        if (!push_node([&](uint8_t* slot, uint32_t stamp, bool coh) {
                store_slot(slot, ss, sc, v, stamp, coh);
            }))
            return false;
        if (lane() == 0) R[0] = v;
        wave_sync();
        take_list(R, 1);
        recompact();
        known_connected = false;  // removing v may split the graph
        return true;
    }

    // Classify the components found: cliques and chordless cycles are
    // solved on the spot (Sec. III-D); the others are listed in
    // R[nc+1 ..].  Returns the number of other components.
    __device__ uint32_t settle_simple_components(uint32_t nc) {
        const uint32_t l = lane();
        uint32_t* NT = R + nc + 1;
        uint32_t nt = 0;
        for (uint32_t c = 0; c < nc; ++c) {
            const uint32_t a = R[c], b = R[c + 1], size = b - a;
            bool clique = true, cyc = true;
            uint32_t mx = 0;
            for (uint32_t i = a + l; i < b; i += 64) {
                uint32_t v = Q[i];
                uint32_t d = DG::get(deg, v);
                clique = clique && d == size - 1u;
                cyc = cyc && d == 2u;
                mx = v > mx ? v : mx;
            }
            clique = ballot(!clique) == 0;
            cyc = ballot(!cyc) == 0;
            mx = wave_max(mx);
            if (clique) {
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    DG::set(deg, v, v == mx ? 0u : DG::IN);
                }
                s += (int)size - 1;
            } else if (cyc) {
                const uint32_t last = Q[b - 1];
                const bool fix = (size & 1u) && !((PB[last >> 5] >> (last & 31u)) & 1u);
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    bool take = ((PB[v >> 5] >> (v & 31u)) & 1u) || (fix && v == last);
                    DG::set(deg, v, take ? DG::IN : 0u);
                }
                s += (int)(size + 1u) / 2;
            } else {
                if (l == 0) NT[nt] = c;
                ++nt;
            }
            wave_sync();
        }
        return nt;
    }

    // Branch on components (Alg. 2): one parent entry plus one child entry
    // per component, best_i = min(best - sum, |V_i| - 1); children other
    // than the first are pushed, the first continues here.  Returns CB_FULL
    // when the registry is full (the caller then branches on a vertex) and
    // CB_PRUNED when the scope's bound leaves no room for the components.
    enum { CB_OK = 0, CB_FULL = 1, CB_PRUNED = 2 };
    __device__ int component_branch(uint32_t nc, uint32_t nt) {
        const uint32_t l = lane();
        const uint32_t* NT = R + nc + 1;
        // the bound may have improved since the node started: every
        // component needs at least one vertex
        const int bnow = scope_best(scope);
        const int base_sum = s;
        if ((int64_t)base_sum + nt >= (int64_t)bnow) return CB_PRUNED;
        uint32_t want = (nt + 1u + 3u) & ~3u;  // whole 128-byte lines
        uint32_t p = NONE;
        if (l == 0) {
            // never bump past the capacity, so a full registry stays full
            uint32_t cur = ld_relaxed(&A.ctl->reg_next);
            while ((uint64_t)cur + want <= A.reg_cap) {
                uint32_t prev = atomicCAS(&A.ctl->reg_next, cur, cur + want);
                if (prev == cur) {
                    p = cur;
                    break;
                }
                cur = prev;
            }
        }
        p = uni(p);
        if (p == NONE) return CB_FULL;
        // parent entry: Sum = |S| (with the settled components), LiveComps
        if (l == 0) init_entry((int)p, base_sum, (int)nt, scope, INF, (int)nt, 0);
        write_in_bitmap(bitmap((int)p));
        // child entries and their initial covers (V_i minus one vertex)
        for (uint32_t j = 0; j < nt; ++j) {
            const uint32_t c = NT[j];
            const uint32_t a = R[c], b = R[c + 1], size = b - a;
            int bi = bnow - base_sum;
            const bool attained = (int)size - 1 <= bi;
            if (attained) bi = (int)size - 1;
            uint32_t mx = 0;
            for (uint32_t i = a + l; i < b; i += 64) mx = Q[i] > mx ? Q[i] : mx;
            mx = wave_max(mx);
            if (l == 0)
                init_entry((int)(p + 1 + j), bi, 1, (int)p, attained ? (int)size - 1 : INF, 0,
                           (int)size);
            if (attained) {
                for (uint32_t i = l; i < bw; i += 64) VB[i] = 0u;
                wave_sync();
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    if (v != mx) atomicOr(&VB[v >> 5], 1u << (v & 31u));
                }
                wave_sync();
                uint32_t* bm = bitmap((int)(p + 1 + j));
                for (uint32_t i = l; i < A.bm_words; i += 64) st_coh(&bm[i], VB[i]);
            }
            wave_sync();
        }
        // entries and initial covers must be visible to whichever worker
        // finishes the last component
        wave_sync();
        if (l == 0) fence_release();
        cbr += 1;
        comps += nt;
        // children 1..nt-1 go out as nodes holding only their component
        for (uint32_t j = nt - 1; j >= 1; --j) {
            const uint32_t c = NT[j];
            const uint32_t a = R[c], b = R[c + 1];
            const int sc = (int)(p + 1 + j);
            // the child's degree array: this component only, built in L
            // (free until child 0 rebuilds it)
            D* cd = reinterpret_cast<D*>(L);
            {
                uint4* z = reinterpret_cast<uint4*>(cd);
                const uint32_t nv = (n_pad * (uint32_t)sizeof(D)) / 16u;
                for (uint32_t i = l; i < nv; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
                wave_sync();
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    cd[v] = (D)DG::get(deg, v);
                }
                wave_sync();
            }
            bool ok = push_node([&](uint8_t* slot, uint32_t stamp, bool coh) {
                write_slot(slot, 0, sc, NONE, b - a, stamp, cd, coh);
            });
            if (!ok) return CB_OK;  // error flagged; the next node stops
        }
        // child 0 continues in LDS: keep only its component, S restarts
        {
            const uint32_t c = NT[0];
            const uint32_t a = R[c], b = R[c + 1];
            for (uint32_t i = l; i < bw; i += 64) VB[i] = 0u;
            wave_sync();
            for (uint32_t i = a + l; i < b; i += 64) {
                uint32_t v = Q[i];
                atomicOr(&VB[v >> 5], 1u << (v & 31u));
            }
            wave_sync();
            for (uint32_t v = l; v < n; v += 64)
                if (!((VB[v >> 5] >> (v & 31u)) & 1u)) DG::set(deg, v, 0u);
            wave_sync();
            s = 0;
            scope = (int)(p + 1);
            build_live();
            known_connected = true;
        }
        return CB_OK;
    }

    // Process one node and, depth-first, its first children in place.
    __device__ void process() {
        for (;;) {
            count_node();
            if (stop_requested()) return;
            best = scope_best(scope);
            if (!reduce()) {
                complete(scope, false);
                return;
            }
            const int64_t b = (int64_t)best - s - 1;
            const uint64_t E = e2 / 2u;
            if (b < 0 || (int64_t)E > b * b) {
                complete(scope, false);
                return;
            }
            if (E == 0) {
                bool w = improve(scope, s, -1);
                complete(scope, w);
                return;
            }
            if (!(A.flags & VC_OPT_NO_COMPONENTS) && !known_connected) {
                const uint32_t nc = find_components();
                const uint32_t nt = settle_simple_components(nc);
                if (nt != nc) recompact();
                if (s >= best) {
                    complete(scope, false);
                    return;
                }
                if (nt == 0) {
                    if (s < best) {
                        bool w = improve(scope, s, -1);
                        complete(scope, w);
                    } else {
                        complete(scope, false);
                    }
                    return;
                }
                if (nt == 1) {
                    known_connected = true;
                    if (nt != nc) continue;  // re-run the rules on what is left
                } else {
                    const int cb = component_branch(nc, nt);
                    if (cb == CB_OK) continue;
                    if (cb == CB_PRUNED) {
                        complete(scope, false);
                        return;
                    }
                }
            }
            if (!vertex_branch()) return;
        }
    }

    __device__ void flush_stats() {
        if (lane() == 0) {
            add_relaxed(&A.ctl->nodes, nodes - nodes_flushed);
            add_relaxed(&A.ctl->comp_branches, cbr);
            add_relaxed(&A.ctl->components, comps);
            add_relaxed(&A.ctl->donations, dons);
            add_relaxed(&A.ctl->pushes, pushes);
        }
    }

    __device__ void run() {
        bool busy = false;
        for (;;) {
            if (top > 0) {
                if (stop_requested()) break;
                --top;
                begin_node(copy_slot(stack + (size_t)top * A.slot_bytes));
            } else {
                if (busy && lane() == 0) add_relaxed(&A.ctl->outstanding, -1);
                busy = false;
                if (lane() == 0) add_relaxed(&A.ctl->idle, 1);
                uint32_t spins = 0;
                bool got = false, quit = false;
                const uint64_t t_idle = wall_clock64();
                for (;;) {
                    int d = 0, outst = 0;
                    uint64_t h = 0, t = 0;
                    if (lane() == 0) {
                        d = ld_relaxed(&A.ctl->done);
                        outst = ld_relaxed(&A.ctl->outstanding);
                        h = ld_relaxed(&A.ctl->wl_head);
                        t = ld_relaxed(&A.ctl->wl_tail);
                    }
                    d = uni(d);
                    outst = uni(outst);
                    h = uni(h);
                    t = uni(t);
                    if (d) { quit = true; break; }
                    if (t > h) {
                        if (wl_take()) { got = true; break; }
                    } else if (outst == 0) {
                        quit = true;
                        break;
                    }
                    if (wall_clock64() - t_idle > A.watchdog_ticks) {
                        // waited far longer than any node takes: give up
                        fail(VC_EDEVICE);
                        quit = true;
                        break;
                    }
                    if (lane() == 0) backoff(spins);
                }
                if (lane() == 0) add_relaxed(&A.ctl->idle, -1);
                if (quit) break;
                busy = got;
            }
            process();
        }
        flush_stats();
    }
};

template <typename D, typename C>
__global__ void __launch_bounds__(64) search_kernel(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    Worker<D, C> w(a, lds);
    w.run();
}

// Root node and control block.  The root node (the whole induced subgraph,
// scope 0) is placed in worklist slot 0.
template <typename D>
__global__ void search_init_kernel(SearchArgs a, int best0, const uint32_t* kdeg) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < a.wl_cap; i += stride) a.wl_seq[i] = (i == 0) ? 1ull : (uint64_t)i;
    D* d = reinterpret_cast<D*>(a.wl_slots + sizeof(SlotHdr));
    for (uint32_t v = tid; v < a.n_pad; v += stride) d[v] = (D)(v < a.n ? kdeg[v] : 0u);
    if (tid == 0) {
        SlotHdr* h = reinterpret_cast<SlotHdr*>(a.wl_slots);
        h->s = 0;
        h->scope = 0;
        h->branch_v = NONE;
        h->nlive = a.n;
        h->stamp = 0;
        *reinterpret_cast<uint32_t*>(a.wl_slots + a.slot_bytes - 16u) = 0u;
        Ctl* c = a.ctl;
        c->wl_head = 0;
        c->wl_tail = 1;
        c->outstanding = 1;
        c->idle = 0;
        c->done = 0;
        c->err = 0;
        c->reg_next = 4;  // entry 0 is the root scope; allocations are 4-aligned
        c->nodes = c->comp_branches = c->components = c->donations = c->pushes = 0;
        c->stale = 0;
        RegEntry r;
        r.best = best0;
        r.live = 1;
        r.up = -1;
        r.lock = 0;
        r.cover_size = INF;
        r.nchild = 0;
        r.size = (int)a.n;
        r.pad = 0;
        a.reg[0] = r;
    }
}

template <typename D, typename C>
static hipError_t launch_t(const SearchArgs& a, uint32_t workers, hipStream_t st) {
    hipLaunchKernelGGL((search_kernel<D, C>), dim3(workers), dim3(64), a.lds_bytes, st, a);
    return hipGetLastError();
}

hipError_t launch_search(const SearchArgs& a, uint32_t deg_bytes, uint32_t col_bytes,
                         uint32_t workers, hipStream_t st) {
    if (col_bytes == 2) {
        if (deg_bytes == 1) return launch_t<uint8_t, uint16_t>(a, workers, st);
        if (deg_bytes == 2) return launch_t<uint16_t, uint16_t>(a, workers, st);
        return launch_t<uint32_t, uint16_t>(a, workers, st);
    }
    if (deg_bytes == 1) return launch_t<uint8_t, uint32_t>(a, workers, st);
    if (deg_bytes == 2) return launch_t<uint16_t, uint32_t>(a, workers, st);
    return launch_t<uint32_t, uint32_t>(a, workers, st);
}

template <typename D, typename C>
static hipError_t occ_t(uint32_t lds_bytes, int* bpc) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, search_kernel<D, C>, 64, lds_bytes);
}

hipError_t search_occupancy(uint32_t deg_bytes, uint32_t col_bytes, uint32_t lds_bytes,
                            int* bpc) {
    if (col_bytes == 2) {
        if (deg_bytes == 1) return occ_t<uint8_t, uint16_t>(lds_bytes, bpc);
        if (deg_bytes == 2) return occ_t<uint16_t, uint16_t>(lds_bytes, bpc);
        return occ_t<uint32_t, uint16_t>(lds_bytes, bpc);
    }
    if (deg_bytes == 1) return occ_t<uint8_t, uint32_t>(lds_bytes, bpc);
    if (deg_bytes == 2) return occ_t<uint16_t, uint32_t>(lds_bytes, bpc);
    return occ_t<uint32_t, uint32_t>(lds_bytes, bpc);
}

hipError_t launch_search_init(const SearchArgs& a, int best0, uint32_t deg_bytes,
                              const uint32_t* kdeg, hipStream_t st) {
    uint32_t work = a.wl_cap > a.n_pad ? a.wl_cap : a.n_pad;
    uint32_t blocks = (work + 255u) / 256u;
    if (blocks > 1024u) blocks = 1024u;
    if (blocks == 0) blocks = 1;
    if (deg_bytes == 1)
        hipLaunchKernelGGL(search_init_kernel<uint8_t>, dim3(blocks), dim3(256), 0, st, a, best0, kdeg);
    else if (deg_bytes == 2)
        hipLaunchKernelGGL(search_init_kernel<uint16_t>, dim3(blocks), dim3(256), 0, st, a, best0, kdeg);
    else
        hipLaunchKernelGGL(search_init_kernel<uint32_t>, dim3(blocks), dim3(256), 0, st, a, best0, kdeg);
    return hipGetLastError();
}

}  // namespace vc
