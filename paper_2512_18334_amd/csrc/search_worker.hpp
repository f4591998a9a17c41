// search_worker.hpp -- the persistent component-aware branch-and-reduce search
// (the worker and its kernels, templated on the degree-array type).
//
// One 64-lane wave is one worker (prior GPU work uses thread blocks, Sec.
// II-C; on gfx950 a wave64 needs no block barriers and many more workers
// fit).  A worker keeps the node it is solving in LDS: the degree array in
// the narrow type chosen after the root reduction (Sec. IV-D) plus a
// compacted list of live vertices (ballot/mbcnt compaction in place of the
// paper's [lo, hi] window, Sec. IV-C), so rules, stopping tests and the
// component search touch live vertices only.  Pending nodes go to the
// worker's private stack in HBM or, while other workers are idle, to a
// shared bounded MPMC worklist (Sec. II-C).  Branches on components (Alg. 2)
// are registered in a registry in HBM whose last descendant does the
// post-processing (Sec. III-C).  A small component is also re-induced as a
// subgraph of its own with local ids (the paper's reduce-then-induce step,
// Sec. IV-B, applied again at every branch on components), held in an LDS
// graph cache while a worker is in its scope, so per-node work scales with
// the component, not with the whole graph.
//
// Memory model: data that crosses workers (worklist slots, cover bitmaps,
// registry entries, arena graphs) is only written and read with coherent
// (device-scope) accesses, and s_waitcnt ordering points separate writing
// a payload from publishing it; private stacks use plain accesses.
#pragma once

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

// Visit every CSR entry of the rows of list[0..cnt) (load-balanced
// expansion): the rows of 64 list entries are laid end to end by a prefix
// sum of their lengths and cut into 64-entry chunks.  In a chunk, every row
// that starts there marks its lane at its start position in MK (64 words
// of LDS), and an inclusive max-scan over the marks gives each entry its
// row; entries before the first start continue the previous chunk's last
// row.  The positions of FOR_ROWS_AHEAD chunks are worked out first and
// their column loads issued together, so a graph read from HBM costs one
// memory latency per group of chunks rather than per chunk.  f(ok, v, w) is
// then called by all lanes in lock-step, chunk by chunk in order; ok is
// false on padding lanes.
constexpr uint32_t FOR_ROWS_AHEAD = 2;  // (4 and 8 measured 2-4% slower on blocks-and-hubs)

template <typename Off, typename Col, typename F>
__device__ __forceinline__ uint32_t for_rows(Off&& off, Col&& col, const uint32_t* list,
                                             uint32_t cnt, uint32_t* MK, F&& f) {
    const uint32_t l = lane();
    uint32_t entries = 0;  // CSR entries visited (wave-uniform)
    for (uint32_t base = 0; base < cnt; base += 64) {
        uint32_t i = base + l;
        uint32_t v = 0, r0 = 0, len = 0;
        if (i < cnt) {
            v = list[i];
            r0 = off(v);
            len = off(v + 1) - r0;
        }
        const uint32_t incl = wave_incl_scan(len);
        const uint32_t excl = incl - len;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        const uint32_t delta = r0 - excl;  // CSR position of flat entry t is t + delta
        uint32_t carry = 0;                // (lane + 1) of the row running into the chunk
        entries += total;
        for (uint32_t g0 = 0; g0 < total; g0 += 64u * FOR_ROWS_AHEAD) {
            uint32_t vv[FOR_ROWS_AHEAD], ee[FOR_ROWS_AHEAD], ww[FOR_ROWS_AHEAD];
            bool okk[FOR_ROWS_AHEAD];
#pragma unroll
            for (uint32_t k = 0; k < FOR_ROWS_AHEAD; ++k) {
                const uint32_t t0 = g0 + 64u * k;
                vv[k] = 0u;
                ee[k] = 0u;
                okk[k] = false;
                if (t0 < total) {  // wave-uniform
                    wave_sync();   // the previous chunk's reads of MK are done
                    MK[l] = 0u;
                    if (len && excl >= t0 && excl - t0 < 64u) MK[excl - t0] = l + 1u;
                    wave_sync();  // other lanes' marks are visible
                    uint32_t own = MK[l];
                    VC_DPP_SCAN(own, op_max, 0u);
                    own = own > carry ? own : carry;
                    carry = __builtin_amdgcn_readlane(own, 63);
                    const uint32_t j = own - 1u;
                    const uint32_t t = t0 + l;
                    okk[k] = t < total;
                    vv[k] = shfl(v, j);
                    ee[k] = t + shfl(delta, j);
                }
            }
#pragma unroll
            for (uint32_t k = 0; k < FOR_ROWS_AHEAD; ++k) ww[k] = okk[k] ? col(ee[k]) : 0u;
#pragma unroll
            for (uint32_t k = 0; k < FOR_ROWS_AHEAD; ++k)
                if (g0 + 64u * k < total) f(okk[k], vv[k], ww[k]);
        }
    }
    return entries;
}

// slot header word 7
constexpr uint32_t SLOT_COUNTED = 1u;  // the node holds a LiveNodes count of its scope
constexpr uint32_t SLOT_INDUCE = 2u;   // first node of a component child: induce its subgraph

template <typename D, bool HL>
struct Worker {
    using DG = Deg<D>;
    SearchArgs A;
    D* deg;
    uint32_t *L, *Q, *R, *VB, *PB, *MK, *G;
    // current graph view
    int view;
    uint32_t vn, vpad, vbw;
    // the view's CSR: in the LDS graph cache (G, columns from GC) or, when it
    // does not fit, in HBM (goff, gcol); every read branches on vlds, a
    // wave-uniform flag, so LDS views are read with LDS instructions only
    bool vlds;
    const uint32_t* goff;
    const uint32_t* gcol;
    uint32_t* GC;
    // node state (wave-uniform)
    uint32_t nl;    // live vertices in L
    int s;          // |S| in scope
    int scope;      // registry entry of the scope
    int best;       // scope bound used at this node
    uint64_t e2;    // sum of live degrees = 2|E|
    uint64_t key;   // max over live v of (deg << 32 | ~v): v_max, lowest id on ties
    bool known_connected;
    bool small_off;  // this node goes through the general path (after a split)
    bool induce_first;  // the fetched node is a component child's first node
    uint64_t *ADJ, *SM;  // small-node solver: adjacency masks, stack masks
    uint32_t* SS;        // and stack counts
    // worker state
    uint8_t* stack;
    uint32_t bot, top;  // private stack as a deque: pop at top, donate from bot
    uint32_t since_poll;
    // shared state read together in one round trip every POLL_EVERY nodes
    // (and when a node comes from elsewhere): stop flag, the instance's
    // state, idle workers, queued nodes and the current scope's Best.  A
    // stale Best is only a weaker bound, never a wrong one.
    static constexpr uint32_t POLL_EVERY = 2;  // (4: 5% slower on blocks-and-hubs)
    int c_done, c_inst_state, c_idle, c_best, c_best_scope;
    int64_t c_queued;
    uint64_t nodes, cbr, comps, dons, pushes, lviews, nodes_flushed;
    uint32_t chist[8];  // branches on components by components registered
    uint64_t cyc[6];
    uint64_t t_mark;
    uint64_t b_nodes, b_reg;  // algorithmic bytes written (node slots; registry)
    uint64_t b_rows;          // CSR bytes of removed vertices' rows read from HBM views
    uint64_t b_views;         // view bytes copied from HBM into the graph cache
    uint32_t inst;            // instance of the current node (batches)
    uint64_t inst_cnt;        // its nodes not yet added to inst_nodes

    __device__ __forceinline__ Worker(const SearchArgs& a, uint8_t* lds) : A(a) {
        deg = reinterpret_cast<D*>(lds);
        // the lists: LDS, or this worker's region of HBM
        uint8_t* lb = HL ? a.hl_base + (size_t)blockIdx.x * a.hl_stride : lds;
        L = reinterpret_cast<uint32_t*>(lb + a.lds_L);
        Q = reinterpret_cast<uint32_t*>(lb + a.lds_Q);
        R = reinterpret_cast<uint32_t*>(lb + a.lds_R);
        VB = reinterpret_cast<uint32_t*>(lds + a.lds_VB);
        PB = reinterpret_cast<uint32_t*>(lds + a.lds_PB);
        MK = reinterpret_cast<uint32_t*>(lds + a.lds_MK);
        ADJ = reinterpret_cast<uint64_t*>(lds + a.lds_MK + 256u);  // 128 x 2 words
        SM = ADJ + 256;                                              // 128 x 4 words
        SS = reinterpret_cast<uint32_t*>(SM + 512);                  // 128 counts
        small_off = false;
        G = reinterpret_cast<uint32_t*>(lds + a.lds_G);
        stack = a.stacks + (size_t)blockIdx.x * a.stack_depth * a.slot_bytes;
        bot = top = 0;
        b_nodes = b_reg = b_rows = b_views = 0;
        inst = 0;
        inst_cnt = 0;
        for (int i = 0; i < 6; ++i) cyc[i] = 0;
        t_mark = clock64();
        since_poll = POLL_EVERY;
        c_done = c_inst_state = c_idle = 0;
        c_best = INF;
        c_best_scope = -1;
        c_queued = 0;
        nodes = cbr = comps = dons = pushes = lviews = nodes_flushed = 0;
        for (int i = 0; i < 8; ++i) chist[i] = 0;
        known_connected = false;
        induce_first = false;
        view = -1;
        vn = vpad = vbw = 0;
        vlds = false;
        goff = gcol = nullptr;
        GC = G;
    }

    // Order the lanes' list traffic: LDS as wave_sync does; with the lists
    // in HBM, every memory operation of the wave is also complete first, so
    // a lane reads what another lane stored before this point.
    __device__ __forceinline__ void wsync() {
        if (HL) order_point();
        wave_sync();
    }

    // charge the shader cycles since the last mark to activity k
    __device__ __forceinline__ void charge(int k) {
        const uint64_t t = clock64();
        cyc[k] += t - t_mark;
        t_mark = t;
    }

    // ------------------------------------------------------- registry access

    __device__ __forceinline__ int reg_field(const int* p) {
        int b = 0;
        if (lane() == 0) b = ld_relaxed(p);
        return uni(b);
    }
    __device__ __forceinline__ int scope_best(int e) { return reg_field(&A.reg[e].best); }

    __device__ __forceinline__ void poll() {
        int d = 0, is = 0, idl = 0, bst = 0;
        uint64_t h = 0, t = 0;
        if (lane() == 0) {
            d = ld_relaxed(&A.ctl->done);
            if (A.batch) is = ld_relaxed(&A.inst_state[inst]);
            if (A.serve && ld_relaxed(&A.inst_cancel[inst])) is |= INST_STOP;
            idl = ld_relaxed(&A.ctl->idle);
            h = ld_relaxed(&A.ctl->wl_head);
            t = ld_relaxed(&A.ctl->wl_tail);
            bst = ld_relaxed(&A.reg[scope].best);
        }
        c_done = uni(d);
        c_inst_state = uni(is);
        c_idle = uni(idl);
        c_queued = (int64_t)(uni(t) - uni(h));
        c_best = uni(bst);
        c_best_scope = scope;
        since_poll = 0;
    }

    // the current scope's Best (cached; read afresh when the scope changed)
    __device__ __forceinline__ int cur_best() {
        if (scope != c_best_scope) {
            c_best = scope_best(scope);
            c_best_scope = scope;
        }
        return c_best;
    }
    __device__ __forceinline__ uint32_t* bitmap(int e) { return A.bitmaps + (size_t)e * A.bm_words; }

    // registry entries are only ever accessed with coherent atomics
    __device__ __forceinline__ void init_entry(int e, int best_or_sum, int live, int up, int cover_size,
                               int nchild, int size, int v, int vnn, uint32_t g_at, int g_nnz) {
        RegEntry* r = &A.reg[e];
        st_relaxed(&r->best, best_or_sum);
        st_relaxed(&r->live, live);
        st_relaxed(&r->up, up);
        st_relaxed(&r->lock, 0);
        st_relaxed(&r->cover_size, cover_size);
        st_relaxed(&r->nchild, nchild);
        st_relaxed(&r->size, size);
        st_relaxed(&r->view, v);
        st_relaxed(&r->vn, vnn);
        st_relaxed(reinterpret_cast<int*>(&r->g_at), (int)g_at);
        st_relaxed(&r->g_nnz, g_nnz);
        st_relaxed(&r->att, 0);
        st_relaxed(&r->unatt, 0);
        st_relaxed(&r->done, 0);
    }

    // ------------------------------------------------------- graph views

    // Make entry v's graph the current view: the root's induced subgraph is
    // read from HBM directly; a component's own subgraph is copied from the
    // arena into the LDS graph cache.
    __device__ __forceinline__ void load_view(int v) {
        if (v == view) return;
        if (v == 0 && !A.batch) {
            // the root's induced subgraph: written before the launch and
            // never changed, so it is copied into the cache with plain
            // loads, eight per lane in flight, when it fits
            vn = A.n;
            const uint32_t words = vn + 1u + A.nnz;
            if (!(A.flags & VC_OPT_NO_ROOT_CACHE) && words <= A.gcache_words) {
                for (uint32_t i0 = 0; i0 < words; i0 += 64u * 8u) {
                    uint32_t x[8];
#pragma unroll
                    for (uint32_t k = 0; k < 8u; ++k) {
                        const uint32_t i = i0 + 64u * k + lane();
                        x[k] = i < words ? (i <= vn ? A.off[i] : A.col[i - vn - 1u]) : 0u;
                    }
#pragma unroll
                    for (uint32_t k = 0; k < 8u; ++k) {
                        const uint32_t i = i0 + 64u * k + lane();
                        if (i < words) G[i] = x[k];
                    }
                }
                wsync();
                vlds = true;
                GC = G + vn + 1u;
                b_views += 4ull * words;
            } else {
                vlds = false;
                goff = A.off;
                gcol = A.col;
            }
        } else {
            const uint32_t g_at = (uint32_t)reg_field(reinterpret_cast<const int*>(&A.reg[v].g_at));
            const uint32_t n = (uint32_t)reg_field(&A.reg[v].vn);
            const uint32_t nnz = (uint32_t)reg_field(&A.reg[v].g_nnz);
            const uint32_t* src = A.arena + g_at;
            const uint32_t words = n + 1u + nnz;
            if (words <= A.gcache_words) {
                for (uint32_t i = lane(); i < words; i += 64) G[i] = ld_coh(&src[i]);
                wsync();
                vlds = true;
                GC = G + n + 1u;
                b_views += 4ull * words;
            } else {
                // an instance graph of a batch too large for the cache: read
                // in place (written before the search started)
                vlds = false;
                goff = src;
                gcol = src + n + 1u;
            }
            vn = n;
        }
        vpad = (vn + 63u) & ~63u;
        vbw = vpad / 32u;
        view = v;
    }

    // (a served instance's graph is written while the kernel runs, so it is
    // read with coherent loads)
    __device__ __forceinline__ uint32_t vo(uint32_t v) const {
        return vlds ? G[v] : (A.serve ? ld_coh(&goff[v]) : goff[v]);
    }
    __device__ __forceinline__ uint32_t vc(uint32_t e) const {
        return vlds ? GC[e] : (A.serve ? ld_coh(&gcol[e]) : gcol[e]);
    }

    // vertex count of view vw
    __device__ __forceinline__ uint32_t view_n(int vw) {
        return (vw == 0 && !A.batch) ? A.n : (uint32_t)reg_field(&A.reg[vw].vn);
    }

    // ------------------------------------------------------- live list

    // L = the live vertices of the view, in id order
    __device__ __forceinline__ void build_live() {
        const uint32_t l = lane();
        uint32_t cnt = 0;
        for (uint32_t base = 0; base < vn; base += 64) {
            const uint32_t v = base + l;
            const bool lv = v < vn && DG::live(DG::get(deg, v));
            const uint64_t m = ballot(lv);
            if (lv) L[cnt + mbcnt(m)] = v;
            cnt += popc(m);
        }
        nl = cnt;
        wsync();
    }

    // drop the vertices of L that are no longer live (order kept)
    __device__ __forceinline__ void recompact() {
        if (A.flags & VC_OPT_NO_COMPACT) {
            build_live();  // ablation: a sweep of the whole degree array
            return;
        }
        const uint32_t l = lane();
        uint32_t cnt = 0;
        for (uint32_t base = 0; base < nl; base += 64) {
            const uint32_t i = base + l;
            const uint32_t v = i < nl ? L[i] : 0u;
            const bool lv = i < nl && DG::live(DG::get(deg, v));
            const uint64_t m = ballot(lv);
            wsync();  // every lane has read its entry before any moves
            if (lv) L[cnt + mbcnt(m)] = v;
            cnt += popc(m);
        }
        nl = cnt;
        wsync();
    }

    // Put the vertices of list[0..cnt) into the cover (duplicates allowed):
    // mark them, then remove their edges.  Returns how many were new.
    __device__ __forceinline__ uint32_t take_list(uint32_t* list, uint32_t cnt) {
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
        wsync();
        const uint32_t ent =
            for_rows([&](uint32_t x) { return vo(x); }, [&](uint32_t e) { return vc(e); }, list, nn,
                     MK, [&](bool ok, uint32_t, uint32_t w) {
                         if (ok && DG::live(DG::get(deg, w))) DG::dec(deg, w);
                     });
        // the rows (and their offsets) came from a view in HBM
        if (!vlds) b_rows += 4ull * ent + 8ull * nn;
        wsync();
        s += (int)nn;
        return nn;
    }

    // ------------------------------------------------------- reduce

    // is w in row u (the shorter of the two rows is scanned, four entries
    // per LDS round trip)
    __device__ __forceinline__ bool adjacent(uint32_t u, uint32_t w) {
        uint32_t a = u, b = w;
        if (vo(w + 1) - vo(w) < vo(u + 1) - vo(u)) {
            a = w;
            b = u;
        }
        const uint32_t end = vo(a + 1);
        for (uint32_t e = vo(a); e < end; e += 4) {
            uint32_t x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = e + k < end ? vc(e + k) : NONE;
            if (x[0] == b || x[1] == b || x[2] == b || x[3] == b) return true;
        }
        return false;
    }

    // the first d (1 or 2) live neighbours of v in row order; returns how
    // many were found
    __device__ __forceinline__ uint32_t live_nbrs(uint32_t v, uint32_t d, uint32_t& u,
                                                  uint32_t& w) {
        const uint32_t end = vo(v + 1);
        uint32_t got = 0;
        u = w = NONE;
        for (uint32_t e = vo(v); got < d && e < end; e += 4) {
            uint32_t x[4];
            bool ok[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ok[k] = e + k < end;
                x[k] = ok[k] ? vc(e + k) : 0u;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) ok[k] = ok[k] && DG::live(DG::get(deg, x[k]));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (ok[k] && got < d) {
                    if (got == 0) u = x[k];
                    else w = x[k];
                    ++got;
                }
            }
        }
        return got;
    }

    // Reduction rules of Sec. II-B to a joint fixpoint.  Applied in parallel
    // in two kinds of rounds: (1) every vertex of degree > best-|S|-1 at
    // once (each is in every cover of size < best); (2) degree-one and
    // degree-two-triangle rules at once, where a degree-one vertex whose
    // neighbour also has degree one defers to the lower id, and of the
    // degree-two vertices of one triangle only the lowest id fires, so the
    // joint effect equals some sequential order.  One sweep over the live
    // list finds the high-degree vertices and, into Q, the vertices of
    // degree one or two; the rules of (2) then run on that compacted list,
    // so every lane of a chunk has a row to walk.  Returns false if pruned.
    __device__ __forceinline__ bool reduce() {
        const uint32_t l = lane();
        bool changed_any = false;
        for (;;) {
            if (s >= best) return false;
            const int64_t b = (int64_t)best - s - 1;
            uint32_t hc = 0, cc = 0;
            uint32_t dsum = 0;  // per lane: at most n/64 degrees of at most n
            uint64_t k = 0;     // max of (degree << 32 | ~id)
            uint32_t vn_next = nl ? L[l < nl ? l : 0] : 0u;
            for (uint32_t base = 0; base < nl; base += 64) {
                const uint32_t i = base + l;
                const uint32_t v = vn_next;
                if (base + 64u < nl) vn_next = L[i + 64u < nl ? i + 64u : base + 64u];
                const uint32_t d = i < nl ? DG::get(deg, v) : 0u;
                const bool hi = i < nl && (int64_t)d > b;
                const bool c12 = i < nl && (d == 1u || d == 2u);
                const uint64_t mh = ballot(hi);
                const uint64_t mc = ballot(c12);
                if (hi) R[hc + mbcnt(mh)] = v;
                if (c12) Q[cc + mbcnt(mc)] = v;
                hc += popc(mh);
                cc += popc(mc);
                if (i < nl) {
                    dsum += d;
                    const uint64_t kk = ((uint64_t)d << 32) | (uint32_t)~v;
                    k = kk > k ? kk : k;
                }
            }
            wsync();
            // 2|E| and the branching key of the current live set (final
            // once a round applies no rule)
            e2 = wave_sum(dsum);
            key = wave_max64(k);
            // (1) high degree first
            if (hc) {
                take_list(R, hc);
                recompact();
                changed_any = true;
                continue;
            }
            // (2) degree one / degree-two triangle, over the candidates
            uint32_t cnt = 0;
            for (uint32_t base = 0; base < cc; base += 64) {
                const uint32_t i = base + l;
                const uint32_t v = i < cc ? Q[i] : 0u;
                const uint32_t d = i < cc ? DG::get(deg, v) : 0u;
                uint32_t u = NONE, w = NONE;
                bool add_u = false, add_w = false;
                if (i < cc && live_nbrs(v, d, u, w) == d) {
                    // (fewer than d live neighbours would mean an inconsistent
                    // input, not a simple symmetric graph: no rule then)
                    if (d == 1u) {
                        add_u = !(DG::get(deg, u) == 1u && u < v);
                    } else if (adjacent(u, w)) {
                        add_u = !(DG::get(deg, u) == 2u && u < v) &&
                                !(DG::get(deg, w) == 2u && w < v);
                        add_w = add_u;
                    }
                }
                const uint64_t m1 = ballot(add_u);
                if (add_u) R[cnt + mbcnt(m1)] = u;
                cnt += popc(m1);
                const uint64_t m2 = ballot(add_w);
                if (add_w) R[cnt + mbcnt(m2)] = w;
                cnt += popc(m2);
            }
            wsync();
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
    __device__ __forceinline__ uint32_t find_components() {
        const uint32_t l = lane();
        for (uint32_t i = l; i < vbw; i += 64) {
            VB[i] = 0u;
            PB[i] = 0u;
        }
        wsync();
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
            wsync();
            uint32_t fa = qn - 1, fb = qn, level = 0;
            while (fa < fb) {
                const bool odd = ((level + 1u) & 1u) != 0u;
                for_rows([&](uint32_t x) { return vo(x); }, [&](uint32_t e) { return vc(e); },
                         Q + fa, fb - fa, MK, [&](bool ok, uint32_t, uint32_t w) {
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
                wsync();
                fa = fb;
                fb = qn;
                ++level;
                if (nc == 1 && qn == nl) break;  // one component: stop early
            }
        }
        R[nc] = qn;
        wsync();
        return nc;
    }

    // ------------------------------------------------------- node I/O

    // Write a slot: header, degree array src (npad elements of view vw) and
    // trailer.  Worklist slots (coh) use coherent stores; private stack
    // slots are written and read by this worker only and use plain stores.
    __device__ __forceinline__ void write_slot(uint8_t* slot, int ss, int sc, uint32_t bv, uint32_t live,
                               uint32_t stamp, const D* src, int vw, uint32_t npad, bool coh,
                               uint32_t carried = 1u) {
        const uint32_t l = lane();
        uint32_t hw = 0;  // header word l (8 words)
        if (l == 0) hw = (uint32_t)ss;
        if (l == 1) hw = (uint32_t)sc;
        if (l == 2) hw = bv;
        if (l == 3) hw = live;
        if (l == 4) hw = stamp;
        if (l == 5) hw = (uint32_t)vw;
        if (l == 6) hw = inst;
        if (l == 7) hw = carried;
        uint32_t* h = reinterpret_cast<uint32_t*>(slot);
        uint32_t* tr = reinterpret_cast<uint32_t*>(slot + A.slot_bytes - 16u);
        const uint32_t nw = (npad * (uint32_t)sizeof(D)) / 8u;
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(src);
        uint64_t* d8 = reinterpret_cast<uint64_t*>(slot + sizeof(SlotHdr));
        b_nodes += 8ull * nw + sizeof(SlotHdr) + 16u;
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

    // copy a private-stack node into LDS; returns its pending branch vertex
    __device__ __forceinline__ uint32_t copy_slot(const uint8_t* slot) {
        const uint32_t l = lane();
        const uint32_t* h = reinterpret_cast<const uint32_t*>(slot);
        uint32_t hw = l < 8 ? h[l] : 0u;
        s = uni((int)shfl(hw, 0));
        scope = uni((int)shfl(hw, 1));
        const uint32_t bv = uni(shfl(hw, 2));
        induce_first = (uni(shfl(hw, 7)) & SLOT_INDUCE) != 0u;
        set_inst(uni(shfl(hw, 6)));
        load_view(uni((int)shfl(hw, 5)));
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(slot + sizeof(SlotHdr));
        uint64_t* d8 = reinterpret_cast<uint64_t*>(deg);
        const uint32_t nw = (vpad * (uint32_t)sizeof(D)) / 8u;
        for (uint32_t i = l; i < nw; i += 64) d8[i] = s8[i];
        wsync();
        return bv;
    }

    // Copy the worklist node published for position `want` into LDS with
    // coherent loads.  Returns false, having changed nothing, when the
    // header or trailer still carries another stamp (an old copy of the
    // slot) or names an entry out of range; the pending branch vertex goes
    // to bv.
    __device__ __forceinline__ bool copy_slot_coh(const uint8_t* slot, uint32_t want, uint32_t& bv) {
        const uint32_t l = lane();
        const uint32_t* h = reinterpret_cast<const uint32_t*>(slot);
        const uint32_t* tr = reinterpret_cast<const uint32_t*>(slot + A.slot_bytes - 16u);
        uint32_t hw = l < 8 ? ld_coh(&h[l]) : 0u;
        uint32_t t0 = l == 0 ? ld_coh(&tr[0]) : 0u;
        const uint32_t st0 = uni(shfl(hw, 4));
        const uint32_t st1 = uni(shfl(t0, 0));
        const uint32_t sc = uni(shfl(hw, 1));
        const uint32_t vw = uni(shfl(hw, 5));
        const uint32_t ins = uni(shfl(hw, 6));
        if (st0 != want || st1 != want || sc >= A.reg_cap || vw >= A.reg_cap ||
            (A.batch && ins >= A.n_roots))
            return false;
        s = uni((int)shfl(hw, 0));
        scope = (int)sc;
        bv = uni(shfl(hw, 2));
        induce_first = (uni(shfl(hw, 7)) & SLOT_INDUCE) != 0u;
        set_inst(ins);
        load_view((int)vw);
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(slot + sizeof(SlotHdr));
        uint64_t* d8 = reinterpret_cast<uint64_t*>(deg);
        const uint32_t nw = (vpad * (uint32_t)sizeof(D)) / 8u;
        for (uint32_t i = l; i < nw; i += 64) d8[i] = ld_coh64(&s8[i]);
        wsync();
        return true;
    }

    // start on a node copied into LDS: live list, then the pending N(v); the
    // first node of a component child registered without its own subgraph
    // induces it here (so the children of one branch are induced by the
    // workers that take them, in parallel)
    __device__ __forceinline__ void begin_node(uint32_t bv) {
        build_live();
        known_connected = false;
        small_off = false;
        if (induce_first) {
            induce_first = false;
            adopt_component_view();
            known_connected = true;  // a component, as registered
        }
        if (bv != NONE) take_neighbours(bv);
    }

    // The node holds exactly its scope's component, in the ids of the view
    // it was found in.  Induce the component as a subgraph of its own (local
    // ids = positions in a breadth-first order), make it the entry's view, rewrite
    // the entry's initial cover in local ids (under its lock: a parent may be
    // reading the children's covers), and move the degree array to local ids.
    __device__ __forceinline__ void adopt_component_view() {
        if (is_root(scope)) return;  // a root's view is fixed before the launch
        const uint32_t l = lane();
        const uint32_t size = nl;
        uint32_t dsum = 0;
        for (uint32_t i = l; i < size; i += 64) dsum += DG::get(deg, L[i]);
        const uint32_t nnz = wave_sum(dsum);
        if (size < 2u || size + 1u + nnz > A.gcache_words || size >= vn) return;
        // local ids in breadth-first order from the component's lowest id,
        // the order a child induced at registration gets (Q)
        if (find_components() != 1u) return;
        const int e = scope;
        lock(e);
        const uint32_t g_at = induce_component(0, size, nnz, R + A.n_pad + 64u, L);
        if (g_at != NONE) {
            const int cs = reg_field(&A.reg[e].cover_size);
            if (cs == (int)size - 1) {
                uint32_t* bm = bitmap(e);
                const uint32_t w = (size + 31u) / 32u;
                for (uint32_t i = l; i < w; i += 64) {
                    uint32_t bits = ~0u;
                    if (i == w - 1u && (size & 31u)) bits = (1u << (size & 31u)) - 1u;
                    if (i == 0) bits &= ~1u;  // all but local vertex 0
                    st_coh(&bm[i], bits);
                }
            }
            if (l == 0) {
                st_relaxed(&A.reg[e].view, e);
                st_relaxed(&A.reg[e].vn, (int)size);
                st_relaxed(reinterpret_cast<int*>(&A.reg[e].g_at), (int)g_at);
                st_relaxed(&A.reg[e].g_nnz, (int)nnz);
            }
            ++lviews;
        }
        unlock(e);
        if (g_at == NONE) {
            build_live();  // L was the induction's scratch
            return;
        }
        // degrees in local ids: position i of Q
        const uint32_t cpad = (size + 63u) & ~63u;
        D* cd = reinterpret_cast<D*>(R);
        for (uint32_t i = l; i < cpad; i += 64) DG::set(cd, i, i < size ? DG::get(deg, Q[i]) : 0u);
        wsync();
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(cd);
        uint64_t* d8 = reinterpret_cast<uint64_t*>(deg);
        for (uint32_t i = l; i < (cpad * (uint32_t)sizeof(D)) / 8u; i += 64) d8[i] = s8[i];
        wsync();
        load_view(e);
        build_live();
    }

    // the N(v) branch: every live neighbour of v goes into the cover
    __device__ __forceinline__ void take_neighbours(uint32_t v) {
        const uint32_t l = lane();
        uint32_t cnt = 0;
        const uint32_t r0 = vo(v), r1 = vo(v + 1);
        for (uint32_t e0 = r0; e0 < r1; e0 += 64) {
            uint32_t e = e0 + l;
            uint32_t w = e < r1 ? vc(e) : 0u;
            bool lv = e < r1 && DG::live(DG::get(deg, w));
            uint64_t m = ballot(lv);
            if (lv) R[cnt + mbcnt(m)] = w;
            cnt += popc(m);
        }
        wsync();
        take_list(R, cnt);
        recompact();
    }

    // ------------------------------------------------------- worklist

    __device__ __forceinline__ void publish_order() {
        if (A.strong_fences) fence_release();
        order_point();
    }

    // idle workers outnumber queued nodes (by the last poll)
    __device__ __forceinline__ bool others_hungry() {
        if (A.flags & VC_OPT_NO_LOAD_BALANCE) return false;
        return c_idle > 0 && (int64_t)c_idle > c_queued + (int64_t)A.donate_slack;
    }

    // reserve a worklist position (UINT64_MAX when full)
    __device__ __forceinline__ uint64_t wl_reserve() {
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

    __device__ __forceinline__ void wl_publish(uint64_t pos) {
        ++c_queued;  // until the next poll
        wsync();
        if (lane() == 0) {
            add_relaxed(&A.ctl->outstanding, 1);
            publish_order();
            __hip_atomic_store(&A.wl_seq[pos % A.wl_cap], pos + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        ++dons;
    }

    // take one node from the worklist into LDS; false if it looked empty
    __device__ __forceinline__ bool wl_take() {
        uint64_t res = ~0ull;
        if (lane() == 0) {
            const uint64_t cap = A.wl_cap;
            uint64_t pos = ld_relaxed(&A.ctl->wl_head);
            for (int tries = 0; tries < 64; ++tries) {
                uint64_t seq = ld_relaxed(&A.wl_seq[pos % cap]);
                int64_t diff = (int64_t)(seq - (pos + 1));
                if (diff == 0) {
                    if (cas_relaxed64(&A.ctl->wl_head, pos, pos + 1)) {
                        if (A.strong_fences) fence_acquire();
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
        wsync();
        const uint8_t* slot = A.wl_slots + (size_t)(res % A.wl_cap) * A.slot_bytes;
        const uint32_t want = (uint32_t)res;
        uint32_t bv = NONE;
        bool fresh = copy_slot_coh(slot, want, bv);
        for (uint32_t tries = 0; !fresh && tries < 100000; ++tries) {
            // an old copy of the slot was read: count it and read again
            if (lane() == 0) {
                if (tries == 0) add_relaxed(&A.ctl->stale, 1ull);
                fence_acquire();
            }
            wsync();
            fresh = copy_slot_coh(slot, want, bv);
        }
        if (!fresh) {
            // the published node never became visible: stop the search
            // (the slot stays taken, so nothing else reads it)
            fail(VC_EDEVICE, FAIL_STALE_SLOT);
            return true;
        }
        if (lane() == 0) {
            order_point();
            __hip_atomic_store(&A.wl_seq[res % A.wl_cap], res + A.wl_cap, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        begin_node(bv);
        return true;
    }

    // Place a pending node with `live` live vertices: the shared worklist
    // when others are idle, else the own stack; fill(slot, stamp, coherent)
    // writes it.
    template <typename Fill>
    __device__ __forceinline__ bool push_node(uint32_t live, Fill&& fill) {
        ++pushes;
        // the threshold applies to what would be donated: the oldest
        // pending node when there is one, else this one
        bool give = false;
        if (others_hungry()) {
            uint32_t cand = live;
            if (top > bot) {
                uint32_t nlv = 0;
                if (lane() == 0)
                    nlv = reinterpret_cast<const SlotHdr*>(stack + (size_t)bot * A.slot_bytes)->nlive;
                cand = uni(nlv);
            }
            give = cand >= A.donate_min;
        }
        if (give) {
            // give away the oldest pending node (it roots the largest subtree)
            // when there is one, else this one
            uint64_t pos = wl_reserve();
            if (pos != ~0ull) {
                uint8_t* dst = A.wl_slots + (size_t)(pos % A.wl_cap) * A.slot_bytes;
                if (top > bot) {
                    donate_bottom(dst, (uint32_t)pos);
                    wl_publish(pos);
                } else {
                    fill(dst, (uint32_t)pos, true);
                    wl_publish(pos);
                    return true;
                }
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
        fail(VC_ENOMEM, FAIL_ARENA);
        return false;
    }

    // move the bottom entry of the private stack into worklist slot dst
    __device__ __forceinline__ void donate_bottom(uint8_t* dst, uint32_t stamp) {
        const uint32_t l = lane();
        const uint8_t* src = stack + (size_t)bot * A.slot_bytes;
        const uint32_t* h = reinterpret_cast<const uint32_t*>(src);
        uint32_t hw = l < 8 ? h[l] : 0u;
        if (l == 4) hw = stamp;
        const uint32_t vw = uni(shfl(hw, 5));
        // a node leaving the worker takes a count of its own (nodes in the
        // worklist always carry one)
        const int bsc = (int)uni(shfl(hw, 1));
        if ((uni(shfl(hw, 7)) & SLOT_COUNTED) == 0u && counted(bsc) && l == 0)
            add_relaxed(&A.reg[bsc].live, 1);
        if (l == 7) hw |= SLOT_COUNTED;
        // the entry's view decides how much of the degree array is in use
        const uint32_t n = view_n((int)vw);
        const uint32_t npad = (n + 63u) & ~63u;
        const uint32_t nw = (npad * (uint32_t)sizeof(D)) / 8u;
        uint32_t* dh = reinterpret_cast<uint32_t*>(dst);
        uint32_t* tr = reinterpret_cast<uint32_t*>(dst + A.slot_bytes - 16u);
        if (l < 8) st_coh(&dh[l], hw);
        if (l < 4) st_coh(&tr[l], l == 0 ? stamp : 0u);
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(src + sizeof(SlotHdr));
        uint64_t* d8 = reinterpret_cast<uint64_t*>(dst + sizeof(SlotHdr));
        for (uint32_t i = l; i < nw; i += 64) st_coh64(&d8[i], s8[i]);
        b_nodes += 8ull * nw + sizeof(SlotHdr) + 16u;
        ++bot;
        if (bot == top) bot = top = 0;
    }

    __device__ __forceinline__ void fail(int code, int site) {
        if (lane() == 0) {
            if (atomicCAS(&A.ctl->err, 0, code) == 0) st_relaxed(&A.ctl->err_site, site);
            st_relaxed(&A.ctl->done, 1);
        }
    }

    // ------------------------------------------------------- covers

    __device__ __forceinline__ void lock(int e) {
        if (lane() == 0) {
            uint32_t spins = 0;
            while (!cas_acquire(&A.reg[e].lock, 0, 1)) backoff(spins);
        }
        wsync();
    }
    __device__ __forceinline__ void unlock(int e) {
        wsync();
        if (lane() == 0) {
            publish_order();
            st_relaxed(&A.reg[e].lock, 0);
        }
    }

    // the IN marks of the LDS degree array as bitmap words (current view)
    __device__ __forceinline__ void write_in_bitmap(uint32_t* bm) {
        const uint32_t l = lane();
        for (uint32_t wi = l; wi < vbw; wi += 64) {
            uint32_t bits = 0;
            const uint32_t v0 = wi * 32u;
            for (uint32_t j = 0; j < 32u; ++j) {
                uint32_t v = v0 + j;
                if (v < vn && DG::get(deg, v) == DG::IN) bits |= 1u << j;
            }
            st_coh(&bm[wi], bits);
        }
    }

    // Offer `val` as a new Best of scope entry e.  The cover is the LDS
    // state (from < 0), or is assembled from parent entry `from` and its
    // children, mapping children with their own view back through their
    // local-to-parent id maps.  Returns true if the cover was written.
    __device__ __forceinline__ bool improve(int e, int val, int from) {
        int prev_cs = INF;
        const bool wrote = improve_once(e, val, from, &prev_cs);
        // PVC (Sec. III-E): a component's better cover travels up the
        // registry chain at once, so the root learns when it is within k
        if (wrote && pvc_now() && !is_root(e)) propagate_up(e, prev_cs, val);
        return wrote;
    }

    // Child entry c's attained cover went from old (INF: none) to val.  Its
    // parent keeps Sum plus the children's attained covers (att) and the
    // number of children still without one (unatt); when none is missing,
    // that total is an attained cover of the parent node and is offered to
    // the ancestor, and so on up to the root.  Partial totals can only be
    // too large (every change is a decrease), never too small.
    __device__ __forceinline__ void propagate_up(int c, int old, int val) {
        for (;;) {
            const int p = reg_field(&A.reg[c].up);
            int u = 0;
            if (lane() == 0) {
                if (old >= INF) {
                    add_relaxed(&A.reg[p].att, val);
                    order_point();
                    u = add_relaxed(&A.reg[p].unatt, -1) - 1;
                } else {
                    add_relaxed(&A.reg[p].att, val - old);
                    order_point();
                    u = ld_relaxed(&A.reg[p].unatt);
                }
            }
            u = uni(u);
            if (u != 0) return;
            const int total = reg_field(&A.reg[p].att);
            const int a = reg_field(&A.reg[p].up);
            int prev = INF;
            if (!improve_once(a, total, p, &prev)) return;
            if (is_root(a)) return;
            c = a;
            old = prev;
            val = total;
        }
    }

    __device__ __forceinline__ bool improve_once(int e, int val, int from, int* prev_cs) {
        const bool pvc = pvc_now();
        int old = 0;
        if (lane() == 0) old = min_relaxed(&A.reg[e].best, val);
        old = uni(old);
        if (e == c_best_scope) c_best = old < val ? old : val;
        if (val >= old) return false;
        lock(e);
        const int cs = reg_field(&A.reg[e].cover_size);
        *prev_cs = cs;
        bool wrote = false;
        if (val < cs) {
            uint32_t* dst = bitmap(e);
            if (from < 0) {
                write_in_bitmap(dst);
            } else {
                const uint32_t l = lane();
                const uint32_t ebw = ((uint32_t)reg_field(&A.reg[e].vn) + 31u) / 32u;
                const int nch = reg_field(&A.reg[from].nchild);
                for (uint32_t wi = l; wi < ebw; wi += 64) VB[wi] = ld_coh(&bitmap(from)[wi]);
                wsync();
                for (int c = from + 1; c <= from + nch; ++c) {
                    // in PVC the children may still be improving: read each
                    // child's cover under its lock (ancestor locks are always
                    // taken before descendant locks)
                    if (pvc) lock(c);
                    const int cv = reg_field(&A.reg[c].view);
                    if (cv == c) {
                        const uint32_t cn = (uint32_t)reg_field(&A.reg[c].vn);
                        const uint32_t g_at =
                            (uint32_t)reg_field(reinterpret_cast<const int*>(&A.reg[c].g_at));
                        const uint32_t nnz = (uint32_t)reg_field(&A.reg[c].g_nnz);
                        const uint32_t* l2g = A.arena + g_at + cn + 1u + nnz;
                        const uint32_t* cb = bitmap(c);
                        for (uint32_t i = l; i < cn; i += 64) {
                            if ((ld_coh(&cb[i >> 5]) >> (i & 31u)) & 1u) {
                                uint32_t w = ld_coh(&l2g[i]);
                                atomicOr(&VB[w >> 5], 1u << (w & 31u));
                            }
                        }
                    } else {
                        for (uint32_t wi = l; wi < ebw; wi += 64) {
                            uint32_t x = ld_coh(&bitmap(c)[wi]);
                            if (x) atomicOr(&VB[wi], x);
                        }
                    }
                    wsync();
                    if (pvc) unlock(c);
                }
                for (uint32_t wi = l; wi < ebw; wi += 64) st_coh(&dst[wi], VB[wi]);
            }
            wsync();
            if (lane() == 0) st_relaxed(&A.reg[e].cover_size, val);
            b_reg += 4ull * vbw;
            wrote = true;
        }
        unlock(e);
        if (is_root(e) && pvc_now() && val <= (A.batch ? A.inst_k[e] : A.k) && lane() == 0) {
            if (A.batch)
                __hip_atomic_fetch_or(&A.inst_state[e], INST_STOP, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            else
                st_relaxed(&A.ctl->done, 1);
        }
        return wrote;
    }

    // A node of scope e has finished.  Walk the registry chain: the last
    // descendant of a component adds its Best to the parent's Sum; the last
    // component of a parent offers Sum to the ancestor's Best and finishes
    // the parent node in the ancestor's scope (Sec. III-C).
    // PVC semantics for the current node: the solve's, or when serving the
    // instance's (a served MVC request has no bound k: inst_k < 0)
    __device__ __forceinline__ bool pvc_now() {
        if (!A.serve) return A.pvc != 0;
        int kk = -1;
        if (lane() == 0) kk = ld_relaxed(&A.inst_k[inst]);
        return uni(kk) >= 0;
    }

    // Live-node counts are kept for every scope except the root of a single
    // solve (its end is the end of the search).
    __device__ __forceinline__ bool counted(int e) { return A.batch || e != 0; }
    __device__ __forceinline__ bool is_root(int e) { return e < (int)A.n_roots; }

    // LiveNodes (Sec. III-C) counts the nodes of a scope, but a worker keeps
    // the count of a chain of its own nodes as one: a child pushed on the
    // private stack carries no count (header word 7 = 0) while the node that
    // pushed it runs, and when a counted node of scope e finishes with an
    // uncounted node of scope e on top of its stack, the count passes to
    // that node instead of being decremented.  A node that leaves the worker
    // (donation, the worklist) takes a count of its own, and so does the top
    // uncounted node when the current node stops being in scope e (a branch
    // on components).  So the counter is zero exactly when no node of the
    // scope is left, with atomics only where work crosses workers or scopes.
    __device__ __forceinline__ uint32_t count_child(int sc, bool leaves) {
        if (!counted(sc)) return 1u;
        if (!leaves) return 0u;
        if (lane() == 0) add_relaxed(&A.reg[sc].live, 1);
        return 1u;
    }

    // the top slot of the private stack, if it is an uncounted node of scope
    // e (its header), else null
    __device__ __forceinline__ uint32_t* uncounted_top(int e) {
        if (top <= bot) return nullptr;
        uint32_t* h = reinterpret_cast<uint32_t*>(stack + (size_t)(top - 1u) * A.slot_bytes);
        uint32_t sc = 0, ca = SLOT_COUNTED;
        if (lane() == 0) {
            sc = h[1];
            ca = h[7];
        }
        return ((int)uni(sc) == e && (uni(ca) & SLOT_COUNTED) == 0u) ? h : nullptr;
    }

    // the current node (scope e) goes on in another scope: the uncounted
    // node it would have handed its count to gets one of its own
    __device__ __forceinline__ void settle_count(int e) {
        if (!counted(e)) return;
        uint32_t* h = uncounted_top(e);
        if (!h) return;
        if (lane() == 0) {
            add_relaxed(&A.reg[e].live, 1);
            h[7] |= SLOT_COUNTED;
        }
        wsync();
    }

    __device__ __forceinline__ void complete(int e) {
        if (counted(e)) {
            uint32_t* h = uncounted_top(e);
            if (h) {
                if (lane() == 0) h[7] |= SLOT_COUNTED;  // the count passes down the stack
                wsync();
                return;
            }
        }
        for (;;) {
            if (is_root(e)) {
                if (A.batch) {
                    // the last node of an instance: its result is final
                    int old = 0;
                    if (lane() == 0) {
                        old = add_relaxed(&A.reg[e].live, -1);
                        if (old == 1) {
                            order_point();
                            __hip_atomic_fetch_or(&A.inst_state[e], INST_FIN, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
                return;
            }
            int old = 0;
            if (lane() == 0) old = add_relaxed(&A.reg[e].live, -1);
            old = uni(old);
            if (old != 1) return;
            const bool audit = (A.flags & VC_OPT_CHECK_REGISTRY) != 0;
            if (lane() == 0 && A.strong_fences) fence_acquire();
            if (lane() == 0 && audit) add_relaxed(&A.reg[e].done, 1);
            const int p = reg_field(&A.reg[e].up);
            const int cb = reg_field(&A.reg[e].best);
            if (lane() == 0) {
                add_relaxed(&A.reg[p].best, cb);
                publish_order();  // the Sum update lands before LiveComps moves
                old = add_relaxed(&A.reg[p].live, -1);
            }
            old = uni(old);
            if (old != 1) return;
            if (lane() == 0 && A.strong_fences) fence_acquire();
            if (lane() == 0 && audit) add_relaxed(&A.reg[p].done, 1);
            wsync();
            const int sum = reg_field(&A.reg[p].best);
            const int a = reg_field(&A.reg[p].up);
            improve(a, sum, p);
            e = a;
        }
    }

    // ------------------------------------------------------- node handling

    // batches: add the current instance's pending node count to its total
    // and stop the instance once it is over its limit
    __device__ __forceinline__ void flush_inst() {
        if (!A.batch || inst_cnt == 0) return;
        if (lane() == 0 && inst < A.n_roots) {
            const uint64_t tot =
                __hip_atomic_fetch_add(&A.inst_nodes[inst], inst_cnt, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) + inst_cnt;
            if (A.inst_node_limit && tot > A.inst_node_limit)
                __hip_atomic_fetch_or(&A.inst_state[inst], INST_STOP | INST_LIMIT,
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        inst_cnt = 0;
    }

    __device__ __forceinline__ void set_inst(uint32_t i) {
        if (i == inst) return;
        flush_inst();
        inst = i;
        since_poll = POLL_EVERY;  // the cached instance state is another's
    }

    __device__ __forceinline__ void count_node() {
        ++nodes;
        if (A.batch && ++inst_cnt >= 64) flush_inst();
        if (A.node_limit && nodes - nodes_flushed >= 256) {
            uint64_t tot = 0;
            if (lane() == 0) tot = add_relaxed(&A.ctl->nodes, nodes - nodes_flushed);
            tot = uni(tot) + (nodes - nodes_flushed);
            nodes_flushed = nodes;
            if (tot > A.node_limit) fail(VC_ETIMEDOUT, FAIL_NODE_LIMIT);
        }
    }

    // 0: go on; 1: the whole search stops; 2: the node's instance has its
    // answer or is over its limit, so the node is dropped
    enum { GO = 0, STOP_ALL = 1, DROP = 2 };
    __device__ __forceinline__ int stop_requested(bool force) {
        if (force || ++since_poll >= POLL_EVERY) poll();
        if (c_done != 0) return STOP_ALL;
        return (c_inst_state & INST_STOP) ? DROP : GO;
    }

    // vertex branch on v_max: the G - N(v) child is pushed (lazily, as the
    // current state plus v), the G - v child continues here
    __device__ __forceinline__ bool vertex_branch() {
        const uint32_t v = ~(uint32_t)(key & 0xFFFFFFFFull);
        const int ss = s, sc = scope;
        if (!push_node(nl, [&](uint8_t* slot, uint32_t stamp, bool coh) {
                write_slot(slot, ss, sc, v, nl, stamp, deg, view, vpad, coh, count_child(sc, coh));
            }))
            return false;
        if (lane() == 0) R[0] = v;
        wsync();
        take_list(R, 1);
        recompact();
        known_connected = false;  // removing v may split the graph
        return true;
    }

    // Classify the components found: cliques and chordless cycles are
    // solved on the spot (Sec. III-D); the others are listed in
    // R[nc+1 ..].  Returns the number of other components.
    __device__ __forceinline__ uint32_t settle_simple_components(uint32_t nc) {
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
            wsync();
        }
        return nt;
    }

    // Induce component Q[a..b) as a subgraph of its own in the arena:
    // off[size+1], col[nnz] (local ids = positions in Q), l2g[size] (ids of
    // the current view).  M is an id map scratch of vn words, CUR one of
    // size words.  Returns the arena word offset, or NONE if it is full.
    __device__ __forceinline__ uint32_t induce_component(uint32_t a, uint32_t b, uint32_t nnz, uint32_t* M,
                                         uint32_t* CUR) {
        const uint32_t l = lane();
        const uint32_t size = b - a;
        const uint32_t words = (size + 1u + nnz + size + 31u) & ~31u;  // whole lines
        uint64_t at = ~0ull;
        if (l == 0) {
            uint64_t cur = ld_relaxed(&A.ctl->arena_next);
            while (cur + words <= A.arena_words) {
                if (cas_relaxed64(&A.ctl->arena_next, cur, cur + words)) {
                    at = cur;
                    break;
                }
                cur = ld_relaxed(&A.ctl->arena_next);
            }
        }
        at = uni(at);
        if (at == ~0ull || at >= 0xFFFFFFFFull) return NONE;
        uint32_t* g = A.arena + at;
        b_reg += 4ull * (size + 1u + nnz + size);
        for (uint32_t i = a + l; i < b; i += 64) M[Q[i]] = i - a;
        // offsets: prefix sums of the live degrees, in Q order
        uint32_t carry = 0;
        for (uint32_t base = 0; base < size; base += 64) {
            uint32_t i = base + l;
            uint32_t d = i < size ? DG::get(deg, Q[a + i]) : 0u;
            uint32_t incl = wave_incl_scan(d);
            if (i < size) {
                CUR[i] = carry + incl - d;
                st_coh(&g[i], carry + incl - d);
                st_coh(&g[size + 1u + nnz + i], Q[a + i]);
            }
            carry += shfl(incl, 63);
        }
        if (l == 0) st_coh(&g[size], carry);
        wsync();
        // columns: the component's rows spread over the lanes (for_rows);
        // each live entry takes the next place of its row (CUR: row cursors,
        // so the order inside a row is arbitrary)
        uint32_t* gc = g + size + 1u;
        for_rows([&](uint32_t x) { return vo(x); }, [&](uint32_t e) { return vc(e); }, Q + a, size,
                 MK, [&](bool ok, uint32_t x, uint32_t w) {
                     if (ok && DG::live(DG::get(deg, w))) {
                         const uint32_t pos = __hip_atomic_fetch_add(
                             &CUR[M[x]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                         st_coh(&gc[pos], M[w]);
                     }
                 });
        wsync();
        return (uint32_t)at;
    }

    // Branch on components (Alg. 2): one parent entry plus one child entry
    // per component, best_i = min(best - sum, |V_i| - 1); children other
    // than the first are pushed, the first continues here.  Returns CB_FULL
    // when the registry is full (the caller then branches on a vertex) and
    // CB_PRUNED when the scope's bound leaves no room for the components.
    enum { CB_OK = 0, CB_FULL = 1, CB_PRUNED = 2 };
    __device__ __forceinline__ int component_branch(uint32_t nc, uint32_t nt) {
        const uint32_t l = lane();
        const uint32_t* NT = R + nc + 1;
        uint32_t* M = R + A.n_pad + 64u;  // id map scratch (n_pad words)
        // the bound may have improved since the node started: every
        // component needs at least one vertex
        const int bnow = scope_best(scope);
        if (scope == c_best_scope) c_best = bnow;
        const int base_sum = s;
        if ((int64_t)base_sum + nt >= (int64_t)bnow) return CB_PRUNED;
        const uint32_t want = (nt + 1u + 1u) & ~1u;  // whole 128-byte lines
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
        settle_count(scope);
        if (l == 0) init_entry((int)p, base_sum, (int)nt, scope, INF, (int)nt, 0, view, (int)vn, 0u, 0);
        write_in_bitmap(bitmap((int)p));
        b_reg += (uint64_t)(nt + 1u) * sizeof(RegEntry) + 4ull * vbw * (nt + 1u);
        // child entries, their graph views and their initial covers (the
        // component minus one vertex: |V_i| - 1 is always attained)
        for (uint32_t j = 0; j < nt; ++j) {
            const uint32_t c = NT[j];
            const uint32_t a = R[c], b = R[c + 1], size = b - a;
            int bi = bnow - base_sum;
            const bool attained = (int)size - 1 <= bi;
            if (attained) bi = (int)size - 1;
            uint32_t dsum = 0;
            for (uint32_t i = a + l; i < b; i += 64) dsum += DG::get(deg, Q[i]);
            const uint32_t nnz = wave_sum(dsum);
            const int e = (int)(p + 1u + j);
            uint32_t g_at = NONE;
            // child 0 continues here and gets its own subgraph now; the
            // others get theirs from the worker that starts them (or now,
            // under VC_OPT_EAGER_INDUCE)
            const bool now = j == 0 || (A.flags & VC_OPT_EAGER_INDUCE);
            if (now && size + 1u + nnz <= A.gcache_words && size < vn)
                g_at = induce_component(a, b, nnz, M, L);
            const bool own = g_at != NONE;
            if (l == 0)
                init_entry(e, bi, 1, (int)p, attained ? (int)size - 1 : INF, 0, (int)size,
                           own ? e : view, own ? (int)size : (int)vn, own ? g_at : 0u,
                           own ? (int)nnz : 0);
            if (attained) {
                uint32_t* bm = bitmap(e);
                if (own) {
                    const uint32_t w = (size + 31u) / 32u;
                    for (uint32_t i = l; i < w; i += 64) {
                        uint32_t bits = ~0u;
                        if (i == w - 1u && (size & 31u)) bits = (1u << (size & 31u)) - 1u;
                        if (i == 0) bits &= ~1u;  // all but local vertex 0
                        st_coh(&bm[i], bits);
                    }
                } else {
                    for (uint32_t i = l; i < vbw; i += 64) VB[i] = 0u;
                    wsync();
                    for (uint32_t i = a + 1u + l; i < b; i += 64) {
                        uint32_t v = Q[i];
                        atomicOr(&VB[v >> 5], 1u << (v & 31u));
                    }
                    wsync();
                    for (uint32_t i = l; i < vbw; i += 64) st_coh(&bm[i], VB[i]);
                }
            }
            if (own) ++lviews;
            if (l == 0) {
                if (attained) add_relaxed(&A.reg[p].att, (int)size - 1);
                else add_relaxed(&A.reg[p].unatt, 1);
            }
            wsync();
        }
        if (l == 0) add_relaxed(&A.reg[p].att, base_sum);
        // entries, covers and graphs are complete before any child can run
        if (l == 0) publish_order();
        cbr += 1;
        {
            // Table III: components per branch, in power-of-two buckets
            // (constant indices only, so the counters stay in registers)
            uint32_t bk = 0;
            while (bk < 7u && (2u << bk) < nt) ++bk;
#pragma unroll
            for (uint32_t i = 0; i < 8u; ++i) chist[i] += i == bk ? 1u : 0u;
        }
        comps += nt;
        // children 1..nt-1 go out as nodes holding only their component,
        // built in L (free until child 0 rebuilds it)
        D* cd = reinterpret_cast<D*>(L);
        for (uint32_t j = nt - 1; j >= 1; --j) {
            const uint32_t c = NT[j];
            const uint32_t a = R[c], b = R[c + 1], size = b - a;
            const int e = (int)(p + 1u + j);
            const bool own = reg_field(&A.reg[e].view) == e;
            const uint32_t cpad = own ? ((size + 63u) & ~63u) : vpad;
            {
                uint4* z = reinterpret_cast<uint4*>(cd);
                const uint32_t nv = (cpad * (uint32_t)sizeof(D)) / 16u;
                for (uint32_t i = l; i < nv; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
                wsync();
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    cd[own ? i - a : v] = (D)DG::get(deg, v);
                }
                wsync();
            }
            const int vw = own ? e : view;
            const uint32_t flags = SLOT_COUNTED | (own ? 0u : SLOT_INDUCE);
            bool ok = push_node(size, [&](uint8_t* slot, uint32_t stamp, bool coh) {
                write_slot(slot, 0, e, NONE, size, stamp, cd, vw, cpad, coh, flags);
            });
            if (!ok) return CB_OK;  // error flagged; the next node stops
        }
        // child 0 continues in LDS: only its component, S restarts
        {
            const uint32_t c = NT[0];
            const uint32_t a = R[c], b = R[c + 1], size = b - a;
            const int e = (int)(p + 1u);
            const bool own = reg_field(&A.reg[e].view) == e;
            if (own) {
                const uint32_t cpad = (size + 63u) & ~63u;
                uint4* z = reinterpret_cast<uint4*>(cd);
                const uint32_t nv = (cpad * (uint32_t)sizeof(D)) / 16u;
                for (uint32_t i = l; i < nv; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
                wsync();
                for (uint32_t i = a + l; i < b; i += 64) cd[i - a] = (D)DG::get(deg, Q[i]);
                wsync();
                const uint64_t* s8 = reinterpret_cast<const uint64_t*>(cd);
                uint64_t* d8 = reinterpret_cast<uint64_t*>(deg);
                for (uint32_t i = l; i < (cpad * (uint32_t)sizeof(D)) / 8u; i += 64) d8[i] = s8[i];
                wsync();
                load_view(e);
            } else {
                for (uint32_t i = l; i < vbw; i += 64) VB[i] = 0u;
                wsync();
                for (uint32_t i = a + l; i < b; i += 64) {
                    uint32_t v = Q[i];
                    atomicOr(&VB[v >> 5], 1u << (v & 31u));
                }
                wsync();
                for (uint32_t v = l; v < vn; v += 64)
                    if (!((VB[v >> 5] >> (v & 31u)) & 1u)) DG::set(deg, v, 0u);
                wsync();
            }
            s = 0;
            scope = e;
            build_live();
            known_connected = true;
        }
        return CB_OK;
    }

    // ------------------------------------------------------- small nodes

    // A node with at most 128 live vertices is solved by the wave in
    // registers: position p of the live list (ids ascending, so position
    // order is id order) belongs to lane p % 64, slot p / 64, and each lane
    // holds its vertices' adjacency among the live ones as masks of W
    // 64-bit words (W = 1 up to 64 live vertices, 2 up to 128).  A node of
    // the subtree is (live mask, taken mask, number taken).  The same rules,
    // stopping tests, component rules and branching vertex as for a general
    // node apply to the whole subtree, depth first with a stack in LDS.  A
    // split into two or more components that are not cliques or cycles
    // returns to the general path, whose component branch goes through the
    // registry (Alg. 2): the pending nodes of the subtree are pushed as
    // ordinary nodes first.
    enum { SMALL_DONE = 0, SMALL_STOP = 1, SMALL_SPLIT = 2 };

    __device__ __forceinline__ static uint32_t popc64(uint64_t x) {
        return (uint32_t)__builtin_popcountll(x);
    }
    __device__ __forceinline__ static uint32_t low64(uint64_t x) {
        return (uint32_t)__builtin_ctzll(x);
    }
    __device__ __forceinline__ static uint32_t high64(uint64_t x) {
        return 63u - (uint32_t)__builtin_clzll(x);
    }
    // bits of word j for the positions below p
    __device__ __forceinline__ static uint64_t below(uint32_t p, uint32_t j) {
        const uint32_t lo = 64u * j;
        if (p >= lo + 64u) return ~0ull;
        if (p <= lo) return 0ull;
        return (1ull << (p - lo)) - 1ull;
    }

    // Offer the small node's cover (entry marks plus the taken positions) as
    // a new Best of the scope: the marks are put into the LDS degree array
    // for the bitmap and taken out again.
    template <int W>
    __device__ __forceinline__ void small_improve(int val, const uint64_t* tin, const bool* mine,
                                                  const uint32_t* vid, const uint32_t* d0) {
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (mine[k] && ((tin[k] >> lane()) & 1ull)) DG::set(deg, vid[k], DG::IN);
        wsync();
        improve(scope, val, -1);
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (mine[k]) DG::set(deg, vid[k], d0[k]);
        wsync();
        if (val < best) best = val;
    }

    // the entry of position (lane, slot k) in a degree array for the node
    // (lv, ti): its live degree, the in-cover mark, or 0
    template <int W>
    __device__ __forceinline__ static uint32_t small_entry(const uint64_t (*adj)[W],
                                                           const uint64_t* lv, const uint64_t* ti,
                                                           int k, uint32_t l) {
        if ((lv[k] >> l) & 1ull) {
            uint32_t d = 0;
#pragma unroll
            for (int j = 0; j < W; ++j) d += popc64(adj[k][j] & lv[j]);
            return d;
        }
        return ((ti[k] >> l) & 1ull) ? DG::IN : 0u;
    }

    // Push a small node (lv, ti, sv taken in scope) as an ordinary node:
    // its degree array is the entry one with the live list's entries
    // replaced.
    // With donate set the node goes straight to the shared worklist (false
    // when it is full); otherwise it is pushed like any child.
    template <int W>
    __device__ __forceinline__ bool small_export(const uint64_t* lv, const uint64_t* ti, int sv,
                                                 const bool* mine, const uint32_t* vid,
                                                 const uint64_t (*adj)[W], bool donate = false) {
        const uint32_t l = lane();
        uint64_t pos = ~0ull;
        if (donate) {
            pos = wl_reserve();
            if (pos == ~0ull) return false;
        }
        D* cd = reinterpret_cast<D*>(Q);
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(deg);
        uint64_t* d8 = reinterpret_cast<uint64_t*>(cd);
        for (uint32_t i = l; i < (vpad * (uint32_t)sizeof(D)) / 8u; i += 64) d8[i] = s8[i];
        wsync();
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (mine[k]) DG::set(cd, vid[k], small_entry<W>(adj, lv, ti, k, l));
        wsync();
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < W; ++j) live += popc64(lv[j]);
        const int ss = sv, sc = scope;
        if (donate) {
            write_slot(A.wl_slots + (size_t)(pos % A.wl_cap) * A.slot_bytes, ss, sc, NONE, live,
                       (uint32_t)pos, cd, view, vpad, true, count_child(sc, true));
            wl_publish(pos);
            return true;
        }
        return push_node(live, [&](uint8_t* slot, uint32_t stamp, bool coh) {
            write_slot(slot, ss, sc, NONE, live, stamp, cd, view, vpad, coh, count_child(sc, coh));
        });
    }

    template <int W>
    __device__ __forceinline__ int small_solve() {
        constexpr uint32_t NV = 64u * W;
        const uint32_t l = lane();
        const uint32_t n0 = nl;
        bool mine[W];
        uint32_t vid[W], d0[W];
        uint32_t* P = R + A.n_pad + 64u;  // view id -> position
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t p = l + 64u * k;
            mine[k] = p < n0;
            vid[k] = mine[k] ? L[p] : 0u;
            d0[k] = mine[k] ? DG::get(deg, vid[k]) : 0u;
            if (mine[k]) P[vid[k]] = p;
        }
        wsync();
        uint64_t adj[W][W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
#pragma unroll
            for (int j = 0; j < W; ++j) adj[k][j] = 0ull;
            if (mine[k]) {
                const uint32_t r1 = vo(vid[k] + 1);
                for (uint32_t e = vo(vid[k]); e < r1; ++e) {
                    const uint32_t w = vc(e);
                    if (DG::live(DG::get(deg, w))) {
                        const uint32_t q = P[w];
                        adj[k][q >> 6] |= 1ull << (q & 63u);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < W; ++j) ADJ[(l + 64u * k) * W + j] = adj[k][j];
        }
        wsync();
        const int s0 = s;
        uint64_t live[W], tin[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            live[j] = below(n0, j);
            tin[j] = 0ull;
        }
        int sl = 0;
        int top = 0, bot = 0;  // pending nodes: a deque, popped at top, given away at bot
        uint32_t since = 0;
        bool first = true;
        for (;;) {
            if (!first) {
                count_node();
                // shared state (stop flags, the scope's Best, idle workers)
                // every 64 nodes, every 16 once the subtree has taken 256;
                // then, while others are idle, the oldest pending node (the
                // largest subtree) goes to the shared worklist (most small
                // subtrees end sooner, and moving them would cost more than
                // solving them)
                ++since;
                if ((since & (since < 256u ? 63u : 15u)) == 0u) {
                    const int sr = stop_requested(true);
                    if (sr == STOP_ALL) return SMALL_STOP;
                    if (sr == DROP) return SMALL_DONE;
                    const int cb = cur_best();
                    if (cb < best) best = cb;
                    if (since >= 256u && top > bot && others_hungry()) {
                        uint64_t pl[W], pt[W];
                        uint32_t nlv = 0;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            pl[j] = SM[(uint32_t)bot * 2u * W + j];
                            pt[j] = SM[(uint32_t)bot * 2u * W + W + j];
                            nlv += popc64(pl[j]);
                        }
                        if (nlv >= A.donate_min &&
                            small_export<W>(pl, pt, s0 + (int)SS[bot], mine, vid, adj, true)) {
                            ++bot;
                            if (bot == top) bot = top = 0;
                        }
                    }
                }
            }
            first = false;
            bool dead = false;
            uint32_t dg[W];
            bool lv[W];
            // rules to a joint fixpoint, as for a general node
            for (;;) {
                const int b = best - s0 - sl - 1;
                if (b < 0) {
                    dead = true;
                    break;
                }
                bool anyhi = false;
                uint64_t hi[W];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    lv[k] = (live[k] >> l) & 1ull;
                    uint32_t d = 0;
#pragma unroll
                    for (int j = 0; j < W; ++j) d += popc64(adj[k][j] & live[j]);
                    dg[k] = lv[k] ? d : 0u;
                    hi[k] = ballot(lv[k] && (int)dg[k] > b);
                    anyhi = anyhi || hi[k] != 0ull;
                }
                if (anyhi) {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        tin[k] |= hi[k];
                        live[k] &= ~hi[k];
                        sl += (int)popc64(hi[k]);
                    }
                    continue;
                }
                uint64_t d1[W], d2[W], F[W], tk[W];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    d1[k] = ballot(lv[k] && dg[k] == 1u);
                    d2[k] = ballot(lv[k] && dg[k] == 2u);
                }
                // a degree-two vertex whose two neighbours are adjacent
                // fires unless a lower degree-two vertex of that triangle does
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    bool fire = false;
                    if (lv[k] && dg[k] == 2u) {
                        const uint32_t p = l + 64u * k;
                        uint32_t u = NONE, w = NONE;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            const uint64_t nb = adj[k][j] & live[j];
                            if (nb) {
                                const uint32_t a0 = 64u * j + low64(nb);
                                const uint32_t a1 = 64u * j + high64(nb);
                                if (u == NONE) {
                                    u = a0;
                                    if (a1 != a0) w = a1;
                                } else {
                                    w = a0;
                                }
                            }
                        }
                        if (w != NONE && ((ADJ[u * W + (w >> 6)] >> (w & 63u)) & 1ull)) {
                            const bool u2 = (d2[u >> 6] >> (u & 63u)) & 1ull;
                            const bool w2 = (d2[w >> 6] >> (w & 63u)) & 1ull;
                            fire = !(u2 && u < p) && !(w2 && w < p);
                        }
                    }
                    F[k] = ballot(fire);
                }
                // taken: a neighbour of a firing degree-two vertex, or the
                // neighbour of a degree-one vertex (of two adjacent degree-one
                // vertices, the higher id is taken)
                bool anytk = false;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    bool take = false;
                    if (lv[k]) {
                        const uint32_t p = l + 64u * k;
                        bool nbF = false, a1any = false, a1low = false;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            const uint64_t nb = adj[k][j] & live[j];
                            const uint64_t a1 = nb & d1[j];
                            nbF = nbF || (nb & F[j]) != 0ull;
                            a1any = a1any || a1 != 0ull;
                            a1low = a1low || (a1 & below(p, j)) != 0ull;
                        }
                        take = nbF || (a1any && (dg[k] != 1u || a1low));
                    }
                    tk[k] = ballot(take);
                    anytk = anytk || tk[k] != 0ull;
                }
                if (anytk) {
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        tin[k] |= tk[k];
                        live[k] &= ~tk[k];
                        sl += (int)popc64(tk[k]);
                    }
                    continue;
                }
                // no edges left: not live
#pragma unroll
                for (int k = 0; k < W; ++k) live[k] &= ~ballot(lv[k] && dg[k] == 0u);
                break;
            }
            if (!dead) {
                const int64_t b = (int64_t)best - s0 - sl - 1;
                uint32_t dsum = 0;
#pragma unroll
                for (int k = 0; k < W; ++k) dsum += dg[k];
                const uint64_t E = wave_sum(dsum) / 2u;
                if (b < 0 || (int64_t)E > b * b) {
                    dead = true;
                } else if (E == 0) {
                    small_improve<W>(s0 + sl, tin, mine, vid, d0);
                    dead = true;
                }
            }
            if (!dead && !(A.flags & VC_OPT_NO_COMPONENTS)) {
                // components: cliques and chordless cycles are settled
                uint64_t rest[W];
#pragma unroll
                for (int j = 0; j < W; ++j) rest[j] = live[j];
                uint32_t nt = 0;
                for (;;) {
                    int sw = -1;
#pragma unroll
                    for (int j = W - 1; j >= 0; --j)
                        if (rest[j]) sw = j;
                    if (sw < 0) break;
                    uint64_t vis[W], fr[W], odd[W], last[W];
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        vis[j] = fr[j] = odd[j] = 0ull;
                    }
                    vis[sw] = fr[sw] = 1ull << low64(rest[sw]);
#pragma unroll
                    for (int j = 0; j < W; ++j) last[j] = fr[j];
                    uint32_t depth = 0;
                    for (;;) {
                        uint64_t nx[W];
                        bool anyn = false;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            uint64_t c = 0;
#pragma unroll
                            for (int k = 0; k < W; ++k)
                                if ((fr[k] >> l) & 1ull) c |= adj[k][j];
                            nx[j] = wave_or64(c) & live[j] & ~vis[j];
                            anyn = anyn || nx[j] != 0ull;
                        }
                        if (!anyn) break;
                        ++depth;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            if (depth & 1u) odd[j] |= nx[j];
                            vis[j] |= nx[j];
                            fr[j] = nx[j];
                            last[j] = nx[j];
                        }
                    }
                    uint32_t size = 0;
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        rest[j] &= ~vis[j];
                        size += popc64(vis[j]);
                    }
                    bool notclique = false, notcyc = false;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const bool inC = (vis[k] >> l) & 1ull;
                        notclique = notclique || ballot(inC && dg[k] != size - 1u) != 0ull;
                        notcyc = notcyc || ballot(inC && dg[k] != 2u) != 0ull;
                    }
                    if (!notclique) {
                        // all but the highest position
                        int hw = -1;
#pragma unroll
                        for (int j = 0; j < W; ++j)
                            if (vis[j]) hw = j;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            uint64_t cov = vis[j];
                            if (j == hw) cov &= ~(1ull << high64(vis[j]));
                            tin[j] |= cov;
                            live[j] &= ~vis[j];
                        }
                        sl += (int)size - 1;
                    } else if (!notcyc) {
                        // the odd BFS levels, plus one vertex of an even last
                        // level when the cycle is odd
                        const bool fix = (size & 1u) && !(depth & 1u);
                        int lw = -1;
#pragma unroll
                        for (int j = W - 1; j >= 0; --j)
                            if (last[j]) lw = j;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            uint64_t cov = odd[j];
                            if (fix && j == lw) cov |= 1ull << low64(last[j]);
                            tin[j] |= cov;
                            live[j] &= ~vis[j];
                        }
                        sl += (int)(size + 1u) / 2;
                    } else {
                        ++nt;
                    }
                }
                if (s0 + sl >= best) {
                    dead = true;
                } else if (nt == 0) {
                    small_improve<W>(s0 + sl, tin, mine, vid, d0);
                    dead = true;
                } else if (nt >= 2) {
                    // split: the pending nodes go out as ordinary nodes, this
                    // node continues on the general path
                    while (top > bot) {
                        --top;
                        uint64_t pl[W], pt[W];
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            pl[j] = SM[(uint32_t)top * 2u * W + j];
                            pt[j] = SM[(uint32_t)top * 2u * W + W + j];
                        }
                        if (!small_export<W>(pl, pt, s0 + (int)SS[top], mine, vid, adj))
                            return SMALL_STOP;
                    }
#pragma unroll
                    for (int k = 0; k < W; ++k)
                        if (mine[k]) DG::set(deg, vid[k], small_entry<W>(adj, live, tin, k, l));
                    wsync();
                    s = s0 + sl;
                    recompact();
                    return SMALL_SPLIT;
                }
                // one component left: its degrees are unchanged, so the rules
                // have nothing new and it is branched on
            }
            if (!dead) {
                // branch on the highest degree (lowest id on ties): the
                // N(v) child is pushed, the v child continues
                uint32_t kk = 0;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const bool lvk = (live[k] >> l) & 1ull;
                    const uint32_t p = l + 64u * k;
                    const uint32_t key = lvk ? (dg[k] << 8) | (255u - p) : 0u;
                    kk = key > kk ? key : kk;
                }
                const uint32_t key = wave_max(kk);
                const uint32_t v = 255u - (key & 255u);
                if (top >= (int)NV && bot > 0) {
                    // move the pending entries down over the given-away ones
                    const uint32_t cnt = (uint32_t)(top - bot);
                    for (uint32_t i = l; i < cnt * 2u * W; i += 64)
                        SM[i] = SM[(uint32_t)bot * 2u * W + i];
                    for (uint32_t i = l; i < cnt; i += 64) SS[i] = SS[(uint32_t)bot + i];
                    wsync();
                    top = (int)cnt;
                    bot = 0;
                }
                if (top >= (int)NV) {
                    // cannot happen: every pending entry took a vertex out of
                    // the path's live set
                    fail(VC_EDEVICE, FAIL_SMALL_STACK);
                    return SMALL_STOP;
                }
                uint64_t nbv[W];
                uint32_t cnb = 0;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    nbv[j] = ADJ[v * W + j] & live[j];
                    cnb += popc64(nbv[j]);
                }
                if (lane() == 0) {
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        const uint64_t vb = (uint32_t)j == (v >> 6) ? (1ull << (v & 63u)) : 0ull;
                        SM[(uint32_t)top * 2u * W + j] = live[j] & ~(nbv[j] | vb);
                        SM[(uint32_t)top * 2u * W + W + j] = tin[j] | nbv[j];
                    }
                    SS[top] = (uint32_t)(sl + (int)cnb);
                }
                wsync();
                ++top;
                live[v >> 6] &= ~(1ull << (v & 63u));
                tin[v >> 6] |= 1ull << (v & 63u);
                sl += 1;
                continue;
            }
            if (top == bot) return SMALL_DONE;
            --top;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                live[j] = SM[(uint32_t)top * 2u * W + j];
                tin[j] = SM[(uint32_t)top * 2u * W + W + j];
            }
            sl = (int)SS[top];
            if (top == bot) bot = top = 0;
        }
    }

    // Process one node and, depth-first, its first children in place.
    // Returns true when the whole search stops.
    __device__ __forceinline__ bool process(bool check_now) {
        bool recount = true;
        for (;;) {
            if (recount) count_node();
            recount = true;
            const int sr = stop_requested(check_now);
            check_now = false;
            if (sr == STOP_ALL) return true;
            if (sr == DROP) {
                complete(scope);
                charge(CYC_COMPLETE);
                return false;
            }
            best = cur_best();
            const bool alive = reduce();
            charge(CYC_REDUCE);
            if (!alive) {
                complete(scope);
                charge(CYC_COMPLETE);
                return false;
            }
            const int64_t b = (int64_t)best - s - 1;
            const uint64_t E = e2 / 2u;
            if (b < 0 || (int64_t)E > b * b) {
                complete(scope);
                charge(CYC_COMPLETE);
                return false;
            }
            if (E == 0) {
                improve(scope, s, -1);
                complete(scope);
                charge(CYC_COMPLETE);
                return false;
            }
            if (nl <= A.small_max && !small_off) {
                const int r = nl <= 64u ? small_solve<1>() : small_solve<2>();
                charge(CYC_REDUCE);
                if (r == SMALL_STOP) return true;
                if (r == SMALL_DONE) {
                    complete(scope);
                    charge(CYC_COMPLETE);
                    return false;
                }
                // split into components: on to the component branch
                small_off = true;
                known_connected = false;
                recount = false;
                continue;
            }
            if (!(A.flags & VC_OPT_NO_COMPONENTS) && !known_connected) {
                const uint32_t nc = find_components();
                const uint32_t nt = settle_simple_components(nc);
                if (nt != nc) recompact();
                charge(CYC_COMPONENTS);
                if (s >= best) {
                    complete(scope);
                    charge(CYC_COMPLETE);
                    return false;
                }
                if (nt == 0) {
                    improve(scope, s, -1);
                    complete(scope);
                    charge(CYC_COMPLETE);
                    return false;
                }
                if (nt == 1) {
                    known_connected = true;
                    if (nt != nc) {
                        recount = false;  // same node, rules again with the new bound
                        continue;
                    }
                } else {
                    const int cb = component_branch(nc, nt);
                    charge(CYC_COMPONENTS);
                    if (cb == CB_OK) {
                        small_off = false;
                        continue;
                    }
                    if (cb == CB_PRUNED) {
                        complete(scope);
                        charge(CYC_COMPLETE);
                        return false;
                    }
                    // registry full: branch on a vertex instead; if simple
                    // components were just settled, the rules (and the
                    // branching key) first run again on what is left
                    if (nt != nc) {
                        known_connected = true;
                        recount = false;
                        continue;
                    }
                }
            }
            const bool ok = vertex_branch();
            charge(CYC_BRANCH);
            if (!ok) return false;
            small_off = false;
        }
    }

    __device__ __forceinline__ void flush_stats() {
        if (lane() == 0) {
            add_relaxed(&A.ctl->nodes, nodes - nodes_flushed);
            add_relaxed(&A.ctl->comp_branches, cbr);
            add_relaxed(&A.ctl->components, comps);
            add_relaxed(&A.ctl->donations, dons);
            add_relaxed(&A.ctl->pushes, pushes);
            add_relaxed(&A.ctl->local_views, lviews);
            for (int i = 0; i < 6; ++i) add_relaxed(&A.ctl->cyc[i], cyc[i]);
            add_relaxed(&A.ctl->bytes_nodes, b_nodes);
            add_relaxed(&A.ctl->bytes_registry, b_reg);
            add_relaxed(&A.ctl->bytes_rows, b_rows);
            add_relaxed(&A.ctl->bytes_views, b_views);
            for (int i = 0; i < 8; ++i)
                if (chist[i]) add_relaxed(&A.ctl->comp_hist[i], chist[i]);
        }
    }

    // Batches: take the next unclaimed instance and make its root node (the
    // whole instance graph, nothing decided yet) the current node.
    __device__ __forceinline__ bool claim_instance() {
        if (!A.batch) return false;
        uint32_t got = NONE;
        int got_state = 0;
        if (lane() == 0) {
            // instances 0 .. limit-1 exist: all of a batch, the published
            // ones when serving
            const uint32_t limit = A.serve ? ld_relaxed(&A.ctl->inst_avail) : A.n_roots;
            if (ld_relaxed(&A.ctl->inst_next) < limit) {
                // count this worker as busy first, so that no idle worker
                // sees zero outstanding work while an instance is claimed
                add_relaxed(&A.ctl->outstanding, 1);
                uint32_t cur = ld_relaxed(&A.ctl->inst_next);
                if (A.serve) {
                    // a served launch that is ending claims nothing more
                    // (the next launch does); the count above is seen by
                    // every worker that sees the end after this check
                    fence_seq();
                    if (ld_relaxed(&A.ctl->quit_epoch) == A.launch_epoch) cur = limit;
                }
                while (cur < limit) {
                    const uint32_t prev = atomicCAS(&A.ctl->inst_next, cur, cur + 1u);
                    if (prev != cur) {
                        cur = prev;
                        continue;
                    }
                    // instances answered during set-up have no root node
                    const int st_ = ld_relaxed(&A.inst_state[cur]);
                    if (!(st_ & INST_FIN)) {
                        got = cur;
                        got_state = st_;
                        break;
                    }
                    cur = ld_relaxed(&A.ctl->inst_next);
                }
                if (got == NONE) add_relaxed(&A.ctl->outstanding, -1);
            }
        }
        got = uni(got);
        got_state = uni(got_state);
        if (got == NONE) return false;
        set_inst(got);
        load_view((int)got);
        for (uint32_t v = lane(); v < vpad; v += 64)
            DG::set(deg, v, v < vn ? vo(v + 1) - vo(v) : 0u);
        wsync();
        s = 0;
        scope = (int)got;
        begin_node(NONE);
        // a batch instance, or a request served as it was given, takes its
        // first bound here; other served requests bring one from their
        // root steps
        if (!A.serve || (got_state & INST_GREEDY)) greedy_bound();
        return true;
    }

    // A batch instance's initial bound (Sec. II-B: an attained cover such as
    // a greedy one).  From the instance's root node, the degree rules run to
    // their fixpoint and a maximum-degree vertex (lowest id on ties) goes
    // into the cover, repeatedly, until no edge is left; the vertices taken
    // (by the rules and by the greedy choices) form a cover, offered as the
    // root's Best.  A PVC query within k is answered by it at once.  The root
    // node waits meanwhile in the (empty) private stack's first slot and is
    // then restored, so the search starts from it with the high-degree rule
    // under the new bound.
    __device__ __forceinline__ void greedy_bound() {
        uint8_t* keep = stack + (size_t)top * A.slot_bytes;
        write_slot(keep, s, scope, NONE, nl, 0u, deg, view, vpad, false);
        best = INF;  // no bound yet: the degree rules alone
        for (;;) {
            reduce();
            if (e2 == 0) break;
            if (lane() == 0) R[0] = ~(uint32_t)(key & 0xFFFFFFFFull);
            wsync();
            take_list(R, 1);
            recompact();
        }
        improve(scope, s, -1);
        begin_node(copy_slot(keep));
        charge(CYC_REDUCE);
    }

    __device__ __forceinline__ void run() {
        bool busy = false;
        for (;;) {
            if (top > bot) {
                --top;
                begin_node(copy_slot(stack + (size_t)top * A.slot_bytes));
                if (top == bot) bot = top = 0;
                charge(CYC_FETCH);
                if (process(false)) break;
                continue;
            } else {
                bot = top = 0;
                if (busy && lane() == 0) add_relaxed(&A.ctl->outstanding, -1);
                // (a node from the worklist or a new instance starts with a
                // fresh poll; nodes from the own stack use the cached state)
                busy = false;
                if (claim_instance()) {
                    busy = true;
                    charge(CYC_FETCH);
                    if (process(true)) break;
                    continue;
                }
                if (lane() == 0) add_relaxed(&A.ctl->idle, 1);
                uint32_t spins = 0;
                bool got = false, quit = false, claimed = false;
                uint64_t t_idle = wall_clock64(), t_empty = 0;
                // poll the queue tail only; head, the outstanding count and
                // the stop flag are read when it moved or every 16th round
                uint64_t seen_tail = ~0ull;
                for (uint32_t round = 0;; ++round) {
                    uint64_t t = 0;
                    if (lane() == 0) t = ld_relaxed(&A.ctl->wl_tail);
                    t = uni(t);
                    if (t != seen_tail || (round & 15u) == 0) {
                        seen_tail = t;
                        int d = 0, outst = 0, closed = 0, ending = 0;
                        uint64_t h = 0;
                        uint32_t avail = 0, next = 0;
                        if (lane() == 0) {
                            d = ld_relaxed(&A.ctl->done);
                            if (A.serve) {
                                ending = ld_relaxed(&A.ctl->quit_epoch) == A.launch_epoch;
                                fence_seq();
                            }
                            h = ld_relaxed(&A.ctl->wl_head);
                            outst = ld_relaxed(&A.ctl->outstanding);
                            if (A.serve) {
                                closed = ld_relaxed(&A.ctl->closed);
                                avail = ld_relaxed(&A.ctl->inst_avail);
                                next = ld_relaxed(&A.ctl->inst_next);
                            }
                        }
                        d = uni(d);
                        outst = uni(outst);
                        h = uni(h);
                        closed = uni(closed);
                        avail = uni(avail);
                        next = uni(next);
                        ending = uni(ending);
                        if (d) {
                            quit = true;
                            break;
                        }
                        if (t > h) {
                            if (wl_take()) {
                                got = true;
                                break;
                            }
                            spins = 0;
                        } else if (ending) {
                            // the launch is ending: no new claims; leave
                            // once no node of it is left (a worker that
                            // claimed just before may still need help)
                            if (outst == 0) {
                                quit = true;
                                break;
                            }
                        } else if (next < avail) {
                            // a request was published: take it as a new
                            // instance (the claim counts this worker busy)
                            if (lane() == 0) add_relaxed(&A.ctl->idle, -1);
                            if (claim_instance()) {
                                claimed = true;
                                break;
                            }
                            if (lane() == 0) add_relaxed(&A.ctl->idle, 1);
                            spins = 0;
                        } else if (outst == 0 && (!A.serve || closed)) {
                            quit = true;
                            break;
                        }
                        // waiting for requests while nothing is outstanding
                        // is a served kernel's normal state, for a while:
                        // with no node and no unclaimed request left for
                        // linger_ticks the launch ends as a whole (every
                        // worker leaves, none claims again), and the server
                        // launches it again for requests published later
                        // (so the host's side-stream work never waits on a
                        // launch that waits on the host)
                        if (A.serve && outst == 0 && !ending) {
                            const uint64_t now = wall_clock64();
                            t_idle = now;
                            if (next >= avail) {
                                if (t_empty == 0) {
                                    t_empty = now;
                                } else if (now - t_empty > A.linger_ticks) {
                                    if (lane() == 0) {
                                        st_relaxed(reinterpret_cast<int*>(&A.ctl->quit_epoch),
                                                   (int)A.launch_epoch);
                                        fence_seq();
                                    }
                                    quit = true;
                                    break;
                                }
                            } else {
                                t_empty = 0;
                            }
                        }
                    }
                    if (wall_clock64() - t_idle > A.watchdog_ticks) {
                        // waited far longer than any node takes: give up
                        fail(VC_EDEVICE, FAIL_WATCHDOG);
                        quit = true;
                        break;
                    }
                    if (lane() == 0) backoff(spins);
                }
                if (!claimed && lane() == 0) add_relaxed(&A.ctl->idle, -1);
                charge(CYC_IDLE);
                if (quit) break;
                busy = got || claimed;
            }
            if (process(true)) break;
        }
        flush_inst();
        flush_stats();
    }
};

template <typename D, bool HL>
__global__ void __launch_bounds__(64) search_kernel(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    Worker<D, HL> w(a, lds);
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
        h->view = 0;
        h->inst = 0;
        h->flags = SLOT_COUNTED;  // the root entry's LiveNodes = 1 is this node's
        *reinterpret_cast<uint32_t*>(a.wl_slots + a.slot_bytes - 16u) = 0u;
        Ctl* c = a.ctl;
        c->wl_head = 0;
        c->wl_tail = 1;
        c->outstanding = 1;
        c->idle = 0;
        c->done = 0;
        c->err = 0;
        c->err_site = 0;
        c->reg_next = 2;  // entry 0 is the root scope; allocations are 2-aligned
        c->arena_next = 0;
        c->inst_next = 0;
        c->nodes = c->comp_branches = c->components = c->donations = c->pushes = 0;
        c->stale = c->local_views = 0;
        for (int i = 0; i < 8; ++i) c->comp_hist[i] = 0;
        for (int i = 0; i < 6; ++i) c->cyc[i] = 0;
        c->bytes_nodes = c->bytes_registry = c->bytes_rows = c->bytes_views = 0;
        RegEntry r = {};
        r.best = best0;
        r.live = 1;
        r.up = -1;
        r.lock = 0;
        r.cover_size = INF;
        r.nchild = 0;
        r.size = (int)a.n;
        r.view = 0;
        r.vn = (int)a.n;
        a.reg[0] = r;
    }
}

template <typename D, bool HL>
hipError_t launch_t(const SearchArgs& a, uint32_t workers, hipStream_t st) {
    hipLaunchKernelGGL((search_kernel<D, HL>), dim3(workers), dim3(64), a.lds_bytes, st, a);
    return hipGetLastError();
}

template <typename D, bool HL>
hipError_t occ_t(uint32_t lds_bytes, int* bpc) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, search_kernel<D, HL>, 64, lds_bytes);
}

template <typename D>
hipError_t init_t(const SearchArgs& a, int best0, const uint32_t* kdeg, uint32_t blocks,
                  hipStream_t st) {
    hipLaunchKernelGGL(search_init_kernel<D>, dim3(blocks), dim3(256), 0, st, a, best0, kdeg);
    return hipGetLastError();
}

}  // namespace vc
