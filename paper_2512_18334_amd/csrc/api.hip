// api.hip -- host runtime of libvc: the C ABI declared in include/vc.h.
//
// A solve runs, all on the context's stream:
//   validate -> degrees -> greedy bound -> root reduction -> induce ->
//   plan (one small readback) -> persistent search -> cover assembly.
// The host only checks arguments, sizes buffers and launches; every step of
// the method runs in the kernels of root.hip and search.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctx.hpp"
#include "internal.hpp"
#include "root.hpp"
#include "vc.h"

using namespace vc;

namespace vc {

// Exact host-side check of a host CSR against the rules stated in vc.h.
vc_status validate_host(const vc_csr* g) {
    const uint32_t n = g->n;
    const uint32_t* off = g->offsets;
    if (off[0] != 0 || (uint64_t)off[n] != g->nnz) return VC_EINVAL;
    for (uint32_t v = 0; v < n; ++v)
        if (off[v] > off[v + 1]) return VC_EINVAL;
    std::vector<uint32_t> col(g->nnz);
    for (uint64_t e = 0; e < g->nnz; ++e)
        col[e] = g->col_bytes == 2 ? ((const uint16_t*)g->cols)[e] : ((const uint32_t*)g->cols)[e];
    for (uint32_t v = 0; v < n; ++v) {
        auto b = col.begin() + off[v], en = col.begin() + off[v + 1];
        std::sort(b, en);
        for (auto it = b; it != en; ++it) {
            if (*it >= n || *it == v) return VC_EINVAL;
            if (it != b && *(it - 1) == *it) return VC_EINVAL;
        }
    }
    for (uint32_t v = 0; v < n; ++v)
        for (uint32_t e = off[v]; e < off[v + 1]; ++e) {
            const uint32_t w = col[e];
            if (!std::binary_search(col.begin() + off[w], col.begin() + off[w + 1], v))
                return VC_EINVAL;
        }
    return VC_OK;
}

vc_status check_args(const vc_csr* g) {
    if (!g) return VC_EINVAL;
    if (g->col_bytes != 2 && g->col_bytes != 4) return VC_EINVAL;
    if (g->col_bytes == 2 && g->n > 65536u) return VC_EINVAL;
    if (g->nnz >= (1ull << 32)) return VC_ERANGE;
    if (g->n >= 0x7FFFFFFFu) return VC_ERANGE;
    if (!g->offsets) return VC_EINVAL;
    if (g->nnz && !g->cols) return VC_EINVAL;
    return VC_OK;
}

// Workers and LDS layout of a search over degree arrays of n_pad entries:
// the caller's worker count, else one per CU; the LDS graph cache gets the
// caller's size, else the most that fits the workers per CU (at most 16K
// words).
vc_status plan_workers(vc_ctx* c, uint32_t n_pad, uint32_t deg_bytes, LdsPlan* lp,
                       uint32_t* gwords_out, uint32_t* workers_out, uint32_t want) {
    const uint32_t cus = (uint32_t)(c->cus > 0 ? c->cus : 1);
    uint32_t workers = c->opts.workers ? c->opts.workers : (want ? want : cus);
    const uint32_t base_lds = lds_plan(n_pad, deg_bytes, 0).bytes;
    uint32_t gwords = c->opts.gcache_words;
    if (!gwords) {
        const uint32_t cu_lds = (uint32_t)(c->lds_max < 163840 ? c->lds_max : 163840);
        for (uint32_t per = (workers + cus - 1u) / cus; per >= 1; --per) {
            const uint32_t share = cu_lds / per;
            if (share > base_lds + 4096u) {
                gwords = std::min<uint32_t>(32768u, (share - base_lds - 64u) / 4u);
                break;
            }
        }
    }
    *lp = lds_plan(n_pad, deg_bytes, gwords);
    if (lp->bytes > c->lds_max) return VC_ERANGE;
    int bpc = 0;
    HIPCHK(search_occupancy(deg_bytes, lp->bytes, &bpc));
    if (bpc < 1) return VC_ERANGE;
    if (workers > (uint32_t)bpc * cus) workers = (uint32_t)bpc * cus;
    *gwords_out = gwords;
    *workers_out = workers;
    return VC_OK;
}

vc_status plan_workers_hl(vc_ctx* c, uint32_t n_pad, uint32_t deg_bytes, LdsPlan* lp,
                          uint32_t* gwords_out, uint32_t* workers_out, uint64_t* hl_bytes) {
    const uint32_t cus = (uint32_t)(c->cus > 0 ? c->cus : 1);
    uint32_t workers = c->opts.workers ? c->opts.workers : cus;
    const uint32_t base_lds = lds_plan_hl(n_pad, deg_bytes, 0, hl_bytes).bytes;
    uint32_t gwords = c->opts.gcache_words;
    if (!gwords) {
        const uint32_t cu_lds = (uint32_t)(c->lds_max < 163840 ? c->lds_max : 163840);
        const uint32_t per = (workers + cus - 1u) / cus;
        const uint32_t share = cu_lds / (per ? per : 1u);
        gwords = share > base_lds + 4096u
                     ? std::min<uint32_t>(16384u, (share - base_lds - 64u) / 4u) : 0u;
    }
    *lp = lds_plan_hl(n_pad, deg_bytes, gwords, hl_bytes);
    if (lp->bytes > c->lds_max) return VC_ERANGE;
    int bpc = 0;
    HIPCHK(search_occupancy(deg_bytes, lp->bytes, &bpc, true));
    if (bpc < 1) return VC_ERANGE;
    if (workers > (uint32_t)bpc * cus) workers = (uint32_t)bpc * cus;
    *gwords_out = gwords;
    *workers_out = workers;
    return VC_OK;
}

}  // namespace vc

namespace vc {

// End state of the component branch registry after a search that ran to
// its end (Sec. III-C).  Allocations are contiguous blocks from `first`
// on: a parent entry p with nchild = c >= 2, its children p+1 .. p+c, and
// one padding entry when c+1 is odd.  Every parent and child must have
// been completed exactly once (the `done` count) with its LiveComps or
// LiveNodes counter back at 0.  Returns the entries that are not.
uint32_t registry_open_entries(const std::vector<RegEntry>& ents, uint32_t first,
                               uint32_t* parents, uint32_t* max_depth) {
    uint32_t bad = 0, np = 0, dmax = 0;
    const uint32_t used = (uint32_t)ents.size();
    // nesting depth of each parent: one more than the parent of the scope it
    // branched in (a root scope's branches are at depth 1)
    std::vector<uint32_t> depth(used, 0);
    for (uint32_t i = first; i < used;) {
        const RegEntry& p = ents[i];
        if (p.nchild < 2 || i + (uint32_t)p.nchild >= used) {
            ++bad;  // not a parent where one must start
            break;
        }
        ++np;
        const int a = p.up;  // the scope (a child entry, or a root) it branched in
        uint32_t d = 1;
        if (a >= (int)first && a < (int)used) {
            const int gp = ents[a].up;
            if (gp >= (int)first && gp < (int)i) d = depth[gp] + 1u;
            else ++bad;
        }
        depth[i] = d;
        dmax = d > dmax ? d : dmax;
        if (p.live != 0 || p.done != 1) ++bad;
        for (int j = 1; j <= p.nchild; ++j) {
            const RegEntry& ch = ents[i + j];
            if (ch.live != 0 || ch.done != 1 || ch.up != (int)i || ch.nchild != 0) ++bad;
        }
        i += ((uint32_t)p.nchild + 2u) & ~1u;
    }
    *parents = np;
    *max_depth = dmax;
    return bad;
}

}  // namespace vc

namespace {

// the crown reduction runs by default when the degree rules leave at least
// this many vertices (smaller kernels are cheaper to search than to match)
constexpr uint32_t CROWN_AUTO_MIN = 4096;

vc_status device_validate(vc_ctx* c, const RootGraph& rg, int* sorted = nullptr) {
    HIPCHK(ensure(c->pool, c->ctr, CTR_COUNT * 4));
    HIPCHK(ensure(c->pool, c->hsum, 8 * HSUM_SLOTS));
    HIPCHK(hipMemsetAsync(c->ctr.p, 0, CTR_COUNT * 4, c->stream));
    HIPCHK(hipMemsetAsync(c->hsum.p, 0, 8 * HSUM_SLOTS, c->stream));
    uint32_t bad = 0;
    HIPCHK(root_validate(rg, (uint32_t*)c->ctr.p, (unsigned long long*)c->hsum.p, c->stream,
                         c->hm->root, &bad,
                         sorted));
    return bad ? VC_EINVAL : VC_OK;
}

// Place the graph on the device (uploading a host CSR) and validate it.
vc_status stage_graph(vc_ctx* c, const vc_csr* g, RootGraph* rg) {
    vc_status st = check_args(g);
    if (st) return st;
    const bool skip = (c->opts.flags & VC_OPT_VALIDATE_SKIP) != 0;
    rg->n = g->n;
    rg->nnz = g->nnz;
    rg->col_bytes = g->col_bytes;
    if (g->flags & VC_CSR_DEVICE) {
        rg->off = g->offsets;
        rg->col = g->cols;
        st = order_after_default(c);
        if (st) return st;
        if (!skip && g->n) {
            st = device_validate(c, *rg, &rg->sorted);
            if (st) return st;
        }
        return VC_OK;
    }
    if (!skip) {
        st = validate_host(g);
        if (st) return st;
        // strictly increasing rows let the root rules bisect rows
        int inc = 1;
        for (uint32_t v = 0; v < g->n && inc; ++v)
            for (uint32_t e = g->offsets[v] + 1; e < g->offsets[v + 1]; ++e) {
                const uint32_t a = g->col_bytes == 2 ? ((const uint16_t*)g->cols)[e - 1]
                                                     : ((const uint32_t*)g->cols)[e - 1];
                const uint32_t b = g->col_bytes == 2 ? ((const uint16_t*)g->cols)[e]
                                                     : ((const uint32_t*)g->cols)[e];
                if (a >= b) {
                    inc = 0;
                    break;
                }
            }
        rg->sorted = inc;
    }
    HIPCHK(ensure(c->pool, c->in_off, 4ull * (g->n + 1)));
    HIPCHK(ensure(c->pool, c->in_col, (size_t)g->col_bytes * (g->nnz ? g->nnz : 1)));
    HIPCHK(hipMemcpyAsync(c->in_off.p, g->offsets, 4ull * (g->n + 1), hipMemcpyHostToDevice,
                          c->stream));
    if (g->nnz)
        HIPCHK(hipMemcpyAsync(c->in_col.p, g->cols, (size_t)g->col_bytes * g->nnz,
                              hipMemcpyHostToDevice, c->stream));
    rg->off = (const uint32_t*)c->in_off.p;
    rg->col = c->in_col.p;
    return VC_OK;
}

vc_status root_buffers(vc_ctx* c, const RootGraph& g, RootBufs* b) {
    const size_t n = g.n, n1 = g.n + 1;
    HIPCHK(ensure(c->pool, c->rdeg, 4 * n1));
    HIPCHK(ensure(c->pool, c->gdeg, 4 * n1));
    HIPCHK(ensure(c->pool, c->gin, n1));
    HIPCHK(ensure(c->pool, c->addf, n1));
    HIPCHK(ensure(c->pool, c->newly, n1));
    HIPCHK(ensure(c->pool, c->flags, 4 * (n1 + 1)));
    HIPCHK(ensure(c->pool, c->newid, 4 * (n1 + 1)));
    HIPCHK(ensure(c->pool, c->oldid, 4 * n1));
    HIPCHK(ensure(c->pool, c->kdeg, 4 * (n1 + 1)));
    HIPCHK(ensure(c->pool, c->koff, 4 * (n1 + 1)));
    HIPCHK(ensure(c->pool, c->kcol, 4 * (g.nnz ? g.nnz : 1)));
    HIPCHK(ensure(c->pool, c->cover, 4 * n1));
    HIPCHK(ensure(c->pool, c->scan_tmp, 4 * (n / 2048 + 4)));
    HIPCHK(ensure(c->pool, c->ctr, CTR_COUNT * 4));
    HIPCHK(ensure(c->pool, c->hsum, 8 * HSUM_SLOTS));
    b->rdeg = (uint32_t*)c->rdeg.p;
    b->gdeg = (uint32_t*)c->gdeg.p;
    b->gin = (uint8_t*)c->gin.p;
    b->addf = (uint8_t*)c->addf.p;
    b->newly = (uint8_t*)c->newly.p;
    b->flags = (uint32_t*)c->flags.p;
    b->newid = (uint32_t*)c->newid.p;
    b->oldid = (uint32_t*)c->oldid.p;
    b->kdeg = (uint32_t*)c->kdeg.p;
    b->koff = (uint32_t*)c->koff.p;
    b->kcol = c->kcol.p;
    b->cover = (uint32_t*)c->cover.p;
    b->scan_tmp = (uint32_t*)c->scan_tmp.p;
    b->ctr = (uint32_t*)c->ctr.p;
    b->hsum = (unsigned long long*)c->hsum.p;
    b->hm = c->hm->root;
    return VC_OK;
}

// Copy `count` cover ids from the device list into the caller's array.
vc_status fetch_cover(vc_ctx* c, const RootBufs& b, uint32_t count, uint32_t* cover,
                      uint32_t* cover_len) {
    if (cover && count)
        HIPCHK(hipMemcpyAsync(cover, b.cover, 4ull * count, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (cover_len) *cover_len = count;
    return VC_OK;
}

struct Outcome {
    uint32_t size = 0;  // MVC size, or the size of the cover found (PVC)
    int yes = 0;
    uint32_t cover_count = 0;
};

// The whole pipeline.  pvc: 0 = MVC, 1 = PVC with bound k.
vc_status solve(vc_ctx* c, const vc_csr* g, int pvc, uint32_t k, Outcome* out, uint32_t* cover,
                uint32_t* cover_len) {
    const double t0 = now_ms();
    vc_stats stv{};
    RootGraph rg;
    vc_status st = stage_graph(c, g, &rg);
    if (st) return st;
    stv.n_input = g->n;
    if (g->n == 0 || g->nnz == 0) {
        out->size = 0;
        out->yes = 1;
        out->cover_count = 0;
        if (cover_len) *cover_len = 0;
        stv.ms_total = now_ms() - t0;
        c->last = stv;
        return VC_OK;
    }
    RootBufs b;
    st = root_buffers(c, rg, &b);
    if (st) return st;
    hipStream_t s = c->stream;
    HIPCHK(hipMemsetAsync(b.ctr, 0, CTR_COUNT * 4, s));
    HIPCHK(hipEventRecord(c->ev[0], s));
    HIPCHK(root_init(rg, b, s));
    // The degree rules need no bound: they run first, and the greedy bound
    // (Sec. II-B) is taken on what they leave, starting from the vertices
    // they forced (an attained cover either way; on graphs the rules settle,
    // no greedy round is left to run).  VC_OPT_NO_INDUCE skips all root rules.
    const bool no_induce = (c->opts.flags & VC_OPT_NO_INDUCE) != 0;
    uint32_t rounds = 0;
    if (!no_induce) {
        HIPCHK(root_reduce(rg, b, 0x3FFFFFFF, s, 1u << 16, &rounds));
        HIPCHK(root_greedy_rest(rg, b, s));
    }
    uint32_t grounds = 0;
    HIPCHK(root_greedy(rg, b, s, &grounds));
    HostMail* hm = c->hm;
    HIPCHK(hipMemcpyAsync(&hm->ghdr[0], b.ctr + CTR_GSIZE, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hm->ghdr[1], b.ctr + CTR_SROOT, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hm->w[0], b.ctr + CTR_ROUNDS, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const uint32_t ghdr[2] = {hm->ghdr[0], hm->ghdr[1]};
    const uint32_t gsize = ghdr[0] + ghdr[1];  // forced + greedy
    stv.greedy_size = gsize;
    stv.root_rounds = rounds + hm->w[0];  // (small graphs count on the device)
    stv.forced_root = ghdr[1];

    // answers decided at the root: the root steps' device time ends here
    auto root_time = [&]() -> vc_status {
        float ms = 0;
        HIPCHK(hipEventRecord(c->ev[1], s));
        HIPCHK(hipEventSynchronize(c->ev[1]));
        HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        stv.ms_root = ms;
        return VC_OK;
    };
    auto finish_with_greedy = [&](int yes) -> vc_status {
        // the greedy cover is the answer (MVC), or a PVC yes within k
        if (stv.ms_root == 0.0) {
            const vc_status rt = root_time();
            if (rt) return rt;
        }
        HIPCHK(root_cover(rg, b, 0, 0, nullptr, s));
        HIPCHK(hipMemcpyAsync(&hm->cnt, b.newid + rg.n, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const uint32_t cnt = hm->cnt;
        if (cnt != gsize) return broken("greedy cover size");
        out->size = gsize;
        out->yes = yes;
        out->cover_count = cnt;
        vc_status r = fetch_cover(c, b, cnt, cover, cover_len);
        stv.ms_total = now_ms() - t0;
        c->last = stv;
        return r;
    };
    auto finish_no = [&]() -> vc_status {
        if (stv.ms_root == 0.0) {
            const vc_status rt = root_time();
            if (rt) return rt;
        }
        out->yes = 0;
        out->size = 0;
        out->cover_count = 0;
        if (cover_len) *cover_len = 0;
        stv.ms_total = now_ms() - t0;
        c->last = stv;
        return VC_OK;
    };

    int best0;
    if (pvc) {
        if (gsize <= k) return finish_with_greedy(1);
        best0 = (int)k + 1;
    } else {
        best0 = (int)gsize;
    }
    if (!no_induce && ghdr[0] == 0) {
        // the greedy took nothing: the degree rules, which keep a minimum
        // cover, left no edge, so the vertices they forced are a minimum
        // cover (MVC = |S_root|; a PVC bound below it is a no)
        return pvc ? finish_no() : finish_with_greedy(1);
    }

    // root reduction to a fixpoint under the bound best0 (Sec. IV-B)
    // (skipped under VC_OPT_NO_INDUCE: the search starts from the input)
    if (!no_induce) {
        uint32_t r2 = 0;
        HIPCHK(root_reduce(rg, b, best0, s, 1u << 16, &r2));
        rounds += r2;
    }
    HIPCHK(hipMemcpyAsync(&hm->sroot, b.ctr + CTR_SROOT, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hm->w[0], b.ctr + CTR_ROUNDS, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(c->ev[1], s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t sroot = hm->sroot;
    stv.root_rounds = rounds + hm->w[0];
    stv.forced_root = sroot;
    if ((int)sroot >= best0) {
        // no cover below best0 exists
        return pvc ? finish_no() : finish_with_greedy(1);
    }

    // induce the subgraph on the vertices that still have edges
    HIPCHK(root_induce_a(rg, b, s, no_induce));
    HIPCHK(hipMemcpyAsync(&hm->hdr[0], b.newid + rg.n, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hm->hdr[1], b.ctr + CTR_MAXDEG, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t np = hm->hdr[0], dmax = hm->hdr[1];
    // crown reductions (Sec. IV-B), each followed by the degree rules again,
    // while crowns are found: by default on large kernels only
    const uint32_t fl = c->opts.flags;
    const bool crown = !no_induce && !(fl & VC_OPT_NO_CROWN) &&
                       np >= ((fl & VC_OPT_CROWN) ? 2u : CROWN_AUTO_MIN);
    for (uint32_t it = 0; crown && np >= 2u && it < 16u; ++it) {
        HIPCHK(ensure(c->pool, c->crown, 32ull * rg.n));
        b.cw = (uint32_t*)c->crown.p;
        uint32_t h = 0;
        HIPCHK(root_crown(rg, b, s, &h));
        if (h == 0) break;
        ++stv.crown_rounds;
        stv.crown_cover += h;
        uint32_t r2 = 0;
        HIPCHK(root_reduce(rg, b, best0, s, 1u << 16, &r2));
        stv.root_rounds += r2;
        HIPCHK(hipMemcpyAsync(&hm->sroot, b.ctr + CTR_SROOT, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hm->crown_removed, b.ctr + CTR_CROWN_I, 4, hipMemcpyDeviceToHost,
                              s));
        HIPCHK(hipEventRecord(c->ev[1], s));
        HIPCHK(hipStreamSynchronize(s));
        sroot = hm->sroot;
        stv.crown_removed = hm->crown_removed;
        stv.forced_root = sroot;
        if ((int)sroot >= best0) return pvc ? finish_no() : finish_with_greedy(1);
        HIPCHK(hipMemsetAsync(b.ctr + CTR_MAXDEG, 0, 4, s));  // raised by atomicMax
        HIPCHK(root_induce_a(rg, b, s, false));
        HIPCHK(hipMemcpyAsync(&hm->hdr[0], b.newid + rg.n, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hm->hdr[1], b.ctr + CTR_MAXDEG, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        np = hm->hdr[0];
        dmax = hm->hdr[1];
    }
    stv.n_kernel = np;
    stv.max_degree_kernel = dmax;
    const int kbest0 = best0 - (int)sroot;
    int kbest = kbest0;
    bool improved = false;
    uint64_t nnzp = 0;
    uint32_t* root_bitmap = nullptr;
    if (np == 0) {
        // the rules covered every edge: |S_root| < best0 is attained
        kbest = 0;
        improved = true;
    } else {
        const uint32_t kcol_bytes = 4u;  // the search reads 32-bit column ids
        HIPCHK(root_induce_b(rg, b, np, kcol_bytes, s));
        HIPCHK(hipMemcpyAsync(&hm->nz, b.koff + np, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(c->ev[2], s));
        HIPCHK(hipStreamSynchronize(s));
        const uint32_t nz = hm->nz;
        nnzp = nz;
        stv.nnz_kernel = nnzp;

        // ------------------------------------------------ plan
        const uint32_t deg_bytes = dmax <= 254u ? 1u : (dmax <= 65534u ? 2u : 4u);
        stv.deg_bytes = deg_bytes;
        const uint32_t n_pad = (np + 63u) & ~63u;
        LdsPlan lp;
        uint32_t gwords = 0, workers = 0;
        uint64_t hl_bytes = 0;
        st = plan_workers(c, n_pad, deg_bytes, &lp, &gwords, &workers);
        // lists too large for LDS: they go to HBM, one region per worker
        if (st == VC_ERANGE) st = plan_workers_hl(c, n_pad, deg_bytes, &lp, &gwords, &workers,
                                                  &hl_bytes);
        if (st) return st;
        const uint32_t slot_bytes = (uint32_t)sizeof(SlotHdr) + n_pad * deg_bytes + 16u;
        uint32_t depth = std::min<uint32_t>(np, (uint32_t)kbest0) + np / 4u + 16u;
        const uint32_t wl_cap = c->opts.worklist_cap ? c->opts.worklist_cap
                                                     : std::max<uint32_t>(1024u, 4u * workers);
        // the worklist and control block come off the top; stacks take up
        // to 1/2 of the rest, the registry 1/4, the graph arena 1/16
        const uint64_t wl_bytes = (uint64_t)wl_cap * (slot_bytes + 8u) + sizeof(Ctl) + (64u << 10);
        const uint64_t budget = search_budget(c->opts, c->pool, wl_bytes);
        const uint64_t per_worker = (uint64_t)depth * slot_bytes + hl_bytes;
        uint64_t wmax = (budget / 2) / (per_worker ? per_worker : 1);
        if (wmax < 1) wmax = 1;
        if (workers > wmax) workers = (uint32_t)wmax;
        if (workers < 1) workers = 1;
        const uint32_t bm_words = ((np + 31u) / 32u + 31u) & ~31u;  // whole 128-byte lines
        uint64_t reg_cap = c->opts.registry_cap ? c->opts.registry_cap : (1u << 20);
        const uint64_t reg_bytes_each = sizeof(RegEntry) + 4ull * bm_words;
        const uint64_t reg_budget = budget / 4;
        if (reg_cap * reg_bytes_each > reg_budget) reg_cap = reg_budget / reg_bytes_each;
        if (reg_cap < 64) reg_cap = 64;
        stv.workers = workers;

        HIPCHK(ensure(c->pool, c->stacks, (size_t)workers * depth * slot_bytes));
        if (hl_bytes) HIPCHK(ensure(c->pool, c->hl, (size_t)workers * hl_bytes));
        HIPCHK(ensure(c->pool, c->wl_slots, (size_t)wl_cap * slot_bytes));
        HIPCHK(ensure(c->pool, c->wl_seq, 8ull * wl_cap));
        HIPCHK(ensure(c->pool, c->ctl, sizeof(Ctl)));
        HIPCHK(ensure(c->pool, c->reg, sizeof(RegEntry) * reg_cap));
        HIPCHK(ensure(c->pool, c->bitmaps, 4ull * bm_words * reg_cap));
        uint64_t arena_words = std::min<uint64_t>(budget / 16 / 4, 64ull << 20);
        HIPCHK(ensure(c->pool, c->arena, 4ull * arena_words));

        SearchArgs a{};
        a.n = np;
        a.nnz = (uint32_t)nnzp;
        a.n_pad = n_pad;
        a.off = b.koff;
        a.col = (const uint32_t*)b.kcol;
        a.slot_bytes = slot_bytes;
        a.stack_depth = depth;
        a.stacks = (uint8_t*)c->stacks.p;
        a.wl_slots = (uint8_t*)c->wl_slots.p;
        a.wl_seq = (uint64_t*)c->wl_seq.p;
        a.wl_cap = wl_cap;
        a.reg_cap = (uint32_t)reg_cap;
        a.ctl = (Ctl*)c->ctl.p;
        a.reg = (RegEntry*)c->reg.p;
        a.bitmaps = (uint32_t*)c->bitmaps.p;
        a.bm_words = bm_words;
        a.lds_L = lp.L;
        a.lds_Q = lp.Q;
        a.lds_R = lp.R;
        a.lds_VB = lp.VB;
        a.lds_PB = lp.PB;
        a.lds_MK = lp.MK;
        a.lds_G = lp.G;
        a.lds_bytes = lp.bytes;
        a.gcache_words = gwords;
        a.hl = hl_bytes ? 1u : 0u;
        a.hl_base = hl_bytes ? (uint8_t*)c->hl.p : nullptr;
        a.hl_stride = hl_bytes;
        stv.lists_in_hbm = a.hl;
        a.arena = (uint32_t*)c->arena.p;
        a.arena_words = arena_words;
        a.donate_min = c->opts.donate_min ? c->opts.donate_min : 48u;
        a.strong_fences = (c->opts.flags & VC_OPT_STRONG_ORDER) ? 1u : 0u;
        a.pvc = pvc;
        a.k = pvc ? (int)k - (int)sroot : 0;
        a.flags = c->opts.flags;
        a.donate_slack = c->opts.donate_slack;
        // one search: 64 (the tree must split over the workers; subtrees
        // below 64 live vertices stay short)
        a.small_max = (c->opts.flags & VC_OPT_NO_SMALL) ? 0u
                      : std::min<uint32_t>(c->opts.small_max ? c->opts.small_max : 64u, 128u);
        a.node_limit = c->opts.node_limit;
        a.n_roots = 1;  // one root scope (entry 0); no instance claims
        a.batch = 0;
        a.watchdog_ticks = (uint64_t)c->wall_khz * (c->opts.watchdog_ms ? c->opts.watchdog_ms : 120000u);

        HIPCHK(launch_search_init(a, kbest0, deg_bytes, b.kdeg, s));
        HIPCHK(hipEventRecord(c->ev[3], s));
        HIPCHK(launch_search(a, deg_bytes, workers, s));
        HIPCHK(hipEventRecord(c->ev[4], s));
        HIPCHK(hipMemcpyAsync(&hm->ctl, c->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hm->reg0, c->reg.p, sizeof(RegEntry), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const Ctl ctl = hm->ctl;
        const RegEntry root = hm->reg0;
        stv.tree_nodes = ctl.nodes;
        stv.component_branches = ctl.comp_branches;
        stv.components = ctl.components;
        stv.donations = ctl.donations;
        stv.pushes = ctl.pushes;
        stv.local_views = ctl.local_views;
        for (int i = 0; i < 6; ++i) stv.cycles[i] = ctl.cyc[i];
        stv.bytes_nodes = ctl.bytes_nodes;
        stv.bytes_registry = ctl.bytes_registry;
        stv.bytes_rows = ctl.bytes_rows;
        stv.bytes_views = ctl.bytes_views;
        for (int i = 0; i < 8; ++i) stv.comp_hist[i] = ctl.comp_hist[i];
        stv.slot_bytes = slot_bytes;
        stv.bitmap_bytes = 4u * bm_words;
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[3], c->ev[4]));
        stv.ms_search = ms;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
        stv.ms_induce = ms;
        if (ctl.err) {
            if (getenv("VC_DEBUG"))
                fprintf(stderr, "libvc: search stopped: status %d at check %d\n", ctl.err,
                        ctl.err_site);
            c->last = stv;
            return (vc_status)ctl.err;
        }
        stv.stale_reads = ctl.stale;
        const uint32_t used = std::min<uint32_t>(ctl.reg_next, (uint32_t)reg_cap);
        stv.reg_entries = used > 2u ? used - 2u : 0u;
        if ((c->opts.flags & VC_OPT_CHECK_REGISTRY) && !ctl.done) {
            // the search ran to its end: every branch on components was
            // completed by its last descendant (Sec. III-C)
            std::vector<RegEntry> ents(used);
            if (used)
                HIPCHK(hipMemcpyAsync(ents.data(), c->reg.p, sizeof(RegEntry) * used,
                                      hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            uint32_t parents = 0, depth = 0;
            stv.reg_open = registry_open_entries(ents, 2u, &parents, &depth);
            stv.reg_parents = parents;
            stv.reg_depth = depth;
            stv.reg_checked = 1;
        }
        if (root.best < kbest0) {
            // internal invariant: the root's bitmap holds a cover of size Best
            if (root.cover_size != root.best) {
                c->last = stv;
                return broken("root cover size != Best");
            }
            improved = true;
            kbest = root.best;
            root_bitmap = (uint32_t*)c->bitmaps.p;
        }
    }
    {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        stv.ms_root = ms;
    }
    if (!improved) return pvc ? finish_no() : finish_with_greedy(1);

    const uint32_t size = sroot + (uint32_t)kbest;
    HIPCHK(root_cover(rg, b, np, 1, root_bitmap, s));
    HIPCHK(hipMemcpyAsync(&hm->cnt, b.newid + rg.n, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const uint32_t cnt = hm->cnt;
    // internal invariant: |cover| == size (MVC); in PVC a cover assembled
    // while components were still improving may be smaller than its bound
    if (pvc ? cnt > size : cnt != size) {
        c->last = stv;
        return broken("assembled cover size");
    }
    out->size = pvc ? cnt : size;
    out->yes = pvc ? (size <= k) : 1;
    out->cover_count = cnt;
    st = fetch_cover(c, b, cnt, cover, cover_len);
    stv.ms_total = now_ms() - t0;
    c->last = stv;
    return st;
}

}  // namespace

namespace vc {

vc_status stage_input(vc_ctx* c, const vc_csr* g, RootGraph* rg) { return stage_graph(c, g, rg); }

vc_status solve_one(vc_ctx* c, const vc_csr* g, int pvc, uint32_t k, uint32_t* size, int* yes,
                    uint32_t* cover, uint32_t* cover_len) {
    if (pvc && k > 0x3FFFFFF0u) k = 0x3FFFFFF0u;
    Outcome o;
    vc_status st = solve(c, g, pvc, k, &o, cover, cover_len);
    if (st) return st;
    if (size) *size = o.size;
    if (yes) *yes = o.yes;
    if (pvc && !o.yes && cover_len) *cover_len = 0;
    return VC_OK;
}

}  // namespace vc

namespace vc {

// every device buffer of a context (teardown and pool resets)
std::vector<DevBuf*> ctx_buffers(vc_ctx* c) {
    std::vector<DevBuf*> v = {
        &c->in_off, &c->in_col, &c->rdeg,    &c->gdeg,   &c->gin,     &c->addf,    &c->newly,
        &c->flags,  &c->newid,  &c->oldid,   &c->kdeg,   &c->koff,    &c->kcol,    &c->cover,
        &c->scan_tmp, &c->ctr,  &c->hsum,    &c->crown,  &c->stacks,  &c->wl_slots, &c->wl_seq,
        &c->ctl,    &c->reg,    &c->bitmaps, &c->arena,  &c->hl,     &c->b_n,     &c->b_nnz,   &c->b_ob,
        &c->b_cb,   &c->b_gat,  &c->b_rbase, &c->b_cbase, &c->b_k,    &c->b_state, &c->b_nodes,
        &c->b_bad,  &c->b_hs,   &c->b_cnt,   &c->b_cov};
    for (auto& b : c->en) v.push_back(&b);
    return v;
}

hipError_t host_mail(HostMail** out) {
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, sizeof(HostMail), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    memset(p, 0, sizeof(HostMail));
    *out = (HostMail*)p;
    return hipSuccess;
}

void host_mail_free(HostMail* m) {
    if (m) hipHostFree(m);
}

void pool_reset(vc_ctx* c) {
    if (!c->pool.base) return;
    for (DevBuf* b : ctx_buffers(c)) forget(*b);
    if (c->batch_exec) {
        hipGraphExecDestroy(c->batch_exec);
        c->batch_exec = nullptr;
    }
    c->batch_key.clear();
    server_forget_buffers(c);
    c->pool.used = 0;
}

// Device inputs are read on the context's stream.  A context that made its
// own stream first waits for the legacy default stream (an event recorded
// there completes after all earlier work of the blocking streams, PyTorch's
// default stream among them), so a graph written there is complete.
vc_status order_after_default(vc_ctx* c) {
    if (!c->wait_default) return VC_OK;
    HIPCHK(hipEventRecord(c->ev[5], nullptr));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev[5], 0));
    return VC_OK;
}

}  // namespace vc

namespace {

// Scratch of vc_min_static: a file-scope device array, one copy per GPU.
// Host code never uses the array's name as an address: its device address
// on each GPU comes from hipGetSymbolAddress, taken once per device when
// the first context on that device is created.
constexpr size_t SCRATCH_BYTES = 256ull << 20;
constexpr uint32_t STATIC_MAX_N = 1u << 20;
constexpr uint64_t STATIC_MAX_NNZ = 1ull << 24;
__device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};
hipError_t scratch_err[MAX_DEVICES] = {};

// with `device` current
void scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch_ptr[device] || scratch_err[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        if (getenv("VC_DEBUG"))
            fprintf(stderr, "libvc: hipGetSymbolAddress(scratch) -> %s\n", hipGetErrorString(e));
        return;
    }
    scratch_ptr[device] = p;
}

void* scratch_address(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(scratch_mu);
    return scratch_ptr[device];
}

}  // namespace

extern "C" {

vc_status vc_ctx_create(int device, void* stream, void* arena, uint64_t arena_bytes,
                        const vc_opts* opts, vc_ctx** out) {
    if (!out) return VC_EINVAL;
    *out = nullptr;
    if ((arena == nullptr) != (arena_bytes == 0)) return VC_EINVAL;
    int count = 0;
    hipError_t he = hipGetDeviceCount(&count);
    if (he != hipSuccess || device < 0 || device >= count) {
        if (getenv("VC_DEBUG"))
            fprintf(stderr, "libvc: hipGetDeviceCount -> %s, count %d, device %d\n",
                    hipGetErrorString(he), count, device);
        return VC_EDEVICE;
    }
    he = hipSetDevice(device);
    if (he != hipSuccess) {
        if (getenv("VC_DEBUG"))
            fprintf(stderr, "libvc: hipSetDevice -> %s\n", hipGetErrorString(he));
        return VC_EDEVICE;
    }
    if (arena) {
        // the arena must be device memory of this device
        hipPointerAttribute_t pa{};
        if (hipPointerGetAttributes(&pa, arena) != hipSuccess ||
            pa.type != hipMemoryTypeDevice || pa.device != device)
            return VC_EINVAL;
    }
    vc_ctx* c = new (std::nothrow) vc_ctx();
    if (!c) return VC_ENOMEM;
    c->device = device;
    if (opts) c->opts = *opts;
    c->pool.poison = (c->opts.flags & VC_OPT_POISON) != 0;
    if (arena) {
        const uintptr_t a0 = (uintptr_t)arena, a1 = (a0 + 255u) & ~(uintptr_t)255u;
        c->pool.base = (uint8_t*)a1;
        c->pool.cap = arena_bytes > (a1 - a0) ? arena_bytes - (a1 - a0) : 0;
        c->pool.used = 0;
    }
    hipDeviceProp_t prop;
    he = hipGetDeviceProperties(&prop, device);
    if (he != hipSuccess) {
        if (getenv("VC_DEBUG"))
            fprintf(stderr, "libvc: hipGetDeviceProperties -> %s\n", hipGetErrorString(he));
        delete c;
        return VC_EDEVICE;
    }
    c->cus = prop.multiProcessorCount;
    c->lds_max = prop.sharedMemPerBlock;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
        khz > 0)
        c->wall_khz = khz;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (he != hipSuccess) {
            if (getenv("VC_DEBUG"))
                fprintf(stderr, "libvc: hipStreamCreateWithFlags -> %s\n", hipGetErrorString(he));
            delete c;
            return VC_EDEVICE;
        }
        c->own_stream = true;
        c->wait_default = true;
    }
    for (auto& e : c->ev) {
        he = hipEventCreateWithFlags(&e, hipEventDefault);
        if (he != hipSuccess) {
            if (getenv("VC_DEBUG"))
                fprintf(stderr, "libvc: hipEventCreate -> %s\n", hipGetErrorString(he));
            vc_ctx_destroy(c);
            return VC_EDEVICE;
        }
    }
    he = host_mail(&c->hm);
    if (he != hipSuccess) {
        if (getenv("VC_DEBUG"))
            fprintf(stderr, "libvc: hipHostMalloc -> %s\n", hipGetErrorString(he));
        vc_ctx_destroy(c);
        return he == hipErrorOutOfMemory ? VC_ENOMEM : VC_EDEVICE;
    }
    // the static scratch's address on this device (library set-up, once per
    // device; vc_min_static reports a failure here)
    scratch_init(device);
    *out = c;
    return VC_OK;
}

vc_status vc_ctx_destroy(vc_ctx* c) {
    if (!c) return VC_OK;
    hipSetDevice(c->device);
    if (c->scratch_ctx) {
        vc_ctx_destroy(c->scratch_ctx);
        c->scratch_ctx = nullptr;
    }
    server_shutdown(c);
    if (c->stream) hipStreamSynchronize(c->stream);
    if (c->batch_exec) hipGraphExecDestroy(c->batch_exec);
    for (DevBuf* b : ctx_buffers(c)) release(*b);
    if (!c->shared_events) {
        for (auto& e : c->ev)
            if (e) hipEventDestroy(e);
        host_mail_free(c->hm);
    }
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    delete c;
    return VC_OK;
}

vc_status vc_validate(vc_ctx* c, const vc_csr* g) {
    vc_status st = check_args(g);
    if (st) return st;
    if (!(g->flags & VC_CSR_DEVICE)) return validate_host(g);
    if (!c) return VC_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    if (g->n == 0) return g->nnz == 0 ? VC_OK : VC_EINVAL;
    if (!server_busy(c)) pool_reset(c);
    {
        const vc_status o = order_after_default(c);
        if (o) return o;
    }
    RootGraph rg{g->n, g->nnz, g->offsets, g->cols, g->col_bytes};
    return device_validate(c, rg);
}

vc_status vc_min(vc_ctx* c, const vc_csr* g, uint32_t* size, uint32_t* cover,
                 uint32_t* cover_len) {
    if (!c || !size) return VC_EINVAL;
    if (server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    pool_reset(c);
    return solve_one(c, g, 0, 0, size, nullptr, cover, cover_len);
}

vc_status vc_param(vc_ctx* c, const vc_csr* g, uint32_t k, int* yes, uint32_t* cover,
                   uint32_t* cover_len) {
    if (!c || !yes) return VC_EINVAL;
    if (server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    pool_reset(c);
    return solve_one(c, g, 1, k, nullptr, yes, cover, cover_len);
}

vc_status vc_min_static(vc_ctx* c, const vc_csr* g, uint32_t* size, uint32_t* cover,
                        uint32_t* cover_len) {
    if (!c || !size) return VC_EINVAL;
    vc_status st = check_args(g);
    if (st) return st;
    if (g->n > STATIC_MAX_N || g->nnz > STATIC_MAX_NNZ) return VC_ERANGE;
    if (server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    void* base = scratch_address(c->device);
    if (!base) return VC_EDEVICE;
    if (!c->scratch_ctx) {
        // host-side state only: the stream, events and device facts are the
        // caller context's, every device buffer is carved from the scratch
        vc_ctx* s = new (std::nothrow) vc_ctx();
        if (!s) return VC_ENOMEM;
        s->device = c->device;
        s->stream = c->stream;
        s->own_stream = false;
        s->wait_default = c->wait_default;
        s->cus = c->cus;
        s->lds_max = c->lds_max;
        s->wall_khz = c->wall_khz;
        for (int i = 0; i < 6; ++i) s->ev[i] = c->ev[i];
        s->hm = c->hm;
        s->shared_events = true;
        c->scratch_ctx = s;
    }
    vc_ctx* s = c->scratch_ctx;
    s->opts = c->opts;
    s->pool.base = (uint8_t*)base;
    s->pool.cap = SCRATCH_BYTES;
    s->pool.used = 0;
    s->pool.poison = c->pool.poison;
    pool_reset(s);
    st = solve_one(s, g, 0, 0, size, nullptr, cover, cover_len);
    c->last = s->last;
    // the scratch could not hold the graph's buffers or its search plan
    return st == VC_ENOMEM ? VC_ERANGE : st;
}

vc_status vc_last_stats(vc_ctx* c, vc_stats* out) {
    if (!c || !out) return VC_EINVAL;
    *out = c->last;
    return VC_OK;
}

const char* vc_status_str(vc_status s) {
    switch (s) {
        case VC_OK: return "ok";
        case VC_EINVAL: return "invalid argument or graph";
        case VC_ENOMEM: return "out of device memory or capacity";
        case VC_EDEVICE: return "device error";
        case VC_EAGAIN: return "pending";
        case VC_ETIMEDOUT: return "node limit reached";
        case VC_ECANCELED: return "cancelled";
        case VC_ERANGE: return "size beyond the library's limits";
    }
    return "unknown status";
}

}  // extern "C"
