// batch.hip -- many independent graphs in one persistent search launch
// (vc_min_batch, vc_param_batch).
//
// Every instance becomes a root scope of its own in the component branch
// registry (entries 0 .. count-1) with its graph, 32-bit and with local ids,
// in the graph arena.  Workers claim instances through a device-side cursor
// and then share every node through the one worklist, so a hard instance
// is helped by workers whose own instances are done.  Instances never
// exchange anything else: each has its own bound, cover bitmap, node count
// and PVC stop bit.  The sequence pack -> init -> search -> cover lists is
// captured as a hipGraph and replayed while the batch geometry stays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "ctx.hpp"
#include "dev_common.hpp"
#include "internal.hpp"
#include "vc.h"

using namespace vc;

namespace {

// splitmix64 finaliser of an ordered pair: the symmetry test adds
// +h(v, w) for an entry v -> w with v < w and -h(w, v) for w -> v, so the
// sum over a symmetric graph is zero
__device__ __forceinline__ uint64_t pair_hash(uint32_t a, uint32_t b) {
    uint64_t x = ((uint64_t)a << 32) | b;
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Device-side check of a packed batch.  bad[i] bits: 1 offsets, 2 range or
// self-loop, 4 repeated entry; hs[i] the symmetry hash sum; *maxdeg the
// largest row.  64 consecutive rows of the packed batch per wave, one per
// lane; a row longer than 32 entries is checked by the whole wave.
__global__ void __launch_bounds__(256) k_batch_check(
    uint32_t count, const uint64_t* rbase, const uint32_t* n, const uint64_t* nnz,
    const uint64_t* offs_base, const uint64_t* cols_base, const uint32_t* offsets,
    const void* cols, uint32_t col_bytes, uint32_t* bad, unsigned long long* hs,
    uint32_t* maxdeg) {
    __shared__ uint32_t red[256];
    __shared__ uint32_t tbl_all[4 * ROWCHK_TBL];
    uint32_t* tbl = tbl_all + (threadIdx.x >> 6) * ROWCHK_TBL;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = gid; i < count; i += stride) {
        const uint32_t* off = offsets + offs_base[i];
        if (off[0] != 0u || (uint64_t)off[n[i]] != nnz[i]) atomicOr(&bad[i], 1u);
    }
    auto hash = [](uint32_t v, uint32_t w) -> uint64_t {
        return v < w ? pair_hash(v, w) : (uint64_t)0 - pair_hash(w, v);
    };
    const uint32_t l = threadIdx.x & 63u;
    uint32_t dmax = 0;
    const uint64_t rows = rbase[count];
    for (uint64_t base = (gid >> 6) << 6; base < rows; base += stride) {
        const uint64_t r = base + l;
        uint32_t i = 0, v = 0, ni = 0, o0 = 0, o1 = 0;
        bool longrow = false;
        if (r < rows) {
            uint32_t lo = 0, hi = count;  // largest i with rbase[i] <= r
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (rbase[mid] <= r) lo = mid;
                else hi = mid;
            }
            i = lo;
            v = (uint32_t)(r - rbase[i]);
            ni = n[i];
            const uint32_t* off = offsets + offs_base[i];
            o0 = off[v];
            o1 = off[v + 1];
            uint32_t flags = 0;
            if (o0 > o1 || (uint64_t)o1 > nnz[i]) {
                flags |= 1u;
            } else {
                const uint32_t d = o1 - o0;
                dmax = d > dmax ? d : dmax;
                longrow = d > 32u;
            }
            if (!longrow && !flags) {
                const uint64_t cb = cols_base[i];
                auto col = [&](uint32_t e) -> uint32_t {
                    return col_bytes == 2
                               ? (uint32_t)reinterpret_cast<const uint16_t*>(cols)[cb + e]
                               : reinterpret_cast<const uint32_t*>(cols)[cb + e];
                };
                uint64_t sum = 0;
                int64_t prev = -1;
                bool sorted = true;
                for (uint32_t e = o0; e < o1; ++e) {
                    const uint32_t w = col(e);
                    if (w >= ni || w == v) flags |= 2u;
                    if ((int64_t)w <= prev) sorted = false;
                    prev = (int64_t)w;
                    sum += hash(v, w);
                }
                if (!sorted)
                    for (uint32_t e = o0; e < o1; ++e)
                        for (uint32_t f = e + 1u; f < o1; ++f)
                            if (col(e) == col(f)) flags |= 4u;
                if (sum) atomicAdd(&hs[i], (unsigned long long)sum);
            }
            if (flags) atomicOr(&bad[i], flags);
        }
        uint64_t m = ballot(longrow);
        while (m) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t ij = shfl(i, j);
            const uint64_t cb = cols_base[ij];
            auto col = [&](uint32_t e) -> uint32_t {
                return col_bytes == 2 ? (uint32_t)reinterpret_cast<const uint16_t*>(cols)[cb + e]
                                      : reinterpret_cast<const uint32_t*>(cols)[cb + e];
            };
            uint64_t acc = 0;
            const uint32_t res = wave_row_check(shfl(v, j), shfl(ni, j), shfl(o0, j), shfl(o1, j),
                                                col, hash, tbl, &acc);
            acc = wave_sum64(acc);
            if (l == 0) {
                uint32_t f = 0;
                if (res & ROWCHK_ENTRY) f |= 2u;
                if (res & ROWCHK_REPEAT) f |= 4u;
                if (f) atomicOr(&bad[ij], f);
                if (acc) atomicAdd(&hs[ij], (unsigned long long)acc);
            }
        }
    }
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = std::max(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicMax(maxdeg, red[0]);
}

// fill a buffer with zeros (kernels, not memsets, so the batch launch can
// be captured)
__global__ void k_zero_u32(uint32_t* p, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t zero_u32(void* p, uint64_t words, hipStream_t s) {
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)blocks), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

struct BatchOut {
    std::vector<RegEntry> roots;
    std::vector<int> state;
    std::vector<uint64_t> nodes;
    std::vector<uint32_t> cnt;
    std::vector<uint32_t> cov;
    std::vector<uint64_t> cbase;
};

template <typename T>
hipError_t upload(vc::Pool& pool, vc::DevBuf& b, const T* src, size_t count, hipStream_t s) {
    hipError_t e = ensure(pool, b, sizeof(T) * (count ? count : 1));
    if (e) return e;
    if (!count) return hipSuccess;
    return hipMemcpyAsync(b.p, src, sizeof(T) * count, hipMemcpyHostToDevice, s);
}

// The whole batch: checks, plan, launch, results.  pvc: 0 MVC, 1 PVC with
// per-instance bounds k.
vc_status run_batch(vc_ctx* c, const vc_batch* b, int pvc, const uint32_t* k, BatchOut* out) {
    const double t0 = now_ms();
    vc_stats stv{};
    if (!b) return VC_EINVAL;
    if (b->col_bytes != 2 && b->col_bytes != 4) return VC_EINVAL;
    const uint32_t count = b->count;
    if (count == 0) {
        stv.ms_total = now_ms() - t0;
        c->last = stv;
        return VC_OK;
    }
    if (count >= (1u << 30)) return VC_ERANGE;
    if (!b->offs_base || !b->cols_base || !b->n || !b->nnz || !b->offsets) return VC_EINVAL;
    if (pvc && !k) return VC_EINVAL;
    const bool dev_in = (b->flags & VC_CSR_DEVICE) != 0;
    const bool skip = (c->opts.flags & VC_OPT_VALIDATE_SKIP) != 0;
    hipStream_t s = c->stream;

    // geometry: spans of the packed arrays, arena places, output bases
    uint64_t off_len = 0, col_len = 0, sum_n = 0, words = 0;
    uint32_t n_max = 0;
    std::vector<uint64_t> g_at(count), rbase(count + 1);
    out->cbase.assign(count, 0);
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t ni = b->n[i];
        const uint64_t mi = b->nnz[i];
        if (ni >= 0x7FFFFFFFu || mi >= (1ull << 32)) return VC_ERANGE;
        if (b->col_bytes == 2 && ni > 65536u) return VC_EINVAL;
        if (mi && !b->cols) return VC_EINVAL;
        off_len = std::max<uint64_t>(off_len, b->offs_base[i] + ni + 1u);
        col_len = std::max<uint64_t>(col_len, b->cols_base[i] + mi);
        rbase[i] = sum_n;
        out->cbase[i] = sum_n;
        sum_n += ni;
        g_at[i] = words;
        words += (ni + 1u + mi + 31u) & ~31ull;
        n_max = std::max(n_max, ni);
    }
    rbase[count] = sum_n;
    if (words >= (1ull << 32)) return VC_ERANGE;
    stv.n_input = (uint32_t)std::min<uint64_t>(sum_n, 0xFFFFFFFFu);

    // checks and the largest degree
    uint32_t dmax = 0;
    const uint32_t* d_off;
    const void* d_col;
    if (!dev_in) {
        for (uint32_t i = 0; i < count; ++i) {
            vc_csr gi{b->n[i], b->nnz[i], b->offsets + b->offs_base[i],
                      b->nnz[i] ? (const void*)((const char*)b->cols +
                                                b->cols_base[i] * b->col_bytes)
                                : nullptr,
                      b->col_bytes, 0u};
            if (!skip) {
                vc_status st = validate_host(&gi);
                if (st) return st;
            }
            for (uint32_t v = 0; v < gi.n; ++v)
                dmax = std::max(dmax, gi.offsets[v + 1] - gi.offsets[v]);
        }
        HIPCHK(upload(c->pool, c->in_off, b->offsets, off_len, s));
        HIPCHK(ensure(c->pool, c->in_col, (size_t)b->col_bytes * (col_len ? col_len : 1)));
        if (col_len)
            HIPCHK(hipMemcpyAsync(c->in_col.p, b->cols, (size_t)b->col_bytes * col_len,
                                  hipMemcpyHostToDevice, s));
        d_off = (const uint32_t*)c->in_off.p;
        d_col = c->in_col.p;
    } else {
        d_off = b->offsets;
        d_col = b->cols;
        vc_status o = order_after_default(c);
        if (o) return o;
    }
    HIPCHK(upload(c->pool, c->b_n, b->n, count, s));
    HIPCHK(upload(c->pool, c->b_nnz, b->nnz, count, s));
    HIPCHK(upload(c->pool, c->b_ob, b->offs_base, count, s));
    HIPCHK(upload(c->pool, c->b_cb, b->cols_base, count, s));
    HIPCHK(upload(c->pool, c->b_gat, g_at.data(), count, s));
    HIPCHK(upload(c->pool, c->b_cbase, out->cbase.data(), count, s));
    if (dev_in) {
        HIPCHK(upload(c->pool, c->b_rbase, rbase.data(), count + 1u, s));
        HIPCHK(ensure(c->pool, c->b_bad, 4ull * count + 4u));  // flags, then the max degree
        HIPCHK(ensure(c->pool, c->b_hs, 8ull * count));
        HIPCHK(zero_u32(c->b_bad.p, count + 1ull, s));
        HIPCHK(zero_u32(c->b_hs.p, 2ull * count, s));
        uint64_t blocks = (std::max<uint64_t>(sum_n, count) + 255u) / 256u;
        blocks = std::min<uint64_t>(std::max<uint64_t>(blocks, 1u), 2048u);
        uint32_t* badp = (uint32_t*)c->b_bad.p;
        hipLaunchKernelGGL(k_batch_check, dim3((uint32_t)blocks), dim3(256), 0, s, count,
                           (const uint64_t*)c->b_rbase.p, (const uint32_t*)c->b_n.p,
                           (const uint64_t*)c->b_nnz.p, (const uint64_t*)c->b_ob.p,
                           (const uint64_t*)c->b_cb.p, d_off, d_col, b->col_bytes, badp,
                           (unsigned long long*)c->b_hs.p, badp + count);
        HIPCHK(hipGetLastError());
        std::vector<uint32_t> bad(count + 1u);
        std::vector<uint64_t> hs(count);
        HIPCHK(hipMemcpyAsync(bad.data(), badp, 4ull * (count + 1u), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hs.data(), c->b_hs.p, 8ull * count, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        dmax = bad[count];
        if (!skip)
            for (uint32_t i = 0; i < count; ++i)
                if ((bad[i] & 7u) || hs[i]) return VC_EINVAL;
    }

    // plan (Sec. IV-D: the narrowest degree type that holds every degree)
    const uint32_t deg_bytes = dmax <= 254u ? 1u : (dmax <= 65534u ? 2u : 4u);
    const uint32_t n_pad = std::max<uint32_t>(64u, (n_max + 63u) & ~63u);
    LdsPlan lp;
    uint32_t gwords = 0, workers = 0;
    // two workers per CU by default: a batch's small instances leave LDS for
    // two, and the measured sweep (vc_autotune over workers, worklist size
    // and donation threshold) halved the 4,096-graph batch's time with them
    const uint32_t cus = (uint32_t)(c->cus > 0 ? c->cus : 1);
    vc_status pst = plan_workers(c, n_pad, deg_bytes, &lp, &gwords, &workers, 2u * cus);
    if (pst) return pst;
    const uint32_t slot_bytes = (uint32_t)sizeof(SlotHdr) + n_pad * deg_bytes + 16u;
    const uint32_t depth = n_max + n_max / 4u + 16u;
    const uint32_t wl_cap = c->opts.worklist_cap ? c->opts.worklist_cap
                                                 : std::max<uint32_t>(1024u, 4u * workers);
    // per-instance arrays, the worklist and the instance graphs come off the
    // top (pool mode); stacks take up to 1/2 of the rest, the registry 1/4
    const uint64_t fixed = (uint64_t)wl_cap * (slot_bytes + 8u) + sizeof(Ctl) + 4ull * words +
                           40ull * count + 4ull * sum_n + (64u << 10);
    const uint64_t budget = search_budget(c->opts, c->pool, fixed);
    const uint64_t wmax = std::max<uint64_t>(1u, (budget / 2) / ((uint64_t)depth * slot_bytes));
    workers = (uint32_t)std::min<uint64_t>(workers, wmax);
    const uint32_t bm_words = ((n_max + 31u) / 32u + 31u) & ~31u;
    const uint64_t reg_bytes_each = sizeof(RegEntry) + 4ull * std::max<uint32_t>(bm_words, 1u);
    uint64_t reg_cap = c->opts.registry_cap ? c->opts.registry_cap : (1u << 20);
    reg_cap = std::max<uint64_t>(reg_cap, (uint64_t)count + 64u);
    if (reg_cap * reg_bytes_each > budget / 4) {
        reg_cap = std::max<uint64_t>((budget / 4) / reg_bytes_each, (uint64_t)count + 64u);
        if (reg_cap * reg_bytes_each > budget / 2) return VC_ENOMEM;
    }
    const uint64_t arena_words = words + std::min<uint64_t>(budget / 16 / 4, 64ull << 20);
    stv.deg_bytes = deg_bytes;
    stv.max_degree_kernel = dmax;
    stv.n_kernel = n_max;
    stv.workers = workers;
    stv.slot_bytes = slot_bytes;
    stv.bitmap_bytes = 4u * bm_words;

    HIPCHK(ensure(c->pool, c->stacks, (size_t)workers * depth * slot_bytes));
    HIPCHK(ensure(c->pool, c->wl_slots, (size_t)wl_cap * slot_bytes));
    HIPCHK(ensure(c->pool, c->wl_seq, 8ull * wl_cap));
    HIPCHK(ensure(c->pool, c->ctl, sizeof(Ctl)));
    HIPCHK(ensure(c->pool, c->reg, sizeof(RegEntry) * reg_cap));
    HIPCHK(ensure(c->pool, c->bitmaps, 4ull * std::max<uint32_t>(bm_words, 1u) * reg_cap));
    HIPCHK(ensure(c->pool, c->arena, 4ull * arena_words));
    HIPCHK(ensure(c->pool, c->b_state, 4ull * count));
    HIPCHK(ensure(c->pool, c->b_nodes, 8ull * count));
    HIPCHK(ensure(c->pool, c->b_cnt, 4ull * count));
    HIPCHK(ensure(c->pool, c->b_cov, 4ull * std::max<uint64_t>(sum_n, 1u)));
    if (pvc) {
        std::vector<int> kk(count);
        for (uint32_t i = 0; i < count; ++i) kk[i] = (int)std::min<uint32_t>(k[i], INT_MAX - 1);
        HIPCHK(upload(c->pool, c->b_k, kk.data(), count, s));
    } else {
        HIPCHK(ensure(c->pool, c->b_k, 4ull * count));
    }

    SearchArgs a{};
    a.n = n_max;
    a.n_pad = n_pad;
    a.off = nullptr;
    a.col = nullptr;
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
    a.arena = (uint32_t*)c->arena.p;
    a.arena_words = arena_words;
    a.gcache_words = gwords;
    a.lds_L = lp.L;
    a.lds_Q = lp.Q;
    a.lds_R = lp.R;
    a.lds_VB = lp.VB;
    a.lds_PB = lp.PB;
    a.lds_MK = lp.MK;
    a.lds_G = lp.G;
    a.lds_bytes = lp.bytes;
    a.pvc = pvc;
    a.k = 0;
    a.flags = c->opts.flags;
    a.donate_slack = c->opts.donate_slack;
    // many instances keep the workers busy: up to 128 live vertices
    a.small_max = (c->opts.flags & VC_OPT_NO_SMALL) ? 0u
                  : std::min<uint32_t>(c->opts.small_max ? c->opts.small_max : 128u, 128u);
    a.donate_min = c->opts.donate_min ? c->opts.donate_min : 48u;
    a.strong_fences = (c->opts.flags & VC_OPT_STRONG_ORDER) ? 1u : 0u;
    a.node_limit = 0;
    a.watchdog_ticks =
        (uint64_t)c->wall_khz * (c->opts.watchdog_ms ? c->opts.watchdog_ms : 120000u);
    a.n_roots = count;
    a.batch = 1;
    a.inst_state = (int*)c->b_state.p;
    a.inst_nodes = (uint64_t*)c->b_nodes.p;
    a.inst_k = (const int*)c->b_k.p;
    a.inst_node_limit = c->opts.node_limit;

    BatchDesc d{};
    d.count = count;
    d.n = (const uint32_t*)c->b_n.p;
    d.nnz = (const uint64_t*)c->b_nnz.p;
    d.offs_base = (const uint64_t*)c->b_ob.p;
    d.cols_base = (const uint64_t*)c->b_cb.p;
    d.g_at = (const uint64_t*)c->b_gat.p;
    d.offsets = d_off;
    d.cols = d_col;
    d.col_bytes = b->col_bytes;
    d.inst_words = words;
    const uint64_t* cbase_d = (const uint64_t*)c->b_cbase.p;
    uint32_t* cov_d = (uint32_t*)c->b_cov.p;
    uint32_t* cnt_d = (uint32_t*)c->b_cnt.p;

    auto launch_all = [&]() -> hipError_t {
        hipError_t e = launch_batch_pack(a, d, s);
        if (!e) e = launch_batch_init(a, d, s);
        if (!e) e = launch_search(a, deg_bytes, workers, s);
        if (!e) e = launch_batch_cover(a, d, cbase_d, cov_d, cnt_d, s);
        return e;
    };
    HIPCHK(hipEventRecord(c->ev[3], s));
    const bool use_graph = !(c->opts.flags & VC_OPT_NO_GRAPH) && s != nullptr;
    if (use_graph) {
        // the captured launch depends on nothing but these arguments
        std::vector<unsigned char> key(sizeof(a) + sizeof(d) + 3 * sizeof(void*) + 8);
        unsigned char* kp = key.data();
        memcpy(kp, &a, sizeof(a));
        kp += sizeof(a);
        memcpy(kp, &d, sizeof(d));
        kp += sizeof(d);
        memcpy(kp, &cbase_d, sizeof(void*));
        kp += sizeof(void*);
        memcpy(kp, &cov_d, sizeof(void*));
        kp += sizeof(void*);
        memcpy(kp, &cnt_d, sizeof(void*));
        kp += sizeof(void*);
        memcpy(kp, &workers, 4);
        memcpy(kp + 4, &deg_bytes, 4);
        if (!c->batch_exec || key != c->batch_key) {
            if (c->batch_exec) {
                HIPCHK(hipGraphExecDestroy(c->batch_exec));
                c->batch_exec = nullptr;
            }
            c->batch_key.clear();
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            const hipError_t le = launch_all();
            const hipError_t ce = hipStreamEndCapture(s, &graph);
            if (le || ce) {
                if (graph) hipGraphDestroy(graph);
                HIPCHK(le ? le : ce);
            }
            const hipError_t ie = hipGraphInstantiate(&c->batch_exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (ie) c->batch_exec = nullptr;
            HIPCHK(ie);
            c->batch_key = key;
        }
        HIPCHK(hipGraphLaunch(c->batch_exec, s));
    } else {
        HIPCHK(launch_all());
    }
    HIPCHK(hipEventRecord(c->ev[4], s));

    out->roots.resize(count);
    out->state.resize(count);
    out->nodes.resize(count);
    out->cnt.resize(count);
    out->cov.resize(std::max<uint64_t>(sum_n, 1u));
    Ctl ctl;
    HIPCHK(hipMemcpyAsync(&ctl, c->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out->roots.data(), c->reg.p, sizeof(RegEntry) * count,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out->state.data(), c->b_state.p, 4ull * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out->nodes.data(), c->b_nodes.p, 8ull * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(out->cnt.data(), cnt_d, 4ull * count, hipMemcpyDeviceToHost, s));
    if (sum_n)
        HIPCHK(hipMemcpyAsync(out->cov.data(), cov_d, 4ull * sum_n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
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
    stv.stale_reads = ctl.stale;
    {
        const uint32_t first = (count + 1u) & ~1u;
        const uint32_t used = std::min<uint32_t>(ctl.reg_next, (uint32_t)reg_cap);
        stv.reg_entries = used > first ? used - first : 0u;
    }
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[3], c->ev[4]));
    stv.ms_search = ms;
    stv.ms_total = now_ms() - t0;
    c->last = stv;
    if (ctl.err) return (vc_status)ctl.err;
    return VC_OK;
}

// Lay the covers out densely for the caller.
void pack_covers(const BatchOut& o, uint32_t count, const uint32_t* take, uint32_t* covers,
                 uint64_t* cover_offs) {
    uint64_t at = 0;
    for (uint32_t i = 0; i < count; ++i) {
        cover_offs[i] = at;
        if (take[i]) {
            memcpy(covers + at, o.cov.data() + o.cbase[i], 4ull * take[i]);
            at += take[i];
        }
    }
    cover_offs[count] = at;
}

}  // namespace

extern "C" {

vc_status vc_min_batch(vc_ctx* c, const vc_batch* b, uint32_t* sizes, int32_t* inst_status,
                       uint32_t* covers, uint64_t* cover_offs) {
    if (!c || !b || !sizes) return VC_EINVAL;
    if ((covers == nullptr) != (cover_offs == nullptr)) return VC_EINVAL;
    if (server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    pool_reset(c);
    BatchOut o;
    vc_status st = run_batch(c, b, 0, nullptr, &o);
    if (st) return st;
    const uint32_t count = b->count;
    std::vector<uint32_t> take(count, 0);
    std::vector<int32_t> status(count, VC_OK);
    bool limited = false;
    for (uint32_t i = 0; i < count; ++i) {
        const RegEntry& r = o.roots[i];
        // internal invariant: the root bitmap holds a cover of size Best
        if (r.cover_size != r.best || o.cnt[i] != (uint32_t)r.best) return VC_EDEVICE;
        take[i] = o.cnt[i];
        if (o.state[i] & INST_LIMIT) {
            status[i] = VC_ETIMEDOUT;
            limited = true;
        }
    }
    if (limited && !inst_status) return VC_ETIMEDOUT;
    for (uint32_t i = 0; i < count; ++i) sizes[i] = (uint32_t)o.roots[i].best;
    if (inst_status) memcpy(inst_status, status.data(), 4ull * count);
    if (covers) pack_covers(o, count, take.data(), covers, cover_offs);
    return VC_OK;
}

vc_status vc_param_batch(vc_ctx* c, const vc_batch* b, const uint32_t* k, int* yes,
                         int32_t* inst_status, uint32_t* covers, uint64_t* cover_offs) {
    if (!c || !b || !k || !yes) return VC_EINVAL;
    if ((covers == nullptr) != (cover_offs == nullptr)) return VC_EINVAL;
    if (server_busy(c)) return VC_EAGAIN;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    pool_reset(c);
    BatchOut o;
    vc_status st = run_batch(c, b, 1, k, &o);
    if (st) return st;
    const uint32_t count = b->count;
    std::vector<uint32_t> take(count, 0);
    std::vector<int32_t> status(count, VC_OK);
    std::vector<int> ans(count, 0);
    bool limited = false;
    for (uint32_t i = 0; i < count; ++i) {
        const RegEntry& r = o.roots[i];
        if ((int64_t)r.cover_size <= (int64_t)k[i]) {
            // a cover within k was attained; the bitmap may be smaller
            if (o.cnt[i] > (uint32_t)r.cover_size) return VC_EDEVICE;
            ans[i] = 1;
            take[i] = o.cnt[i];
        } else if (o.state[i] & INST_LIMIT) {
            status[i] = VC_ETIMEDOUT;
            limited = true;
        }
    }
    if (limited && !inst_status) return VC_ETIMEDOUT;
    memcpy(yes, ans.data(), sizeof(int) * count);
    if (inst_status) memcpy(inst_status, status.data(), 4ull * count);
    if (covers) pack_covers(o, count, take.data(), covers, cover_offs);
    return VC_OK;
}

}  // extern "C"
