// serve.hip -- serving with continuous batching (vc_submit, vc_poll,
// vc_cancel).
//
// A server thread per context owns two streams: a side stream for the root
// steps of each request (validation, greedy bound, root reduction, induce;
// Sec. IV-B) and for publishing, and a search stream holding one resident
// persistent search launch in serving mode.  A request whose root steps do
// not decide it becomes an instance of that launch: its induced subgraph is
// copied into the launch's graph arena, its root registry entry is written,
// and the count of published instances is raised; an idle worker of the
// running kernel then claims it (as in a batch) while the other instances
// go on.  Admission is by footprint: an instance slot, arena room for the
// induced subgraph and pool room for the maps that turn its result back
// into original ids.  When a launch runs out of slots or room it drains and
// is launched again; the server closes it as soon as nothing is left, so it
// never sits on the GPU idle for long.  All device memory is allocated
// while no resident launch runs (freeing memory may wait for the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <initializer_list>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"
#include "internal.hpp"
#include "req_ring.hpp"
#include "root.hpp"
#include "vc.h"

namespace vc {

namespace {

__global__ void k_srv_zero(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
__global__ void k_srv_mark_list(const uint32_t* list, uint32_t cnt, uint32_t* flags) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        flags[list[i]] = 1u;
}
__global__ void k_srv_mark_bits(uint32_t np, const uint32_t* oldid, const uint32_t* bitmap,
                                uint32_t* flags) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
        if ((bitmap[i >> 5] >> (i & 31u)) & 1u) flags[oldid[i]] = 1u;
}
__global__ void k_srv_emit(uint32_t n, const uint32_t* flags, const uint32_t* pos, uint32_t* out) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (flags[v]) out[pos[v]] = v;
}

uint32_t grid_of(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(b, 1), 4096);
}

struct Req {
    uint64_t ticket = 0;
    int kind = VC_MIN;
    uint32_t k = 0;
    uint32_t n = 0;
    uint64_t nnz = 0;
    uint32_t col_bytes = 4;
    std::vector<uint32_t> off;
    std::vector<uint8_t> col;
    // root steps
    uint32_t np = 0, sroot = 0, gsize = 0, dmax = 0, nforced = 0;
    uint64_t nnzp = 0;
    int kbest0 = 0;
    uint64_t save_at = 0;  // pool words: forced list, greedy list, new -> old ids
    uint32_t slot = 0;
    bool admitted = false, cancel_sent = false;
    bool raw = false;  // admitted as given (no root steps; INST_GREEDY)
    bool small_rooted = false;  // at most RAW_N_MAX vertices, took the root steps
    // a device graph kept on the device: offsets at byte ring_at of the
    // server's request ring, columns at ring_at + ring_col
    bool on_ring = false;
    uint64_t ring_at = 0, ring_col = 0;
    // outcome
    std::atomic<bool> canceled{false};
    bool done = false;
    vc_result res{};
    std::vector<uint32_t> cover;
    double t_submit = 0, t_admit = 0;
};

}  // namespace

// Requests of at most this many vertices go to the resident search as they
// are (INST_GREEDY); larger ones take the root steps on the side stream
// (in one workgroup up to 4,096 vertices, over the whole chip above).  On
// the served stream 256 measured best: 1,024 and 64 gave 1.5-2x the p99.
constexpr uint32_t RAW_N_MAX = 256;
// device memory for served device graphs waiting for their root steps
constexpr uint64_t RING_BYTES = 64ull << 20;

struct Server {
    vc_ctx* c = nullptr;
    // shared with the API threads (under mu)
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t pending = 0;  // submitted and not finished
    std::deque<std::shared_ptr<Req>> incoming;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> table;
    std::thread th;
    bool resident_flag = false;  // a resident launch exists (read by server_busy)
    // pinned staging of vc_submit's device-graph copies (any caller thread)
    std::mutex sub_mu;
    uint8_t* sub_stage = nullptr;
    size_t sub_cap = 0;
    std::vector<void*> old_sub;
    // Device graphs larger than RAW_N_MAX stay on the device: vc_submit
    // copies them into this ring (device to device) and the root steps read
    // them there; pieces are taken in submission order and come back in any
    // order (ReqRing).  Under sub_mu.  Only a context whose buffers come
    // from hipMalloc has a ring (a caller's arena is reset by blocking calls).
    uint8_t* ring = nullptr;
    ReqRing ring_map;
    bool ring_take(uint64_t bytes, uint64_t* at) { return ring && ring_map.take(bytes, at); }
    void ring_give_locked(uint64_t at) { ring_map.give(at); }
    // a request's ring piece comes back once the side stream has finished
    // every read of it
    void ring_give(Req& r) {
        if (!r.on_ring) return;
        (void)hipStreamSynchronize(ss);
        std::lock_guard<std::mutex> g(sub_mu);
        ring_give_locked(r.ring_at);
        r.on_ring = false;
    }

    // owned by the server thread
    hipStream_t ss = nullptr, ks = nullptr;
    hipEvent_t ready = nullptr;
    std::deque<std::shared_ptr<Req>> queue;
    std::vector<std::shared_ptr<Req>> slot_req;
    bool resident = false;
    // how much the root steps shrink small requests: 1 for one they decide,
    // else the share of its vertices they remove (moving average over about
    // 16).  While no launch runs, a small request takes the root steps when
    // they have been removing most of such graphs (every 8th one takes them
    // anyway, to keep measuring), else it goes in as given
    double small_root_ema = 0.5;
    uint32_t small_seen = 0;
    uint32_t published = 0, active = 0;
    uint64_t host_next = 0, host_cap = 0, pool_next = 0, pool_cap = 0;
    double idle_since = 0;
    // root step buffers (capacity n_root vertices, nnz_root entries)
    uint64_t n_root = 0, nnz_root = 0;
    DevBuf in_off, in_col, rdeg, gdeg, gin, addf, newly, flags, newid, oldid, kdeg, koff, kcol,
        cover, scan_tmp, ctr, hsum, pool;
    // resident launch
    DevBuf stacks, wl_slots, wl_seq, ctl, reg, bitmaps, arena, st, nodes, kk, cancel;
    SearchArgs a{};
    uint32_t deg_bytes = 2, workers = 0;
    bool planned = false;
    std::vector<int> h_state;
    std::vector<uint64_t> h_nodes;
    // read-backs go through pinned memory (a copy into pageable memory can
    // wait for the resident launch to end): the mailbox, and a staging area
    // for longer results (a grown one keeps the old one until shutdown)
    HostMail* hm = nullptr;
    uint8_t* hstage = nullptr;
    size_t hstage_cap = 0;
    std::vector<void*> old_pinned;
    struct Piece {
        void* dst;
        const void* src;
        size_t bytes;
    };
    // copy device pieces to host memory on the side stream and wait
    vc_status fetch(std::initializer_list<Piece> ps) {
        size_t need = 0;
        for (const Piece& q : ps) need += (q.bytes + 15u) & ~(size_t)15u;
        if (need > hstage_cap) {
            const size_t cap = std::max<size_t>(need, std::max<size_t>(2 * hstage_cap, 1u << 20));
            void* np_ = nullptr;
            HIPCHK(hipHostMalloc(&np_, cap, hipHostMallocDefault));
            if (hstage) old_pinned.push_back(hstage);
            hstage = (uint8_t*)np_;
            hstage_cap = cap;
        }
        size_t at = 0;
        for (const Piece& q : ps) {
            if (q.bytes)
                HIPCHK(hipMemcpyAsync(hstage + at, q.src, q.bytes, hipMemcpyDeviceToHost, ss));
            at += (q.bytes + 15u) & ~(size_t)15u;
        }
        HIPCHK(hipStreamSynchronize(ss));
        at = 0;
        for (const Piece& q : ps) {
            if (q.bytes) memcpy(q.dst, hstage + at, q.bytes);
            at += (q.bytes + 15u) & ~(size_t)15u;
        }
        return VC_OK;
    }

    std::vector<DevBuf*> buffers() {
        return {&in_off, &in_col, &rdeg,   &gdeg,     &gin,    &addf,  &newly, &flags,
                &newid,  &oldid,  &kdeg,   &koff,     &kcol,   &cover, &scan_tmp, &ctr,
                &hsum,   &pool,   &stacks, &wl_slots, &wl_seq, &ctl,   &reg,   &bitmaps,
                &arena,  &st,     &nodes,  &kk,       &cancel};
    }
    vc_status plan();
    vc_status root_bufs(uint64_t n, uint64_t nnz, RootBufs* b);
    vc_status open_resident();
    vc_status resume_if_ended();
    hipEvent_t kend = nullptr;  // recorded after each search launch
    bool running = false;       // a search launch may still be running
    uint32_t epoch = 0;         // launches so far (SearchArgs::launch_epoch)
    vc_status close_resident();
    vc_status start(Req& r, bool raw_only);
    vc_status admit(Req& r, const uint32_t* gcsr, uint64_t words, const uint32_t* save,
                    uint64_t save_words);
    vc_status finish(Req& r, int state);
    vc_status check_done();
    double last_dump = 0;
    // An admitted instance whose FIN never comes although no node of the
    // launch exists any more (no busy worker, nothing queued, nothing left
    // to claim, the node count still) would keep the server from closing
    // the launch and from shutting down: after 200 ms of that state it is
    // answered with VC_EDEVICE and its slot is freed.  (An internal error:
    // its LiveNodes count did not return to 0.)
    double still_since = 0, last_still_check = 0;
    uint64_t still_nodes = ~0ull;
    vc_status check_stuck() {
        const double t = now_ms();
        if (t - last_still_check < 20.0) return VC_OK;
        last_still_check = t;
        Ctl h{};
        {
            const vc_status fs = fetch({{&h, a.ctl, sizeof(Ctl)}});
            if (fs) return fs;
        }
        const bool quiet = h.outstanding == 0 && h.wl_head == h.wl_tail &&
                           h.inst_next >= h.inst_avail && h.nodes == still_nodes;
        still_nodes = h.nodes;
        if (!quiet) {
            still_since = 0;
            return VC_OK;
        }
        if (still_since == 0) still_since = t;
        if (t - still_since < 200.0) return VC_OK;
        still_since = 0;
        debug_dump_now(h);
        for (uint32_t i = 0; i < published; ++i) {
            auto& p = slot_req[i];
            if (!p || p->done || (h_state[i] & INST_FIN)) continue;
            fprintf(stderr, "libvc serve: request %llu (slot %u) has no node left but did not "
                            "finish; answered with VC_EDEVICE\n",
                    (unsigned long long)p->ticket, i);
            p->res.status = VC_EDEVICE;
            --active;
            auto keep = p;
            p = nullptr;
            complete(*keep);
        }
        return VC_OK;
    }
    // VC_DEBUG_SERVE: every 5 s while instances are active, the state of
    // the resident launch and of every unanswered instance (stderr)
    void debug_dump() {
        const double t = now_ms();
        if (t - last_dump < 5000.0) return;
        last_dump = t;
        Ctl h{};
        if (fetch({{&h, a.ctl, sizeof(Ctl)}})) return;
        debug_dump_now(h);
    }
    void debug_dump_now(const Ctl& h) {
        const double t = now_ms();
        fprintf(stderr,
                "libvc serve: published %u active %u outstanding %d idle %d head %llu tail %llu "
                "next %u avail %u closed %d done %d err %d nodes %llu\n",
                published, active, h.outstanding, h.idle, (unsigned long long)h.wl_head,
                (unsigned long long)h.wl_tail, h.inst_next, h.inst_avail, h.closed, h.done, h.err,
                (unsigned long long)h.nodes);
        for (uint32_t i = 0; i < published; ++i) {
            auto& p = slot_req[i];
            if (!p || p->done) continue;
            RegEntry e{};
            if (fetch({{&e, a.reg + i, sizeof(e)}})) return;
            fprintf(stderr,
                    "libvc serve:   slot %u ticket %llu kind %d n %u np %u state %d nodes %llu "
                    "live %d best %d cover %d waited %.0f ms\n",
                    i, (unsigned long long)p->ticket, p->kind, p->n, p->np, h_state[i],
                    (unsigned long long)h_nodes[i], e.live, e.best, e.cover_size,
                    t - p->t_submit);
        }
    }
    void fail_active(vc_status e);
    void complete(Req& r);
    void loop();
};

namespace {

Server* get_server(vc_ctx* c) { return c->srv; }

}  // namespace

// The resident launch's fixed shape: degree arrays for serve_n_max
// vertices in 16-bit entries, the library's worker plan, one registry root
// per instance slot, and arena / pool regions for the instances' data.
vc_status Server::plan() {
    if (planned) return VC_OK;
    const uint32_t n_max = c->opts.serve_n_max ? c->opts.serve_n_max : 4096u;
    const uint32_t slots = c->opts.serve_slots ? c->opts.serve_slots : 4096u;
    const uint32_t n_pad = std::max<uint32_t>(64u, (n_max + 63u) & ~63u);
    LdsPlan lp;
    uint32_t gwords = 0, w = 0;
    vc_status pw = plan_workers(c, n_pad, deg_bytes, &lp, &gwords, &w);
    if (pw) return pw;
    // leave LDS on every CU for the root-step kernels of the side stream
    // (they take at most 16 KB per block: a kernel that cannot be placed
    // beside the resident search would wait for it forever)
    if (lp.bytes > 128u * 1024u && gwords > 4096u) {
        gwords -= std::min<uint32_t>(gwords - 4096u, (lp.bytes - 128u * 1024u + 3u) / 4u);
        lp = lds_plan(n_pad, deg_bytes, gwords);
    }
    workers = w;
    const uint32_t slot_bytes = (uint32_t)sizeof(SlotHdr) + n_pad * deg_bytes + 16u;
    const uint32_t depth = n_pad / 2u + 64u;
    const uint32_t wl_cap = c->opts.worklist_cap ? c->opts.worklist_cap
                                                 : std::max<uint32_t>(1024u, 4u * workers);
    const uint32_t bm_words = ((n_pad + 31u) / 32u + 31u) & ~31u;
    const uint64_t reg_cap = std::max<uint64_t>(
        c->opts.registry_cap ? c->opts.registry_cap : (1u << 19), (uint64_t)slots + 64u);
    host_cap = 32ull << 20;  // arena words for instance graphs
    const uint64_t arena_words = host_cap + (32ull << 20);
    pool_cap = 16ull << 20;
    a = SearchArgs{};
    a.n = n_max;
    a.n_pad = n_pad;
    a.slot_bytes = slot_bytes;
    a.stack_depth = depth;
    a.wl_cap = wl_cap;
    a.reg_cap = (uint32_t)reg_cap;
    a.bm_words = bm_words;
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
    a.pvc = 0;
    a.flags = c->opts.flags;
    a.donate_slack = c->opts.donate_slack;
    // many instances keep the workers busy: up to 128 live vertices
    a.small_max = (c->opts.flags & VC_OPT_NO_SMALL) ? 0u
                  : std::min<uint32_t>(c->opts.small_max ? c->opts.small_max : 128u, 128u);
    a.donate_min = c->opts.donate_min ? c->opts.donate_min : 48u;
    a.watchdog_ticks =
        (uint64_t)c->wall_khz * (c->opts.watchdog_ms ? c->opts.watchdog_ms : 120000u);
    a.n_roots = slots;
    a.batch = 1;
    a.serve = 1;
    a.strong_fences = (c->opts.flags & VC_OPT_STRONG_ORDER) ? 1u : 0u;
    {
        // a launch with nothing left ends at once (VC_SERVE_LINGER_US sets a
        // grace time): the root steps of requests that arrived meanwhile
        // run between launches
        const char* lu = getenv("VC_SERVE_LINGER_US");
        const uint64_t us = lu ? strtoull(lu, nullptr, 10) : 0ull;
        a.linger_ticks = (uint64_t)c->wall_khz * us / 1000u;
    }
    a.inst_node_limit = c->opts.node_limit;
    HIPCHK(ensure(c->pool, stacks, (size_t)workers * depth * slot_bytes));
    HIPCHK(ensure(c->pool, wl_slots, (size_t)wl_cap * slot_bytes));
    HIPCHK(ensure(c->pool, wl_seq, 8ull * wl_cap));
    HIPCHK(ensure(c->pool, ctl, sizeof(Ctl)));
    HIPCHK(ensure(c->pool, reg, sizeof(RegEntry) * reg_cap));
    HIPCHK(ensure(c->pool, bitmaps, 4ull * bm_words * reg_cap));
    HIPCHK(ensure(c->pool, arena, 4ull * arena_words));
    HIPCHK(ensure(c->pool, st, 4ull * slots));
    HIPCHK(ensure(c->pool, nodes, 8ull * slots));
    HIPCHK(ensure(c->pool, kk, 4ull * slots));
    HIPCHK(ensure(c->pool, cancel, 4ull * slots));
    HIPCHK(ensure(c->pool, pool, 4ull * pool_cap));
    a.stacks = (uint8_t*)stacks.p;
    a.wl_slots = (uint8_t*)wl_slots.p;
    a.wl_seq = (uint64_t*)wl_seq.p;
    a.ctl = (Ctl*)ctl.p;
    a.reg = (RegEntry*)reg.p;
    a.bitmaps = (uint32_t*)bitmaps.p;
    a.arena = (uint32_t*)arena.p;
    a.inst_state = (int*)st.p;
    a.inst_nodes = (uint64_t*)nodes.p;
    a.inst_k = (const int*)kk.p;
    a.inst_cancel = (const int*)cancel.p;
    slot_req.assign(slots, nullptr);
    h_state.assign(slots, 0);
    h_nodes.assign(slots, 0);
    planned = true;
    return VC_OK;
}

// Root step buffers for a graph of n vertices and nnz entries (grown only
// while no resident launch runs).
vc_status Server::root_bufs(uint64_t n, uint64_t nnz, RootBufs* b) {
    if (n > n_root || nnz > nnz_root) {
        if (resident) return VC_EAGAIN;
        n_root = std::max<uint64_t>(n, n_root);
        nnz_root = std::max<uint64_t>(nnz, nnz_root);
        const size_t n1 = n_root + 1;
        HIPCHK(ensure(c->pool, in_off, 4 * n1));
        HIPCHK(ensure(c->pool, in_col, 4 * std::max<uint64_t>(nnz_root, 1)));
        HIPCHK(ensure(c->pool, rdeg, 4 * n1));
        HIPCHK(ensure(c->pool, gdeg, 4 * n1));
        HIPCHK(ensure(c->pool, gin, n1));
        HIPCHK(ensure(c->pool, addf, n1));
        HIPCHK(ensure(c->pool, newly, n1));
        HIPCHK(ensure(c->pool, flags, 4 * (n1 + 1)));
        HIPCHK(ensure(c->pool, newid, 4 * (n1 + 1)));
        HIPCHK(ensure(c->pool, oldid, 4 * n1));
        HIPCHK(ensure(c->pool, kdeg, 4 * (n1 + 1)));
        HIPCHK(ensure(c->pool, koff, 4 * (n1 + 1)));
        HIPCHK(ensure(c->pool, kcol, 4 * std::max<uint64_t>(nnz_root, 1)));
        HIPCHK(ensure(c->pool, cover, 4 * n1));
        HIPCHK(ensure(c->pool, scan_tmp, 4 * (n1 / 2048 + 4)));
        HIPCHK(ensure(c->pool, ctr, CTR_COUNT * 4));
        HIPCHK(ensure(c->pool, hsum, 8 * HSUM_SLOTS));
    }
    b->rdeg = (uint32_t*)rdeg.p;
    b->gdeg = (uint32_t*)gdeg.p;
    b->gin = (uint8_t*)gin.p;
    b->addf = (uint8_t*)addf.p;
    b->newly = (uint8_t*)newly.p;
    b->flags = (uint32_t*)flags.p;
    b->newid = (uint32_t*)newid.p;
    b->oldid = (uint32_t*)oldid.p;
    b->kdeg = (uint32_t*)kdeg.p;
    b->koff = (uint32_t*)koff.p;
    b->kcol = kcol.p;
    b->cover = (uint32_t*)cover.p;
    b->scan_tmp = (uint32_t*)scan_tmp.p;
    b->ctr = (uint32_t*)ctr.p;
    b->hsum = (unsigned long long*)hsum.p;
    b->hm = hm->root;
    return VC_OK;
}

vc_status Server::open_resident() {
    if (resident) return VC_OK;
    vc_status s0 = plan();
    if (s0) return s0;
    published = active = 0;
    host_next = pool_next = 0;
    std::fill(slot_req.begin(), slot_req.end(), nullptr);
    HIPCHK(launch_serve_init(a, host_cap, ks));
    HIPCHK(hipEventRecord(ready, ks));
    HIPCHK(hipStreamWaitEvent(ss, ready, 0));
    // the search itself is launched once requests are admitted
    // (resume_if_ended)
    running = false;
    resident = true;
    {
        std::lock_guard<std::mutex> g(mu);
        resident_flag = true;
    }
    return VC_OK;
}

// Tell the resident launch that nothing more comes, wait for it to end.
// The launch ended by itself (nothing to do for a while): requests
// published since are claimed by launching it again on the same state.
vc_status Server::resume_if_ended() {
    if (!resident) return VC_OK;
    if (running) {
        const hipError_t q = hipEventQuery(kend);
        if (q == hipErrorNotReady) return VC_OK;
        HIPCHK(q);
        running = false;
    }
    // (requests admitted after the launch ended are claimed by the next one)
    if (active == 0) return VC_OK;
    vc_status cs = check_done();  // also fails the active requests on an error
    if (cs) return cs;
    if (!resident || active == 0) return VC_OK;
    a.launch_epoch = ++epoch;
    HIPCHK(launch_search(a, deg_bytes, workers, ks));
    HIPCHK(hipEventRecord(kend, ks));
    running = true;
    return VC_OK;
}

vc_status Server::close_resident() {
    if (!resident) return VC_OK;
    const int one = 1;
    HIPCHK(hipMemcpyAsync(&a.ctl->closed, &one, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipStreamSynchronize(ss));
    HIPCHK(hipStreamSynchronize(ks));
    running = false;
    Ctl h;
    {
        const vc_status fs = fetch({{&h, a.ctl, sizeof(Ctl)}});
        if (fs) return fs;
    }
    resident = false;
    {
        std::lock_guard<std::mutex> g(mu);
        resident_flag = false;
    }
    if (h.err) {
        fail_active((vc_status)h.err);
        return VC_OK;
    }
    // every admitted instance has finished before the launch could end
    return check_done();
}

void Server::complete(Req& r) {
    std::lock_guard<std::mutex> g(mu);
    if (r.done) return;
    r.res.ms_latency = now_ms() - r.t_submit;
    r.done = true;
    if (pending) --pending;
    cv.notify_all();
}

void Server::fail_active(vc_status e) {
    for (auto& p : slot_req) {
        if (p && p->admitted && !p->done) {
            p->res.status = e;
            complete(*p);
        }
        p = nullptr;
    }
    active = 0;
}

// Root steps of request r and, unless they decide it, its admission into
// the resident launch.  Returns VC_EAGAIN (nothing done) when r has to wait,
// and with raw_only (a launch is running) for every request that would need
// root steps.
vc_status Server::start(Req& r, bool raw_only) {
    const double t0 = now_ms();
    r.res.kind = r.kind;
    r.res.n = r.n;
    vc_csr g{r.n, r.nnz, r.off.data(), r.nnz ? (const void*)r.col.data() : nullptr, r.col_bytes, 0};
    if (r.on_ring)
        g = vc_csr{r.n, r.nnz, (const uint32_t*)(ring + r.ring_at), ring + r.ring_at + r.ring_col,
                   r.col_bytes, VC_CSR_DEVICE};
    const bool check = !(c->opts.flags & VC_OPT_VALIDATE_SKIP);
    if (r.n == 0 || r.nnz == 0) {
        // nothing to search; the offsets must still be all zero
        if (check) {
            bool ok = r.off[0] == 0u;
            for (uint32_t v = 0; ok && v < r.n; ++v) ok = r.off[v + 1] == 0u;
            if (!ok || r.nnz) {
                r.res.status = VC_EINVAL;
                return VC_OK;
            }
        }
        r.res.status = VC_OK;
        r.res.size = 0;
        r.res.yes = 1;
        return VC_OK;
    }
    // no free instance slot in the running launch: wait for it to drain
    if (resident && published >= a.n_roots) return VC_EAGAIN;
    {
        // A request that fits the resident search as it is goes in without
        // root steps: the worker that claims it runs the degree rules and a
        // greedy dive for its first bound, as for a batch's instances (no
        // side-stream work, so it is admitted at once)
        vc_status ps0 = plan();
        if (ps0) return ps0;
        const uint64_t words = ((uint64_t)r.n + 1 + r.nnz + 31) & ~31ull;
        bool go_raw = raw_only;
        if (!raw_only && r.n <= RAW_N_MAX) {
            const bool probe = (++small_seen & 7u) == 0;
            go_raw = small_root_ema < 0.5 && !probe;
        }
        if (go_raw && r.n <= a.n && r.n <= RAW_N_MAX && words <= host_cap) {
            if (check) {
                const vc_status vs = validate_host(&g);
                if (vs) {
                    r.res.status = vs;
                    return VC_OK;
                }
            }
            // the cover is assembled in the root step buffers: sized once
            // for every request of this path (they do not grow while a
            // launch is open)
            RootBufs rb;
            const vc_status bs = root_bufs(std::max<uint64_t>(r.n, RAW_N_MAX), 0, &rb);
            if (bs) return bs;
            std::vector<uint32_t> csr((size_t)words, 0u);
            memcpy(csr.data(), r.off.data(), 4ull * (r.n + 1));
            uint32_t* cc = csr.data() + r.n + 1;
            if (r.col_bytes == 2) {
                const uint16_t* c16 = (const uint16_t*)r.col.data();
                for (uint64_t e = 0; e < r.nnz; ++e) cc[e] = c16[e];
            } else {
                memcpy(cc, r.col.data(), 4ull * r.nnz);
            }
            std::vector<uint32_t> ids(r.n);
            for (uint32_t v = 0; v < r.n; ++v) ids[v] = v;
            r.raw = true;
            r.np = r.n;
            r.nnzp = r.nnz;
            r.sroot = r.nforced = r.gsize = 0;
            const int pvc = r.kind == VC_PARAM;
            const uint32_t kq = std::min<uint32_t>(r.k, 0x3FFFFFF0u);
            r.kbest0 = pvc ? (int)kq + 1 : (int)r.n;
            return admit(r, csr.data(), words, ids.data(), r.n);
        }
    }
    if (raw_only) return VC_EAGAIN;
    r.small_rooted = r.n <= RAW_N_MAX;
    RootBufs b;
    vc_status bs = root_bufs(r.n, r.nnz, &b);
    if (bs) return bs;
    RootGraph rg{r.n, r.nnz, (const uint32_t*)in_off.p, in_col.p, r.col_bytes};
    if (r.on_ring) {
        rg.off = (const uint32_t*)g.offsets;
        rg.col = g.cols;
    } else {
        HIPCHK(hipMemcpyAsync(in_off.p, r.off.data(), 4ull * (r.n + 1), hipMemcpyHostToDevice, ss));
        HIPCHK(hipMemcpyAsync(in_col.p, r.col.data(), (size_t)r.col_bytes * r.nnz,
                              hipMemcpyHostToDevice, ss));
    }
    hipLaunchKernelGGL(k_srv_zero, dim3(1), dim3(64), 0, ss, b.ctr, (uint64_t)CTR_COUNT);
    hipLaunchKernelGGL(k_srv_zero, dim3(1), dim3(64), 0, ss, (uint32_t*)b.hsum,
                       (uint64_t)(2 * HSUM_SLOTS));
    HIPCHK(hipGetLastError());
    if (check) {
        // the checks vc_validate applies to a device graph (kernels; the
        // symmetry test by a 64-bit hash of the unordered pairs)
        uint32_t bad = 0;
        HIPCHK(root_validate(rg, b.ctr, b.hsum, ss, hm->root, &bad));
        if (bad) {
            r.res.status = VC_EINVAL;
            return VC_OK;
        }
        hipLaunchKernelGGL(k_srv_zero, dim3(1), dim3(64), 0, ss, b.ctr, (uint64_t)CTR_COUNT);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(root_init(rg, b, ss));
    // the degree rules first (they need no bound), then the greedy bound on
    // what they leave, starting from the vertices they forced
    uint32_t rounds0 = 0;
    HIPCHK(root_reduce(rg, b, 0x3FFFFFFF, ss, 1u << 16, &rounds0));
    HIPCHK(root_greedy_rest(rg, b, ss));
    uint32_t grounds = 0;
    HIPCHK(root_greedy(rg, b, ss, &grounds));
    uint32_t ghdr[2] = {0, 0};
    {
        const vc_status fs = fetch({{&ghdr[0], b.ctr + CTR_GSIZE, 4}, {&ghdr[1], b.ctr + CTR_SROOT, 4}});
        if (fs) return fs;
    }
    r.gsize = ghdr[0] + ghdr[1];  // forced + greedy
    auto list_to_host = [&](int improved, uint32_t np_, const uint32_t* bm) -> vc_status {
        HIPCHK(root_cover(rg, b, np_, improved, bm, ss));
        uint32_t cnt = 0;
        vc_status fs = fetch({{&cnt, b.newid + r.n, 4}});
        if (fs) return fs;
        r.cover.resize(cnt);
        fs = fetch({{r.cover.data(), b.cover, 4ull * cnt}});
        if (fs) return fs;
        r.res.cover_len = cnt;
        return VC_OK;
    };
    const int pvc = r.kind == VC_PARAM;
    const uint32_t kq = std::min<uint32_t>(r.k, 0x3FFFFFF0u);
    if (pvc && r.gsize <= kq) {
        r.res.yes = 1;
        r.res.size = r.gsize;
        return list_to_host(0, 0, nullptr);
    }
    if (ghdr[0] == 0) {
        // the greedy took nothing: the degree rules left no edge, and the
        // vertices they forced are a minimum cover
        if (pvc) return VC_OK;  // no: |S_root| > k
        r.res.size = r.gsize;
        r.res.yes = 1;
        return list_to_host(0, 0, nullptr);
    }
    const int best0 = pvc ? (int)kq + 1 : (int)r.gsize;
    uint32_t rounds = 0;
    HIPCHK(root_reduce(rg, b, best0, ss, 1u << 16, &rounds));
    {
        const vc_status fs = fetch({{&r.sroot, b.ctr + CTR_SROOT, 4}});
        if (fs) return fs;
    }
    if ((int)r.sroot >= best0) {
        if (pvc) return VC_OK;  // no
        r.res.size = r.gsize;
        r.res.yes = 1;
        return list_to_host(0, 0, nullptr);
    }
    HIPCHK(root_induce_a(rg, b, ss));
    uint32_t hdr[2] = {0, 0};
    {
        const vc_status fs = fetch({{&hdr[0], b.newid + r.n, 4}, {&hdr[1], b.ctr + CTR_MAXDEG, 4}});
        if (fs) return fs;
    }
    r.np = hdr[0];
    r.dmax = hdr[1];
    r.kbest0 = best0 - (int)r.sroot;
    if (r.np == 0) {
        // the rules covered every edge
        r.res.yes = 1;
        vc_status ls = list_to_host(1, 0, nullptr);
        r.res.size = r.res.cover_len;
        return ls;
    }
    HIPCHK(root_induce_b(rg, b, r.np, 4, ss));
    uint32_t nz = 0;
    HIPCHK(root_cover(rg, b, 0, 1, nullptr, ss));
    {
        const vc_status fs = fetch({{&nz, b.koff + r.np, 4}, {&r.nforced, b.newid + r.n, 4}});
        if (fs) return fs;
    }
    r.nnzp = nz;
    // footprint in the running launch: the induced graph in the arena, the
    // forced list, the greedy list and the id map in the pool
    const uint64_t words = ((uint64_t)r.np + 1 + nz + 31) & ~31ull;
    const uint64_t pwords = ((uint64_t)r.nforced + r.gsize + r.np + 31) & ~31ull;
    vc_status ps0 = plan();
    if (ps0) return ps0;
    if (r.np > a.n || r.dmax > 65534u || words > host_cap || pwords > pool_cap) {
        // too large for the resident search: solved alone by the plain
        // path once the resident launch is closed
        if (resident && active) return VC_EAGAIN;
        vc_status cs = close_resident();
        if (cs) return cs;
        uint32_t size = 0, clen = 0;
        int yes = 0;
        r.cover.resize(r.n);
        vc_status ps = solve_one(c, &g, pvc, r.k, &size, &yes, r.cover.data(), &clen);
        r.res.status = ps;
        r.res.size = pvc ? clen : size;
        r.res.yes = pvc ? yes : 1;
        r.res.cover_len = clen;
        r.res.tree_nodes = c->last.tree_nodes;
        r.cover.resize(clen);
        return VC_OK;
    }
    if (resident && (host_next + words > host_cap || pool_next + pwords > pool_cap))
        return VC_EAGAIN;  // room comes back when the launch drains
    // keep what the cover needs later: the forced and greedy lists, the map
    // back to the graph's ids (the forced list is in b.cover now)
    vc_status os = open_resident();
    if (os) return os;
    uint32_t* pool_p = (uint32_t*)pool.p;
    r.save_at = pool_next;
    HIPCHK(hipMemcpyAsync(pool_p + r.save_at, b.cover, 4ull * r.nforced, hipMemcpyDeviceToDevice, ss));
    HIPCHK(root_cover(rg, b, 0, 0, nullptr, ss));
    HIPCHK(hipMemcpyAsync(pool_p + r.save_at + r.nforced, b.cover, 4ull * r.gsize,
                          hipMemcpyDeviceToDevice, ss));
    HIPCHK(hipMemcpyAsync(pool_p + r.save_at + r.nforced + r.gsize, b.oldid, 4ull * r.np,
                          hipMemcpyDeviceToDevice, ss));
    pool_next += pwords;
    // the instance: graph into the arena, root entry, cleared bitmap and
    // state, then the published count
    const uint32_t slot = published;
    const uint64_t g_at = host_next;
    uint32_t* ar = a.arena + g_at;
    HIPCHK(hipMemcpyAsync(ar, b.koff, 4ull * (r.np + 1), hipMemcpyDeviceToDevice, ss));
    if (nz) HIPCHK(hipMemcpyAsync(ar + r.np + 1, b.kcol, 4ull * nz, hipMemcpyDeviceToDevice, ss));
    host_next += words;
    RegEntry e{};
    e.best = r.kbest0;
    e.live = 1;
    e.up = -1;
    e.cover_size = INF;
    e.size = (int)r.np;
    e.view = (int)slot;
    e.vn = (int)r.np;
    e.g_at = (uint32_t)g_at;
    e.g_nnz = (int)nz;
    const int zero = 0, kslot = pvc ? (int)kq - (int)r.sroot : -1;
    const uint64_t zero64 = 0;
    HIPCHK(hipMemcpyAsync(a.reg + slot, &e, sizeof(e), hipMemcpyHostToDevice, ss));
    hipLaunchKernelGGL(k_srv_zero, dim3(1), dim3(256), 0, ss, a.bitmaps + (size_t)slot * a.bm_words,
                       (uint64_t)a.bm_words);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(a.inst_state + slot, &zero, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync(a.inst_nodes + slot, &zero64, 8, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync((int*)a.inst_k + slot, &kslot, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync((int*)a.inst_cancel + slot, &zero, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipStreamSynchronize(ss));
    const uint32_t avail = slot + 1;
    HIPCHK(hipMemcpyAsync(&a.ctl->inst_avail, &avail, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipStreamSynchronize(ss));
    published = avail;
    ++active;
    r.slot = slot;
    r.admitted = true;
    r.t_admit = now_ms();
    r.res.ms_queued = r.t_admit - r.t_submit;
    slot_req[slot] = nullptr;  // set by the caller (it holds the shared pointer)
    (void)t0;
    return VC_OK;
}

// Admission of request r from host data: its graph (words of off, col as
// 32-bit ids) into the arena, save_words ids into the pool (the map from the
// graph's vertices to the request's ids), its root entry, cleared bitmap and
// state, then the published count.  VC_EAGAIN when the running launch has no
// room left.
vc_status Server::admit(Req& r, const uint32_t* gcsr, uint64_t words, const uint32_t* save,
                        uint64_t save_words) {
    const uint64_t pwords = (save_words + 31) & ~31ull;
    if (resident && (host_next + words > host_cap || pool_next + pwords > pool_cap))
        return VC_EAGAIN;
    if (!resident && (words > host_cap || pwords > pool_cap)) return VC_ERANGE;
    vc_status os = open_resident();
    if (os) return os;
    uint32_t* pool_p = (uint32_t*)pool.p;
    r.save_at = pool_next;
    if (save_words)
        HIPCHK(hipMemcpyAsync(pool_p + r.save_at, save, 4ull * save_words, hipMemcpyHostToDevice,
                              ss));
    pool_next += pwords;
    const uint32_t slot = published;
    const uint64_t g_at = host_next;
    HIPCHK(hipMemcpyAsync(a.arena + g_at, gcsr, 4ull * (r.np + 1 + r.nnzp),
                          hipMemcpyHostToDevice, ss));
    host_next += words;
    RegEntry e{};
    e.best = r.kbest0;
    e.live = 1;
    e.up = -1;
    e.cover_size = INF;
    e.size = (int)r.np;
    e.view = (int)slot;
    e.vn = (int)r.np;
    e.g_at = (uint32_t)g_at;
    e.g_nnz = (int)r.nnzp;
    const int pvc = r.kind == VC_PARAM;
    const uint32_t kq = std::min<uint32_t>(r.k, 0x3FFFFFF0u);
    const int state0 = r.raw ? INST_GREEDY : 0, zero = 0;
    const int kslot = pvc ? (int)kq - (int)r.sroot : -1;
    const uint64_t zero64 = 0;
    HIPCHK(hipMemcpyAsync(a.reg + slot, &e, sizeof(e), hipMemcpyHostToDevice, ss));
    hipLaunchKernelGGL(k_srv_zero, dim3(1), dim3(256), 0, ss, a.bitmaps + (size_t)slot * a.bm_words,
                       (uint64_t)a.bm_words);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(a.inst_state + slot, &state0, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync(a.inst_nodes + slot, &zero64, 8, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync((int*)a.inst_k + slot, &kslot, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipMemcpyAsync((int*)a.inst_cancel + slot, &zero, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipStreamSynchronize(ss));
    const uint32_t avail = slot + 1;
    HIPCHK(hipMemcpyAsync(&a.ctl->inst_avail, &avail, 4, hipMemcpyHostToDevice, ss));
    HIPCHK(hipStreamSynchronize(ss));
    published = avail;
    ++active;
    r.slot = slot;
    r.admitted = true;
    r.t_admit = now_ms();
    r.res.ms_queued = r.t_admit - r.t_submit;
    slot_req[slot] = nullptr;  // set by the caller (it holds the shared pointer)
    return VC_OK;
}

// The result of admitted request r from its root entry (state: its bits).
vc_status Server::finish(Req& r, int state) {
    RegEntry e;
    {
        const vc_status fs = fetch({{&e, a.reg + r.slot, sizeof(e)}});
        if (fs) return fs;
    }
    r.res.tree_nodes = h_nodes[r.slot];
    if (r.canceled) {
        r.res.status = VC_ECANCELED;
        return VC_OK;
    }
    const int pvc = r.kind == VC_PARAM;
    const int kslot = pvc ? (int)std::min<uint32_t>(r.k, 0x3FFFFFF0u) - (int)r.sroot : -1;
    const bool attained = e.cover_size < INF && (pvc ? e.cover_size <= kslot : e.best < r.kbest0);
    if (!attained) {
        if ((state & INST_LIMIT)) {
            r.res.status = VC_ETIMEDOUT;
            if (pvc) return VC_OK;
        }
        if (pvc) return VC_OK;  // no
        if (r.raw) {
            // the worker's greedy dive attains a cover below |V| at once
            if (!(state & INST_LIMIT)) r.res.status = VC_EDEVICE;
            return VC_OK;
        }
        // nothing below the greedy bound: the greedy cover is minimum
        r.res.size = r.gsize;
        r.res.yes = 1;
        r.cover.resize(r.gsize);
        const uint32_t* gl = (const uint32_t*)pool.p + r.save_at + r.nforced;
        {
            const vc_status fs = fetch({{r.cover.data(), gl, 4ull * r.gsize}});
            if (fs) return fs;
        }
        r.res.cover_len = r.gsize;
        return VC_OK;
    }
    if (!pvc && (state & INST_LIMIT)) r.res.status = VC_ETIMEDOUT;
    // cover = forced vertices + the root bitmap mapped back (ascending)
    RootBufs b;
    vc_status bs = root_bufs(r.n, 0, &b);
    if (bs) return bs;
    const uint32_t* pl = (const uint32_t*)pool.p + r.save_at;
    hipLaunchKernelGGL(k_srv_zero, dim3(grid_of(r.n + 1)), dim3(256), 0, ss, b.flags,
                       (uint64_t)r.n + 1);
    if (r.nforced)
        hipLaunchKernelGGL(k_srv_mark_list, dim3(grid_of(r.nforced)), dim3(256), 0, ss, pl,
                           r.nforced, b.flags);
    hipLaunchKernelGGL(k_srv_mark_bits, dim3(grid_of(r.np)), dim3(256), 0, ss, r.np,
                       pl + r.nforced + r.gsize, a.bitmaps + (size_t)r.slot * a.bm_words, b.flags);
    HIPCHK(hipGetLastError());
    HIPCHK(scan_u32(b.flags, r.n, b.newid, b.scan_tmp, ss));
    hipLaunchKernelGGL(k_srv_emit, dim3(grid_of(r.n)), dim3(256), 0, ss, r.n, b.flags, b.newid,
                       b.cover);
    HIPCHK(hipGetLastError());
    uint32_t cnt = 0;
    vc_status fs = fetch({{&cnt, b.newid + r.n, 4}});
    if (fs) return fs;
    r.cover.resize(cnt);
    fs = fetch({{r.cover.data(), b.cover, 4ull * cnt}});
    if (fs) return fs;
    r.res.cover_len = cnt;
    r.res.yes = 1;
    r.res.size = pvc ? cnt : r.sroot + (uint32_t)e.best;
    // internal invariant: an MVC cover has exactly the reported size
    if (!pvc && cnt != r.res.size && !(state & INST_LIMIT)) r.res.status = VC_EDEVICE;
    return VC_OK;
}

// Read the instances' state; finish those that are answered.
vc_status Server::check_done() {
    if (!published || !active) return VC_OK;
    int ctl_done[2] = {0, 0};
    {
        const vc_status fs = fetch({{h_state.data(), a.inst_state, 4ull * published},
                                    {h_nodes.data(), a.inst_nodes, 8ull * published},
                                    {ctl_done, &a.ctl->done, 8}});
        if (fs) return fs;
    }
    for (uint32_t i = 0; i < published; ++i) {
        auto& p = slot_req[i];
        if (!p || p->done) continue;
        const int s = h_state[i];
        const bool answered = (s & INST_FIN) || (p->kind == VC_PARAM && (s & INST_STOP) &&
                                                 !(s & INST_LIMIT) && !p->canceled);
        if (!answered) {
            if (p->canceled && !p->cancel_sent) {
                const int one = 1;
                HIPCHK(hipMemcpyAsync((int*)a.inst_cancel + i, &one, 4, hipMemcpyHostToDevice, ss));
                HIPCHK(hipStreamSynchronize(ss));
                p->cancel_sent = true;
            }
            continue;
        }
        vc_status fs = finish(*p, s);
        if (fs) p->res.status = fs;
        if (s & INST_FIN) {
            --active;
            auto keep = p;
            p = nullptr;
            if (!keep->done) complete(*keep);
        } else if (!p->done) {
            complete(*p);  // a PVC yes: answered while its nodes drain
        }
    }
    if (getenv("VC_DEBUG_SERVE")) debug_dump();
    {
        vc_status ss_ = check_stuck();
        if (ss_) return ss_;
    }
    // a FIN that arrived for an already answered PVC instance frees its slot
    for (uint32_t i = 0; i < published; ++i) {
        auto& p = slot_req[i];
        if (p && p->done && (h_state[i] & INST_FIN)) {
            --active;
            p = nullptr;
        }
    }
    if (ctl_done[1]) {
        // the resident launch stopped on an error
        const vc_status e = (vc_status)ctl_done[1];
        HIPCHK(hipStreamSynchronize(ks));
        resident = false;
        {
            std::lock_guard<std::mutex> g(mu);
            resident_flag = false;
        }
        fail_active(e);
    }
    return VC_OK;
}

void Server::loop() {
    if (hipSetDevice(c->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        stop = true;
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> g(mu);
            while (!incoming.empty()) {
                queue.push_back(incoming.front());
                incoming.pop_front();
            }
            if (stop)
                for (auto& q : queue) q->canceled = true;  // not started: dropped
            if (stop && queue.empty() && active == 0) break;
        }
        bool progress = false;
        if (resident && active) {
            if (check_done()) fail_active(VC_EDEVICE);
        }
        if (!resident && active) {
            // the launch ended with admitted instances unfinished (an
            // internal error): answer them rather than wait for ever
            fprintf(stderr, "libvc serve: %u admitted requests unfinished after their launch "
                            "ended; answered with VC_EDEVICE\n", active);
            fail_active(VC_EDEVICE);
            progress = true;
        }
        // Requests start between launches: while no search launch runs, the
        // root steps of the queued requests run one after another and the
        // ones they do not decide are admitted; then one launch searches
        // them all.  (Root steps issued while a launch runs were measured to
        // wait for its end, so they are not issued then.)  Requests that go
        // in as given need no root steps: they join a running launch, in
        // queue order, up to the first request that needs them.
        bool busy = false;
        if (resident && running) {
            const hipError_t q = hipEventQuery(kend);
            busy = q == hipErrorNotReady;
        }
        for (uint32_t taken = 0; taken < 64u; ++taken) {
            {
                // requests that arrived during the last root steps join
                std::lock_guard<std::mutex> g(mu);
                while (!incoming.empty()) {
                    queue.push_back(incoming.front());
                    incoming.pop_front();
                }
                if (stop)
                    for (auto& q : queue) q->canceled = true;
            }
            if (queue.empty()) break;
            auto r = queue.front();
            if (r->canceled) {
                queue.pop_front();
                ring_give(*r);
                r->res.status = VC_ECANCELED;
                complete(*r);
                progress = true;
                continue;
            }
            const vc_status s = start(*r, busy);
            if (s == VC_EAGAIN) {
                // waits for room; a launch with nothing active is closed
                // so the next one starts empty
                if (!busy && resident && active == 0) {
                    close_resident();
                    progress = true;
                }
                break;
            }
            queue.pop_front();
            ring_give(*r);
            progress = true;
            if (r->small_rooted && !s && r->res.status == VC_OK)
                small_root_ema += ((r->admitted ? 1.0 - (double)r->np / r->n : 1.0) -
                                   small_root_ema) / 16.0;
            if (s) r->res.status = s;
            if (r->admitted && !s) slot_req[r->slot] = r;
            else complete(*r);
        }
        if (resident && resume_if_ended()) fail_active(VC_EDEVICE);
        if (resident && active == 0 && queue.empty()) {
            // nothing left: end the resident launch after a short grace
            if (idle_since == 0) idle_since = now_ms();
            if (now_ms() - idle_since > 2.0 || stop) {
                close_resident();
                idle_since = 0;
            }
        } else {
            idle_since = 0;
        }
        if (!progress) {
            std::unique_lock<std::mutex> g(mu);
            cv.wait_for(g, std::chrono::microseconds(50), [&] { return !incoming.empty() || stop; });
        }
    }
    close_resident();
}

void server_forget_buffers(vc_ctx* c) {
    Server* s = get_server(c);
    if (!s) return;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->pending > 0 || s->resident_flag) return;  // callers checked server_busy
    for (DevBuf* b : s->buffers()) forget(*b);
    s->planned = false;
    s->n_root = s->nnz_root = 0;
}

bool server_busy(vc_ctx* c) {
    Server* s = get_server(c);
    if (!s) return false;
    std::lock_guard<std::mutex> g(s->mu);
    return s->pending > 0 || s->resident_flag;
}

void server_shutdown(vc_ctx* c) {
    Server* s = get_server(c);
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // requests not yet started are cancelled
        for (auto& r : s->incoming) r->canceled = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    for (DevBuf* b : s->buffers()) release(*b);
    if (s->ring) (void)hipFree(s->ring);
    if (s->ready) hipEventDestroy(s->ready);
    if (s->kend) hipEventDestroy(s->kend);
    if (s->ss) hipStreamDestroy(s->ss);
    if (s->ks) hipStreamDestroy(s->ks);
    host_mail_free(s->hm);
    for (void* p : s->old_pinned) hipHostFree(p);
    if (s->hstage) hipHostFree(s->hstage);
    for (void* p : s->old_sub) hipHostFree(p);
    if (s->sub_stage) hipHostFree(s->sub_stage);
    delete s;
    c->srv = nullptr;
}

}  // namespace vc

using namespace vc;

extern "C" {

vc_status vc_submit(vc_ctx* c, const vc_csr* g, int kind, uint32_t k, uint64_t* ticket) {
    if (!c || !ticket) return VC_EINVAL;
    if (kind != VC_MIN && kind != VC_PARAM) return VC_EINVAL;
    vc_status st = check_args(g);
    if (st) return st;
    if (hipSetDevice(c->device) != hipSuccess) return VC_EDEVICE;
    auto r = std::make_shared<Req>();
    r->kind = kind;
    r->k = k;
    r->n = g->n;
    r->nnz = g->nnz;
    r->col_bytes = g->col_bytes;
    static std::mutex create_mu;
    {
        std::lock_guard<std::mutex> cg(create_mu);
        if (!c->srv) {
            Server* s = new (std::nothrow) Server();
            if (!s) return VC_ENOMEM;
            s->c = c;
            if (hipStreamCreateWithFlags(&s->ss, hipStreamNonBlocking) != hipSuccess ||
                hipStreamCreateWithFlags(&s->ks, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s->kend, hipEventDisableTiming) != hipSuccess ||
                host_mail(&s->hm) != hipSuccess) {
                if (s->ready) (void)hipEventDestroy(s->ready);
                if (s->kend) (void)hipEventDestroy(s->kend);
                if (s->ss) (void)hipStreamDestroy(s->ss);
                if (s->ks) (void)hipStreamDestroy(s->ks);
                host_mail_free(s->hm);
                delete s;
                return VC_EDEVICE;
            }
            if (!c->pool.base) {
                // the request ring (without it device graphs go through the host)
                void* rp = nullptr;
                if (hipMalloc(&rp, RING_BYTES) == hipSuccess) {
                    s->ring = (uint8_t*)rp;
                    s->ring_map.reset(RING_BYTES);
                } else {
                    (void)hipGetLastError();
                }
            }
            c->srv = s;
            s->th = std::thread([s] { s->loop(); });
        }
    }
    Server* s = c->srv;
    // the request keeps its own copy: the caller may free the graph now.  A
    // device graph is read after the work queued before on the caller's
    // stream (the default stream when the context has its own), through
    // pinned staging memory.
    const size_t ob = 4ull * (g->n + 1), cb = (size_t)g->col_bytes * g->nnz;
    hipStream_t cs = c->own_stream ? nullptr : c->stream;
    if (g->flags & VC_CSR_DEVICE && g->n > RAW_N_MAX && g->nnz) {
        // into the request ring when it has room
        std::lock_guard<std::mutex> sg(s->sub_mu);
        const uint64_t colat = (ob + 255u) & ~(uint64_t)255u;
        uint64_t at = 0;
        if (s->ring_take(colat + cb, &at)) {
            if (hipMemcpyAsync(s->ring + at, g->offsets, ob, hipMemcpyDeviceToDevice, cs) != hipSuccess ||
                hipMemcpyAsync(s->ring + at + colat, g->cols, cb, hipMemcpyDeviceToDevice, cs) !=
                    hipSuccess ||
                hipStreamSynchronize(cs) != hipSuccess) {
                s->ring_give_locked(at);
                return VC_EDEVICE;
            }
            r->on_ring = true;
            r->ring_at = at;
            r->ring_col = colat;
        }
    }
    if (r->on_ring) {
        // on the device already
    } else if (g->flags & VC_CSR_DEVICE) {
        r->off.resize((size_t)g->n + 1);
        r->col.resize(cb);
        std::lock_guard<std::mutex> sg(s->sub_mu);
        const size_t need = ((ob + 15u) & ~(size_t)15u) + cb;
        if (need > s->sub_cap) {
            void* np_ = nullptr;
            const size_t cap = std::max<size_t>(need, std::max<size_t>(2 * s->sub_cap, 1u << 20));
            if (hipHostMalloc(&np_, cap, hipHostMallocDefault) != hipSuccess) return VC_ENOMEM;
            if (s->sub_stage) s->old_sub.push_back(s->sub_stage);
            s->sub_stage = (uint8_t*)np_;
            s->sub_cap = cap;
        }
        uint8_t* st0 = s->sub_stage;
        uint8_t* st1 = st0 + ((ob + 15u) & ~(size_t)15u);
        if (hipMemcpyAsync(st0, g->offsets, ob, hipMemcpyDeviceToHost, cs) != hipSuccess)
            return VC_EDEVICE;
        if (cb && hipMemcpyAsync(st1, g->cols, cb, hipMemcpyDeviceToHost, cs) != hipSuccess)
            return VC_EDEVICE;
        if (hipStreamSynchronize(cs) != hipSuccess) return VC_EDEVICE;
        memcpy(r->off.data(), st0, ob);
        if (cb) memcpy(r->col.data(), st1, cb);
    } else {
        r->off.resize((size_t)g->n + 1);
        r->col.resize(cb);
        memcpy(r->off.data(), g->offsets, ob);
        if (g->nnz) memcpy(r->col.data(), g->cols, cb);
    }
    r->t_submit = now_ms();
    std::lock_guard<std::mutex> gl(s->mu);
    if (s->stop) {
        if (r->on_ring) {
            std::lock_guard<std::mutex> sg(s->sub_mu);
            s->ring_give_locked(r->ring_at);
        }
        return VC_ECANCELED;
    }
    r->ticket = s->next_ticket++;
    s->table[r->ticket] = r;
    s->incoming.push_back(r);
    ++s->pending;
    *ticket = r->ticket;
    s->cv.notify_all();
    return VC_OK;
}

vc_status vc_poll(vc_ctx* c, uint64_t ticket, vc_result* out, uint32_t* cover) {
    if (!c || !out) return VC_EINVAL;
    Server* s = c->srv;
    if (!s) return VC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return VC_EINVAL;
    Req& r = *it->second;
    if (!r.done) return VC_EAGAIN;
    *out = r.res;
    if (cover && r.res.cover_len) memcpy(cover, r.cover.data(), 4ull * r.res.cover_len);
    const vc_status rs = r.res.status == VC_ECANCELED ? VC_ECANCELED : VC_OK;
    s->table.erase(it);
    return rs;
}

vc_status vc_cancel(vc_ctx* c, uint64_t ticket) {
    if (!c) return VC_EINVAL;
    Server* s = c->srv;
    if (!s) return VC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return VC_EINVAL;
    it->second->canceled = true;
    s->cv.notify_all();
    return VC_OK;
}

}  // extern "C"
