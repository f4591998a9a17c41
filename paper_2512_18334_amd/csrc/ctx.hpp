// ctx.hpp -- the solver context and host helpers shared by the host
// runtime files of libvc.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <vector>

#include "internal.hpp"
#include "vc.h"

namespace vc {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool pooled = false;  // carved from a fixed pool (never freed one by one)
};

// A fixed region of device memory that a context's buffers are carved from
// instead of hipMalloc: a caller's arena (vc_ctx_create) or the library's
// static scratch (vc_min_static).  Carving is a bump of `used`; a buffer
// that has to grow takes a new region and leaves its old one unused until
// the pool is reset, which the blocking entry points do before they start
// (every buffer of the context is then forgotten).
struct Pool {
    uint8_t* base = nullptr;  // null: buffers come from hipMalloc
    size_t cap = 0;
    size_t used = 0;
    bool poison = false;  // VC_OPT_POISON: fill new buffers with 0xA7
};

inline hipError_t poison_fill(const Pool& pool, void* p, size_t bytes) {
    if (!pool.poison) return hipSuccess;
    hipError_t e = hipMemset(p, 0xA7, bytes);
    return e ? e : hipDeviceSynchronize();
}

// grow b to at least `bytes` (contents are not kept)
inline hipError_t ensure(Pool& pool, DevBuf& b, size_t bytes) {
    if (bytes <= b.cap && b.p) return hipSuccess;
    size_t want = bytes < 256 ? 256 : bytes;
    want = (want + 4095) & ~(size_t)4095;
    if (pool.base) {
        const size_t at = (pool.used + 255) & ~(size_t)255;
        if (at > pool.cap || want > pool.cap - at) return hipErrorOutOfMemory;
        b.p = pool.base + at;
        b.cap = want;
        b.pooled = true;
        pool.used = at + want;
        return poison_fill(pool, b.p, want);
    }
    if (b.p) {
        hipError_t e = b.pooled ? hipSuccess : hipFree(b.p);
        if (e) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e) return e;
    b.cap = want;
    b.pooled = false;
    return poison_fill(pool, b.p, want);
}

// drop a buffer without freeing it (pooled buffers only)
inline void forget(DevBuf& b) {
    b.p = nullptr;
    b.cap = 0;
    b.pooled = false;
}

// release a buffer that came from hipMalloc
inline void release(DevBuf& b) {
    if (b.p && !b.pooled) hipFree(b.p);
    forget(b);
}

// Bytes a search plan may use: the caller's budget (default 48 GiB) and, in
// pool mode, no more than the pool has left once `reserve` bytes are set
// aside.
inline uint64_t search_budget(const vc_opts& o, const Pool& pool, uint64_t reserve) {
    uint64_t b = o.hbm_budget ? o.hbm_budget : (48ull << 30);
    if (pool.base) {
        const uint64_t left = pool.cap > pool.used ? pool.cap - pool.used : 0;
        const uint64_t avail = left > reserve ? left - reserve : 0;
        b = b < avail ? b : avail;
    }
    return b;
}

inline double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

inline vc_status hip_status(hipError_t e) {
    if (e == hipErrorOutOfMemory) return VC_ENOMEM;
    return VC_EDEVICE;
}

}  // namespace vc

namespace vc {
// A host-side consistency check of a search's result failed: VC_EDEVICE,
// named on stderr under VC_DEBUG.
inline vc_status broken(const char* what) {
    if (getenv("VC_DEBUG")) fprintf(stderr, "libvc: internal check failed: %s\n", what);
    return VC_EDEVICE;
}
}  // namespace vc

#define HIPCHK(x)                                                                 \
    do {                                                                          \
        hipError_t _e = (x);                                                      \
        if (_e != hipSuccess) {                                                   \
            if (getenv("VC_DEBUG"))                                               \
                fprintf(stderr, "libvc: %s failed: %s\n", #x, hipGetErrorString(_e)); \
            return vc::hip_status(_e);                                            \
        }                                                                         \
    } while (0)

namespace vc {
struct Server;
}

namespace vc {
// Pinned host memory for the small read-backs of a call: a copy into
// pageable memory is staged by the runtime and can wait until every kernel
// on the device has finished (a resident search launch included); a copy
// into pinned memory is a plain transfer on its stream.
struct HostMail {
    uint32_t root[16];  // RootBufs::hm
    uint32_t ghdr[2];
    uint32_t hdr[2];
    uint32_t sroot, cnt, nz, crown_removed;
    uint32_t w[8];      // general words
    Ctl ctl;
    RegEntry reg0;
};
hipError_t host_mail(HostMail** out);
void host_mail_free(HostMail* m);
}  // namespace vc

struct vc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    vc_opts opts{};
    vc_stats last{};
    int cus = 0;
    size_t lds_max = 0;
    int wall_khz = 100000;  // wall_clock64() rate
    // input copies (host CSR) and root buffers
    vc::DevBuf in_off, in_col;
    vc::DevBuf rdeg, gdeg, gin, addf, newly, flags, newid, oldid, kdeg, koff, kcol, cover,
        scan_tmp, ctr, hsum, crown;
    // search buffers
    vc::DevBuf stacks, wl_slots, wl_seq, ctl, reg, bitmaps, arena, hl;
    // batch buffers: descriptors, per-instance state and results
    vc::DevBuf b_n, b_nnz, b_ob, b_cb, b_gat, b_rbase, b_cbase, b_k, b_state, b_nodes, b_bad,
        b_hs, b_cnt, b_cov;
    // the captured batch launch and the arguments it was captured with
    hipGraphExec_t batch_exec = nullptr;
    std::vector<unsigned char> batch_key;
    // serving (vc_submit): created on the first request
    vc::Server* srv = nullptr;
    hipEvent_t ev[6] = {};
    // enumeration of minimal covers (vc_param_enum)
    vc::DevBuf en[13];
    // a caller's arena (vc_ctx_create), else buffers come from hipMalloc
    vc::Pool pool;
    // the context that vc_min_static runs on: same device, stream, events
    // and options, with its pool over the library's static scratch
    vc_ctx* scratch_ctx = nullptr;
    bool shared_events = false;  // events (and the mailbox) belong to another context
    vc::HostMail* hm = nullptr;  // pinned read-back words of this context's calls
    bool wait_default = false;   // own stream: device inputs wait for the default stream
};

namespace vc {
struct RootGraph;
// Place a graph on the device (uploading a host CSR) and validate it.
vc_status stage_input(vc_ctx* c, const vc_csr* g, RootGraph* rg);
// Exact host-side check of a host CSR against the rules stated in vc.h.
vc_status validate_host(const vc_csr* g);
vc_status check_args(const vc_csr* g);
uint32_t registry_open_entries(const std::vector<RegEntry>& ents, uint32_t first,
                               uint32_t* parents, uint32_t* max_depth);
// want: the worker count to plan for when vc_opts.workers is 0 (0: one per CU)
vc_status plan_workers(vc_ctx* c, uint32_t n_pad, uint32_t deg_bytes, LdsPlan* lp,
                       uint32_t* gwords, uint32_t* workers, uint32_t want = 0);
// the same with the lists in HBM (hl_bytes per worker), for nodes whose
// lists do not fit LDS
vc_status plan_workers_hl(vc_ctx* c, uint32_t n_pad, uint32_t deg_bytes, LdsPlan* lp,
                          uint32_t* gwords, uint32_t* workers, uint64_t* hl_bytes);
// one blocking solve on the context's own buffers and stream (vc_min and
// vc_param; also the server for requests too large for its resident search)
vc_status solve_one(vc_ctx* c, const vc_csr* g, int pvc, uint32_t k, uint32_t* size, int* yes,
                    uint32_t* cover, uint32_t* cover_len);
// serving: true while requests are in flight (other solves must wait)
bool server_busy(vc_ctx* c);
// pool mode: forget the server's buffers (it is idle) so the pool can be reset
void server_forget_buffers(vc_ctx* c);
// pool mode: forget every buffer of the context and reset its pool (called
// by the blocking entry points before they start; no-op without a pool)
void pool_reset(vc_ctx* c);
// own stream: order the context's stream after the legacy default stream
// before device inputs are read
vc_status order_after_default(vc_ctx* c);
// stop the server thread and its resident kernel (context teardown)
void server_shutdown(vc_ctx* c);
}  // namespace vc
