// ctx.hpp -- the solver context and host helpers shared by the host
// runtime files of libvc.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.hpp"
#include "vc.h"

namespace vc {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// grow b to at least `bytes` (contents are not kept)
inline hipError_t ensure(DevBuf& b, size_t bytes) {
    if (bytes <= b.cap && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    want = (want + 4095) & ~(size_t)4095;
    hipError_t e = hipMalloc(&b.p, want);
    if (e) return e;
    b.cap = want;
    return hipSuccess;
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
    vc::DevBuf stacks, wl_slots, wl_seq, ctl, reg, bitmaps, arena;
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
};

namespace vc {
struct RootGraph;
// Place a graph on the device (uploading a host CSR) and validate it.
vc_status stage_input(vc_ctx* c, const vc_csr* g, RootGraph* rg);
// Exact host-side check of a host CSR against the rules stated in vc.h.
vc_status validate_host(const vc_csr* g);
vc_status check_args(const vc_csr* g);
vc_status plan_workers(vc_ctx* c, uint32_t n_pad, uint32_t deg_bytes, LdsPlan* lp,
                       uint32_t* gwords, uint32_t* workers);
// one blocking solve on the context's own buffers and stream (vc_min and
// vc_param; also the server for requests too large for its resident search)
vc_status solve_one(vc_ctx* c, const vc_csr* g, int pvc, uint32_t k, uint32_t* size, int* yes,
                    uint32_t* cover, uint32_t* cover_len);
// serving: true while requests are in flight (other solves must wait)
bool server_busy(vc_ctx* c);
// stop the server thread and its resident kernel (context teardown)
void server_shutdown(vc_ctx* c);
}  // namespace vc
