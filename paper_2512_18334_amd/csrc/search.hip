// search.hip -- launchers of the persistent search (one object per
// degree-array type, search_deg.hip) and the set-up kernels of batches and
// serving.
#include "dev_common.hpp"
#include "internal.hpp"
#include "vc.h"

namespace vc {

#define VC_DECL(sfx)                                                                  \
    hipError_t launch_search_##sfx(const SearchArgs& a, uint32_t workers, hipStream_t st); \
    hipError_t search_occupancy_##sfx(uint32_t lds_bytes, int* bpc);
VC_DECL(d1)
VC_DECL(d2)
VC_DECL(d4)
VC_DECL(d1h)
VC_DECL(d2h)
VC_DECL(d4h)
#undef VC_DECL
hipError_t launch_search_init_d1(const SearchArgs& a, int best0, const uint32_t* kdeg,
                                 uint32_t blocks, hipStream_t st);
hipError_t launch_search_init_d2(const SearchArgs& a, int best0, const uint32_t* kdeg,
                                 uint32_t blocks, hipStream_t st);
hipError_t launch_search_init_d4(const SearchArgs& a, int best0, const uint32_t* kdeg,
                                 uint32_t blocks, hipStream_t st);

hipError_t launch_search(const SearchArgs& a, uint32_t deg_bytes, uint32_t workers,
                         hipStream_t st) {
    if (a.hl) {
        if (deg_bytes == 1) return launch_search_d1h(a, workers, st);
        if (deg_bytes == 2) return launch_search_d2h(a, workers, st);
        return launch_search_d4h(a, workers, st);
    }
    if (deg_bytes == 1) return launch_search_d1(a, workers, st);
    if (deg_bytes == 2) return launch_search_d2(a, workers, st);
    return launch_search_d4(a, workers, st);
}

hipError_t search_occupancy(uint32_t deg_bytes, uint32_t lds_bytes, int* bpc, bool hl) {
    if (hl) {
        if (deg_bytes == 1) return search_occupancy_d1h(lds_bytes, bpc);
        if (deg_bytes == 2) return search_occupancy_d2h(lds_bytes, bpc);
        return search_occupancy_d4h(lds_bytes, bpc);
    }
    if (deg_bytes == 1) return search_occupancy_d1(lds_bytes, bpc);
    if (deg_bytes == 2) return search_occupancy_d2(lds_bytes, bpc);
    return search_occupancy_d4(lds_bytes, bpc);
}

hipError_t launch_search_init(const SearchArgs& a, int best0, uint32_t deg_bytes,
                              const uint32_t* kdeg, hipStream_t st) {
    uint32_t work = a.wl_cap > a.n_pad ? a.wl_cap : a.n_pad;
    uint32_t blocks = (work + 255u) / 256u;
    if (blocks > 1024u) blocks = 1024u;
    if (blocks == 0) blocks = 1;
    if (deg_bytes == 1) return launch_search_init_d1(a, best0, kdeg, blocks, st);
    if (deg_bytes == 2) return launch_search_init_d2(a, best0, kdeg, blocks, st);
    return launch_search_init_d4(a, best0, kdeg, blocks, st);
}

// ------------------------------------------------------------ batches

// Copy every instance graph of a batch into the arena as a 32-bit CSR with
// instance-local ids: off[n+1] then col[nnz].  One block per instance.
__global__ void batch_pack_kernel(SearchArgs a, BatchDesc d) {
    for (uint32_t i = blockIdx.x; i < d.count; i += gridDim.x) {
        const uint32_t n = d.n[i];
        const uint64_t nnz = d.nnz[i];
        const uint32_t* so = d.offsets + d.offs_base[i];
        uint32_t* dst = a.arena + d.g_at[i];
        for (uint32_t v = threadIdx.x; v <= n; v += blockDim.x) dst[v] = so[v];
        uint32_t* dc = dst + n + 1u;
        if (d.col_bytes == 2) {
            const uint16_t* sc = reinterpret_cast<const uint16_t*>(d.cols) + d.cols_base[i];
            for (uint64_t e = threadIdx.x; e < nnz; e += blockDim.x) dc[e] = sc[e];
        } else {
            const uint32_t* sc = reinterpret_cast<const uint32_t*>(d.cols) + d.cols_base[i];
            for (uint64_t e = threadIdx.x; e < nnz; e += blockDim.x) dc[e] = sc[e];
        }
    }
}

// Root entries, initial covers and state of every instance, the empty
// worklist and the control block.  An instance's first bound is |V|-1
// (V minus its last vertex is a cover); PVC starts from k+1 unless that
// trivial cover already answers it.  Edgeless instances and trivial PVC
// answers are final before the search.
__global__ void batch_init_kernel(SearchArgs a, BatchDesc d) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < a.wl_cap; i += stride) a.wl_seq[i] = (uint64_t)i;
    for (uint32_t i = tid; i < d.count; i += stride) {
        const uint32_t n = d.n[i];
        const bool edges = d.nnz[i] != 0;
        int best0, cs, state = 0;
        bool all_but_last = false;
        if (!edges) {
            best0 = 0;
            cs = 0;
            state = INST_STOP | INST_FIN;
        } else if (a.pvc && (int64_t)n - 1 <= (int64_t)a.inst_k[i]) {
            best0 = (int)n - 1;
            cs = best0;
            all_but_last = true;
            state = INST_STOP | INST_FIN;
        } else if (a.pvc) {
            best0 = a.inst_k[i] + 1;
            cs = INF;
        } else {
            best0 = (int)n - 1;
            cs = best0;
            all_but_last = true;
        }
        RegEntry r = {};
        r.best = best0;
        r.live = 1;
        r.up = -1;
        r.lock = 0;
        r.cover_size = cs;
        r.nchild = 0;
        r.size = (int)n;
        r.view = (int)i;
        r.vn = (int)n;
        r.g_at = (uint32_t)d.g_at[i];
        r.g_nnz = (int)d.nnz[i];
        a.reg[i] = r;
        a.inst_state[i] = state;
        a.inst_nodes[i] = 0;
        uint32_t* bm = a.bitmaps + (size_t)i * a.bm_words;
        for (uint32_t w = 0; w < a.bm_words; ++w) {
            uint32_t bits = 0;
            if (all_but_last) {
                const uint32_t lo = w * 32u;
                const uint32_t m = n - 1u;  // bits lo .. m-1
                if (m >= lo + 32u) bits = ~0u;
                else if (m > lo) bits = (1u << (m - lo)) - 1u;
            }
            bm[w] = bits;
        }
    }
    if (tid == 0) {
        Ctl* c = a.ctl;
        c->wl_head = 0;
        c->wl_tail = 0;
        c->outstanding = 0;
        c->idle = 0;
        c->done = 0;
        c->err = 0;
        c->err_site = 0;
        c->reg_next = (d.count + 1u) & ~1u;
        c->arena_next = d.inst_words;
        c->inst_next = 0;
        c->nodes = c->comp_branches = c->components = c->donations = c->pushes = 0;
        c->stale = c->local_views = 0;
        for (int i = 0; i < 8; ++i) c->comp_hist[i] = 0;
        for (int i = 0; i < 6; ++i) c->cyc[i] = 0;
        c->bytes_nodes = c->bytes_registry = c->bytes_rows = c->bytes_views = 0;
    }
}

// Instance i's root bitmap as ascending vertex ids at out + cbase[i] and
// their number in cnt[i].  One wave per instance.
__global__ void __launch_bounds__(64) batch_cover_kernel(SearchArgs a, BatchDesc d,
                                                         const uint64_t* cbase, uint32_t* out,
                                                         uint32_t* cnt) {
    const uint32_t l = lane();
    for (uint32_t i = blockIdx.x; i < d.count; i += gridDim.x) {
        const uint32_t n = d.n[i];
        const uint32_t words = (n + 31u) / 32u;
        const uint32_t* bm = a.bitmaps + (size_t)i * a.bm_words;
        uint32_t* o = out + cbase[i];
        uint32_t total = 0;
        for (uint32_t w0 = 0; w0 < words; w0 += 64) {
            const uint32_t w = w0 + l;
            uint32_t bits = w < words ? bm[w] : 0u;
            if (w == words - 1u && (n & 31u)) bits &= (1u << (n & 31u)) - 1u;
            const uint32_t c = (uint32_t)__builtin_popcount(bits);
            const uint32_t incl = wave_incl_scan(c);
            uint32_t at = total + incl - c;
            while (bits) {
                const uint32_t b = (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1u;
                o[at++] = w * 32u + b;
            }
            total += shfl(incl, 63);
        }
        if (l == 0) cnt[i] = total;
    }
}

hipError_t launch_batch_pack(const SearchArgs& a, const BatchDesc& d, hipStream_t st) {
    const uint32_t blocks = d.count < 4096u ? (d.count ? d.count : 1u) : 4096u;
    hipLaunchKernelGGL(batch_pack_kernel, dim3(blocks), dim3(256), 0, st, a, d);
    return hipGetLastError();
}

hipError_t launch_batch_init(const SearchArgs& a, const BatchDesc& d, hipStream_t st) {
    const uint32_t work = a.wl_cap > d.count ? a.wl_cap : d.count;
    uint32_t blocks = (work + 255u) / 256u;
    if (blocks > 1024u) blocks = 1024u;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(batch_init_kernel, dim3(blocks), dim3(256), 0, st, a, d);
    return hipGetLastError();
}

hipError_t launch_batch_cover(const SearchArgs& a, const BatchDesc& d, const uint64_t* cbase,
                              uint32_t* out, uint32_t* cnt, hipStream_t st) {
    const uint32_t blocks = d.count < 8192u ? (d.count ? d.count : 1u) : 8192u;
    hipLaunchKernelGGL(batch_cover_kernel, dim3(blocks), dim3(64), 0, st, a, d, cbase, out, cnt);
    return hipGetLastError();
}

// Serving: the empty worklist and the control block of a resident launch
// (instances are published into it later by the host).
__global__ void serve_init_kernel(SearchArgs a, uint64_t host_words) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < a.wl_cap; i += stride) a.wl_seq[i] = (uint64_t)i;
    if (tid == 0) {
        Ctl* c = a.ctl;
        c->wl_head = 0;
        c->wl_tail = 0;
        c->outstanding = 0;
        c->idle = 0;
        c->done = 0;
        c->err = 0;
        c->err_site = 0;
        c->reg_next = (a.n_roots + 1u) & ~1u;
        c->arena_next = host_words;
        c->inst_next = 0;
        c->inst_avail = 0;
        c->closed = 0;
        c->quit_epoch = 0;
        c->nodes = c->comp_branches = c->components = c->donations = c->pushes = 0;
        c->stale = c->local_views = 0;
        for (int i = 0; i < 8; ++i) c->comp_hist[i] = 0;
        for (int i = 0; i < 6; ++i) c->cyc[i] = 0;
        c->bytes_nodes = c->bytes_registry = c->bytes_rows = c->bytes_views = 0;
    }
}

hipError_t launch_serve_init(const SearchArgs& a, uint64_t host_words, hipStream_t st) {
    uint32_t blocks = (a.wl_cap + 255u) / 256u;
    if (blocks > 1024u) blocks = 1024u;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(serve_init_kernel, dim3(blocks), dim3(256), 0, st, a, host_words);
    return hipGetLastError();
}

}  // namespace vc
