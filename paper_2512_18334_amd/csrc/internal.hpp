// internal.hpp -- structures shared by the libvc host runtime and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vc {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int INF = 0x3FFFFFFF;

// Search-node slot in HBM (private stacks and the shared worklist): this
// 32-byte header, the degree array of the node's graph view (entry 0 = no
// remaining edge, all-ones = in the cover, else the live degree; Sec. IV-A),
// and at the end of the slot a 16-byte trailer whose first word repeats the
// stamp.  Slots have room for the largest view; a node moves only the part
// its view needs.
struct SlotHdr {
    int32_t s;         // |S| counted in the node's scope
    int32_t scope;     // registry entry of the scope (0 = the root)
    uint32_t branch_v; // NONE, or: first put N(branch_v) into the cover
    uint32_t nlive;    // live vertices when stored (diagnostic)
    uint32_t stamp;    // worklist position the slot was published for (0 on stacks)
    int32_t view;      // registry entry whose graph the degree array indexes
    uint32_t inst;     // instance the node belongs to (batches; 0 otherwise)
    uint32_t flags;    // SLOT_COUNTED, SLOT_INDUCE
};
static_assert(sizeof(SlotHdr) == 32, "slot header is 32 bytes");

// Component branch registry entry (Sec. III-C).  A child entry (a component,
// or the root scope at index 0) holds {Best, LiveNodes, ParentIdx}; a parent
// entry (a node that branched on components) holds {Sum, LiveComps,
// AncestorIdx}.  Entries of one branch are contiguous: parent p, then its
// children p+1 .. p+nchild.  Every entry owns one cover bitmap: a child's
// best cover found so far, a parent's vertices taken before the split, both
// in the ids of the entry's graph view.
//
// Graph views: a small component gets its own induced subgraph with local
// ids 0..size-1 (CSR plus the map back to the ids of the view it was cut
// from) in the graph arena; its entry is then its own view.  Otherwise it
// keeps the view of the scope it was found in.  The root's view is the
// subgraph induced after the root reduction.
struct RegEntry {
    int best;       // child: Best          | parent: Sum
    int live;       // child: LiveNodes     | parent: LiveComps
    int up;         // child: ParentIdx     | parent: AncestorIdx (a child/root)
    int lock;       // guards the cover bitmap
    int cover_size; // vertices in the bitmap (INF: no attained cover yet)
    int nchild;     // parent: number of children
    int size;       // child: vertices of the component
    int view;       // child/root: entry whose graph ids the scope uses
    int vn;         // child/root: vertex count of that view
    uint32_t g_at;  // own view: word offset in the arena of off[vn+1], col[nnz], l2g[vn]
    int g_nnz;      // own view: CSR entries
    int att;        // parent, PVC: Sum plus the children's attained covers
    int unatt;      // parent, PVC: children without an attained cover yet
    int done;       // times the entry was completed (VC_OPT_CHECK_REGISTRY)
    int pad[2];
};
static_assert(sizeof(RegEntry) == 64, "registry entry is 64 bytes");

// Control block (one per solve), fields on separate 128-byte lines.
struct Ctl {
    uint64_t wl_head;
    uint64_t _p0[15];
    uint64_t wl_tail;
    uint64_t _p1[15];
    int outstanding;  // queued nodes + busy workers
    int _p2[31];
    int idle;         // workers waiting for work
    int _p3[31];
    int done;         // stop flag (PVC answer found, error, limit)
    int err;          // vc_status of a device-side failure
    uint32_t reg_next;
    int err_site;     // which check raised it (FAIL_*), for diagnostics
    int _p4[28];
    uint64_t arena_next;  // words of the graph arena in use
    uint64_t _p6[15];
    uint32_t inst_next;   // batches: next instance to claim
    uint32_t _p8[31];
    uint32_t inst_avail;  // serving: instances published so far (host writes)
    int closed;           // serving: no more instances will be published
    uint32_t quit_epoch;  // serving: the launch of this epoch is ending (no new claims)
    uint32_t _p9[29];
    uint64_t nodes;   // statistics
    uint64_t comp_branches;
    uint64_t components;
    uint64_t donations;
    uint64_t pushes;
    uint64_t stale;   // worklist reads that saw an old payload and re-read
    uint64_t local_views;  // components given their own induced subgraph
    uint32_t comp_hist[8]; // branches on components by number of components
                           // registered: 2, 3-4, 5-8, 9-16, 17-32, 33-64, 65-128, more
    uint64_t _p5[5];
    // shader cycles summed over workers, by activity (the time breakdown
    // of Sec. V-D): fetching nodes, rules, component search and
    // registration, vertex branching, registry completion, waiting for work
    uint64_t cyc[6];
    uint64_t bytes_nodes;     // bytes written into node slots (each is read back once)
    uint64_t bytes_registry;  // bytes of registry entries, cover bitmaps and arena graphs written
    uint64_t bytes_rows;      // CSR bytes read from HBM for the rows of removed vertices
    uint64_t bytes_views;     // view bytes copied from HBM into the LDS graph caches
    uint64_t _p7[6];
};
// Device-side checks that stop a search (Ctl::err_site)
enum { FAIL_NONE = 0, FAIL_STALE_SLOT, FAIL_ARENA, FAIL_NODE_LIMIT, FAIL_SMALL_STACK, FAIL_WATCHDOG };
enum { CYC_FETCH = 0, CYC_REDUCE, CYC_COMPONENTS, CYC_BRANCH, CYC_COMPLETE, CYC_IDLE };

// Per-instance state bits of a batch (SearchArgs::inst_state)
enum : int {
    INST_STOP = 1,    // answered (PVC yes) or over its node limit: drop its nodes
    INST_LIMIT = 2,   // the node limit was reached
    INST_FIN = 4,     // no node of the instance is left
    INST_GREEDY = 8,  // serving: admitted without root steps; the claiming
                      // worker takes its bound from the rules and a greedy dive
};

struct SearchArgs {
    uint32_t n;           // vertices of the induced subgraph (root view)
    uint32_t nnz;         // its CSR entries
    uint32_t n_pad;       // largest degree array (multiple of 64)
    const uint32_t* off;  // CSR of the induced subgraph
    const uint32_t* col;
    uint32_t slot_bytes;
    uint32_t stack_depth;
    uint8_t* stacks;      // [workers][stack_depth][slot_bytes]
    uint8_t* wl_slots;    // [wl_cap][slot_bytes]
    uint64_t* wl_seq;     // [wl_cap]
    uint32_t wl_cap;
    uint32_t reg_cap;
    Ctl* ctl;
    RegEntry* reg;
    uint32_t* bitmaps;    // [reg_cap][bm_words]
    uint32_t bm_words;
    uint32_t* arena;      // graph arena (local views)
    uint64_t arena_words;
    uint32_t gcache_words;  // LDS graph cache capacity (words)
    uint32_t lds_L, lds_Q, lds_R, lds_VB, lds_PB, lds_MK, lds_G, lds_bytes;
    int pvc;              // 1: parameterized (stop once the root is <= k)
    int k;
    uint32_t flags;       // VC_OPT_* ablation switches
    uint32_t donate_slack;
    uint32_t donate_min;  // donate only nodes with at least this many live vertices
    uint32_t strong_fences;  // 1: agent-scope release/acquire fences as well
    uint64_t node_limit;  // 0: none
    uint64_t watchdog_ticks;  // idle wait limit in wall_clock64() ticks
    // Batches: registry entries 0 .. n_roots-1 are the instances' root
    // scopes, each with its own graph (CSR in the arena, ids local to the
    // instance).  Workers claim instances through Ctl::inst_next.  A
    // single solve has one root (entry 0) whose view is off/col above.
    uint32_t n_roots;
    uint32_t batch;           // 1: the roots are claimed instances
    int* inst_state;          // [n_roots] INST_* bits
    uint64_t* inst_nodes;     // [n_roots] tree nodes per instance
    const int* inst_k;        // [n_roots] PVC bound per instance (batch PVC)
    uint64_t inst_node_limit; // per instance, 0: none
    // Serving: instances 0 .. Ctl::inst_avail-1 are published while the
    // kernel runs (n_roots is the slot capacity); the kernel ends once
    // Ctl::closed is set and no work is left.  inst_cancel[i] != 0 stops
    // instance i like a PVC answer does.
    uint32_t serve;
    const int* inst_cancel;
    uint64_t linger_ticks;  // serving: an empty launch ends after this long
    uint32_t launch_epoch;  // serving: number of this launch of the resident search
    uint32_t small_max;  // live vertices up to which a node is solved in registers (0: never)
    // Lists in HBM (nodes whose lists do not fit LDS): the live list and the
    // scratch lists L, Q, R of worker w are at hl_base + w * hl_stride (the
    // lds_L, lds_Q, lds_R offsets are then offsets in that region); the
    // degree array, bitmaps, row markers and graph cache stay in LDS.
    uint32_t hl;
    uint8_t* hl_base;
    uint64_t hl_stride;
};

// LDS layout of one worker: degree array, live list L, scratch lists Q and
// R (R doubles as an id map of n_pad words), two bitmaps, 64 words of row
// markers for the row expansion and the small-node solver's masks and stack,
// graph cache.
struct LdsPlan {
    uint32_t L, Q, R, VB, PB, MK, G, bytes;
};
inline LdsPlan lds_plan(uint32_t n_pad, uint32_t sd, uint32_t gcache_words) {
    LdsPlan p;
    uint32_t at = n_pad * sd;
    at = (at + 15u) & ~15u;
    p.L = at; at += 4u * n_pad;
    p.Q = at; at += 4u * n_pad;
    p.R = at; at += 4u * (2u * n_pad + 64u);
    uint32_t bw = (n_pad + 31u) / 32u;
    p.VB = at; at += 4u * bw;
    p.PB = at; at += 4u * bw;
    at = (at + 15u) & ~15u;
    // row markers (64 words), then the small-node solver's adjacency masks
    // and stack: 128 x 2 u64 adjacency, 128 x (2 u64 live, 2 u64 taken),
    // 128 u32 counts
    p.MK = at; at += 4u * 64u + 8u * 128u * 2u + 8u * 128u * 4u + 4u * 128u;
    p.G = at; at += 4u * gcache_words;
    p.bytes = (at + 15u) & ~15u;
    return p;
}

// The same layout with the lists L, Q and R moved to a per-worker region of
// HBM (hl_bytes long, offsets L, Q, R in it): LDS then holds the degree
// array, the bitmaps, the row markers with the small-node solver's masks,
// and the graph cache, about sizeof(D) + 1/4 bytes per vertex instead of
// about sizeof(D) + 16.
inline LdsPlan lds_plan_hl(uint32_t n_pad, uint32_t sd, uint32_t gcache_words,
                           uint64_t* hl_bytes) {
    LdsPlan p;
    uint32_t at = n_pad * sd;
    at = (at + 15u) & ~15u;
    const uint32_t bw = (n_pad + 31u) / 32u;
    p.VB = at; at += 4u * bw;
    p.PB = at; at += 4u * bw;
    at = (at + 15u) & ~15u;
    p.MK = at; at += 4u * 64u + 8u * 128u * 2u + 8u * 128u * 4u + 4u * 128u;
    p.G = at; at += 4u * gcache_words;
    p.bytes = (at + 15u) & ~15u;
    p.L = 0;
    p.Q = 4u * n_pad;
    p.R = 8u * n_pad;
    *hl_bytes = ((uint64_t)4u * (4u * n_pad + 64u) + 255u) & ~255ull;
    return p;
}

// ------------------------------------------------------ kernel launchers
// (defined in the .hip files; all launch on `st`)

hipError_t launch_search(const SearchArgs& a, uint32_t deg_bytes, uint32_t workers,
                         hipStream_t st);
hipError_t search_occupancy(uint32_t deg_bytes, uint32_t lds_bytes, int* blocks_per_cu,
                            bool hl = false);
hipError_t launch_search_init(const SearchArgs& a, int best0, uint32_t deg_bytes,
                              const uint32_t* kdeg, hipStream_t st);

// Batch set-up: instance graphs copied into the arena, root entries,
// initial covers, per-instance state and the control block.
struct BatchDesc {
    uint32_t count;
    const uint32_t* n;          // [count]
    const uint64_t* nnz;        // [count]
    const uint64_t* offs_base;  // [count]
    const uint64_t* cols_base;  // [count]
    const uint64_t* g_at;       // [count] arena word offset of each instance graph
    const uint32_t* offsets;    // packed input
    const void* cols;
    uint32_t col_bytes;
    uint64_t inst_words;        // arena words taken by the instance graphs
};
hipError_t launch_batch_pack(const SearchArgs& a, const BatchDesc& d, hipStream_t st);
// serving: the control block and worklist of a resident launch; the graph
// arena's first host_words words hold the instances' graphs
hipError_t launch_serve_init(const SearchArgs& a, uint64_t host_words, hipStream_t st);
hipError_t launch_batch_init(const SearchArgs& a, const BatchDesc& d, hipStream_t st);
// cover lists: instance i's root bitmap as ascending ids at out + cbase[i],
// the count in cnt[i]
hipError_t launch_batch_cover(const SearchArgs& a, const BatchDesc& d, const uint64_t* cbase,
                              uint32_t* out, uint32_t* cnt, hipStream_t st);

}  // namespace vc
